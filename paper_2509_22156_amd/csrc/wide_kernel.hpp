// The wide streaming solver: the implicit steps of a few large systems
// (streaming grids, vectors in HBM) spread over many work-groups each, for
// launches whose task count would leave most of the chip idle under the
// one-work-group-per-task streaming kernel (the sequential coarse chain of
// MGRIT, one task per grid; time-sequential stepping). Every Krylov phase
// is one launch over all work-groups of all tasks of the range (grid
// dimension y = task), and the kernel boundaries are the only grid-wide
// synchronisation: nothing ever waits on another work-group.
//
// The arithmetic is the streaming kernel's: FP64, the same (2d+1)-point
// operator evaluated per point, the same exact line-block preconditioner
// (chunks of kSK unknowns per lane, factors in the task's scratch), CG or
// right-preconditioned BiCGStab (Section 4.1) with the same stopping tests.
// BiCGStab's next rho = (r^, r) is formed as (r^, s) - omega (r^, t) from
// the sums of the t-phase (r = s - omega t), so that the x/r update, the
// direction update and the next preconditioner application share one
// launch; the convergence test uses the directly summed (r, r).
//
// Sums: every work-group writes its partial sums, and the last work-group
// of the task to arrive (an atomic counter) adds them in block order, so
// the result does not depend on the arrival order. A kernel reads only sums
// that earlier launches completed; the per-task `done` flag is read once
// per work-group (LDS broadcast), and every work-group of a task derives
// the same decision from the same sums.
#pragma once

#include "stream_kernel.hpp"

namespace ctm {

static_assert(kWideSK == kSK, "the wide solver reads the streaming kernel's line factors");

__device__ __forceinline__ int wide_point_blocks(const GridDev& g) {
  return (g.npts + kWP - 1) / kWP;
}
__device__ __forceinline__ int wide_line_blocks(const GridDev& g) {
  const int Lc = pow2ceil((g.ns + kSK - 1) / kSK);
  const int waves = (g.nlines + (64 / Lc) - 1) / (64 / Lc);
  return (waves + kWW - 1) / kWW;
}

// Shared preamble: the launch-level skip, the task's grid (LDS) and its
// coefficient tables, the block range of the grid, and the done flag.
// Returns false (uniformly over the work-group) when the block has nothing
// to do.
struct WideSmem {
  GridDev g;
  double red[2 * 64];
  int flag;  // done broadcast / last-arrival broadcast
};

template <int OPC>
__device__ __forceinline__ bool wide_begin(const WideArgs& w, WideSmem& sm, double* tl,
                                           bool line, bool check_done) {
  const ChainArgs& a = w.a;
  if (a.skip && *a.skip != 0.0) return false;
  const int2 task = a.tasks[blockIdx.y];
  {
    const int* src = reinterpret_cast<const int*>(a.grids + task.x);
    int* dst = reinterpret_cast<int*>(&sm.g);
    for (int t = threadIdx.x; t < (int)(sizeof(GridDev) / sizeof(int)); t += kWT) dst[t] = src[t];
  }
  if (threadIdx.x == 0) sm.flag = check_done ? w.st[blockIdx.y].done : 0;
  __syncthreads();
  const int nb = line ? wide_line_blocks(sm.g) : wide_point_blocks(sm.g);
  if ((int)blockIdx.x >= nb || sm.flag) return false;
  load_tables<OPC, double, kWT>(sm.g, a.tab64, a.dt, tl);
  __syncthreads();
  return true;
}

__device__ __forceinline__ double* wide_sv(const WideArgs& w) {
  return w.scratch + (long long)blockIdx.y * SV_N * w.ss;
}

// Sum NS values over the work-groups of the task into sum[slot0 ..]: every
// work-group stores its partials; the last to arrive adds them in block
// order and resets the counter. nblk = the task's participating blocks.
template <int NS>
__device__ __forceinline__ void wide_reduce(const WideArgs& w, WideSmem& sm, int nblk, int kind,
                                            int slot0, double (&v)[NS]) {
  RedRing ring{sm.red, 0};
  block_sum<kWW, NS, double>(v, ring);
  WideTask* T = w.st + blockIdx.y;
  double* part = w.part + (size_t)blockIdx.y * WS_N * w.maxblk;
  if (threadIdx.x == 0) {
#pragma unroll
    for (int s = 0; s < NS; ++s) part[(size_t)(slot0 + s) * w.maxblk + blockIdx.x] = v[s];
    __threadfence();
    const unsigned prev = atomicAdd(&T->cnt[kind], 1u);
    sm.flag = (prev == (unsigned)(nblk - 1));
  }
  __syncthreads();
  if (!sm.flag) return;
  __threadfence();
  double acc[NS];
#pragma unroll
  for (int s = 0; s < NS; ++s) {
    acc[s] = 0.0;
    for (int b = threadIdx.x; b < nblk; b += kWT)
      acc[s] += __hip_atomic_load(part + (size_t)(slot0 + s) * w.maxblk + b, __ATOMIC_RELAXED,
                                  __HIP_MEMORY_SCOPE_AGENT);
  }
  block_sum<kWW, NS, double>(acc, ring);
  if (threadIdx.x == 0) {
#pragma unroll
    for (int s = 0; s < NS; ++s) T->sum[slot0 + s] = acc[s];
    atomicExch(&T->cnt[kind], 0u);
  }
}

// Stops the task's step (thread 0 of any deciding work-group; idempotent).
__device__ __forceinline__ void wide_stop(WideTask* T, int it, int flag) {
  if (threadIdx.x != 0) return;
  if (flag) atomicOr(&T->flag, flag);
  T->it = it;
  __threadfence();
  T->done = 1;
}

__device__ __forceinline__ bool isnan_(double x) { return !(x == x); }

// ------------------------------------------------------- stopping tests
// The start of a step (iteration 1): the initial residual.
__device__ __forceinline__ bool wide_test_init(const WideTask* T, double tol2, int& it, int& fl) {
  const double rr0 = T->sum[WS_RR0], bb = T->sum[WS_BB];
  it = 0;
  fl = 0;
  if (isnan_(rr0) || isnan_(bb)) {
    fl = FLAG_NONFINITE;
    return true;
  }
  return rr0 <= tol2 * bb;
}
// After the r update of iteration it (CG: (r, r); BiCGStab: also a
// breakdown found in the direction update).
__device__ __forceinline__ bool wide_test_rr(const WideTask* T, double tol2, int itd, int& it,
                                             int& fl) {
  const double rr = T->sum[WS_RR], bb = T->sum[WS_BB];
  it = itd;
  fl = 0;
  if (isnan_(rr)) {
    fl = FLAG_NONFINITE;
    return true;
  }
  if (rr <= tol2 * bb) return true;
  if (T->pend) {
    fl = FLAG_BREAKDOWN;
    return true;
  }
  return false;
}
// The test the next kernel of iteration i would make first (BiCGStab: the
// start of K_B(i); CG: the start of the preconditioner phase of i).
__device__ __forceinline__ bool wide_test_next(const WideTask* T, double tol2, int i, int& it,
                                               int& fl) {
  return (i == 1) ? wide_test_init(T, tol2, it, fl) : wide_test_rr(T, tol2, i - 1, it, fl);
}

// BiCGStab scalars from the t-phase sums of iteration k (k >= 1).
__device__ __forceinline__ const double* wide_dsums(const WideTask* T, int k) {
  return T->sum + WS_D + 5 * (k & 1);
}
// rho_k = (r^, r_{k-1}): rho_1 = (r0, r0); rho_k = rhs - omega rht of k-1.
__device__ __forceinline__ double wide_rho(const WideTask* T, int k) {
  if (k == 1) return T->sum[WS_RR0];
  const double* D = wide_dsums(T, k - 1);
  return D[3] - (D[0] / D[1]) * D[4];
}

// ------------------------------------------------------- point-wise helpers
template <int OPC, int D, class F>
__device__ __forceinline__ double wide_Ax(const GridDev& g, const double* tl, double dt,
                                          double amp, int p, F x) {
  PointCoef<OPC, D> c;
  point_coef<OPC, D>(g, tl, dt, amp, p, c);
  double v = c.diag * x(p);
#pragma unroll
  for (int i = 0; i < D; ++i) {
    if (i >= g.d) continue;
    const int st = g.stride[i];
    if (c.lo[i] != 0.0) v += c.lo[i] * x(p - st);
    if (c.up[i] != 0.0) v += c.up[i] * x(p + st);
  }
  return v;
}

// ------------------------------------------------------- line helpers
// Lane of this thread in the line layout (block b, wave w: virtual wave
// b * kWW + w of the task).
template <int D>
__device__ __forceinline__ void wide_lane(const GridDev& g, SLane& L) {
  stream_lane_at<D>(g, (int)blockIdx.x * kWW + (threadIdx.x >> 6), threadIdx.x & 63, L);
}
__device__ __forceinline__ long long lane_pt(const SLane& L, int k) {
  return L.base + (long long)(L.j0 + k) * L.step;
}

// z = M^-1 r on the chunk of lane L, everything in registers (r and z hold
// the chunk's kSK unknowns; entries past nval are ignored / returned 0).
__device__ __forceinline__ void wide_pre(const double* sv, long long ss, const SLane& L,
                                         const double (&r)[kSK], double (&z)[kSK]) {
  const double* FM = sv + SV_FM * ss;
  const double* FID = sv + SV_FID * ss;
  const double* FCU = sv + SV_FCU * ss;
  const double* FPHI = sv + SV_FPHI * ss;
  const double* FPSI = sv + SV_FPSI * ss;
  const bool full = (L.nval == kSK);
  const int ne = L.nval < kSK - 1 ? L.nval : kSK - 1;
  double fm[kSK], fid[kSK], fcu[kSK], fph[kSK], fps[kSK];
#pragma unroll
  for (int k = 0; k < kSK; ++k) {
    const bool v = k < L.nval;
    const long long p = lane_pt(L, k);
    fm[k] = v ? FM[p] : 0.0;
    fid[k] = v ? FID[p] : 0.0;
    fcu[k] = v ? FCU[p] : 0.0;
    fph[k] = v ? FPHI[p] : 0.0;
    fps[k] = v ? FPSI[p] : 0.0;
  }
  // forward elimination over the eliminated unknowns 0..ne-1
  double y[kSK];
#pragma unroll
  for (int k = 0; k < kSK - 1; ++k) y[k] = (k == 0) ? r[0] : r[k] - fm[k] * y[k - 1];
  y[kSK - 1] = 0.0;
  // back-substitution from ne-1
  double yn = 0.0;
#pragma unroll
  for (int k = kSK - 2; k >= 0; --k) {
    if (k < ne) {
      yn = (k == kSK - 2) ? y[k] * fid[k] : (y[k] - fcu[k] * yn) * fid[k];
      y[k] = yn;
    }
  }
  const double y0 = (ne > 0) ? y[0] : 0.0;
  const double y2 = (ne == kSK - 1) ? y[kSK - 2] : 0.0;
  const double phi0 = (L.nval > 0) ? fph[0] : 0.0, psi0 = (L.nval > 0) ? fps[0] : 0.0;
  const double phi2 = (L.nval > kSK - 2) ? fph[kSK - 2] : 0.0;
  const double psi2 = (L.nval > kSK - 2) ? fps[kSK - 2] : 0.0;
  const double aL = full ? fph[kSK - 1] : 0.0, cL = full ? fps[kSK - 1] : 0.0;
  const double bL = full ? fm[kSK - 1] : 1.0;
  const double rL = full ? r[kSK - 1] : 0.0;
  const double phi0n = from_plus(phi0, 1, L.Lc), psi0n = from_plus(psi0, 1, L.Lc);
  const double y0n = from_plus(y0, 1, L.Lc);
  double A = -aL * phi2;
  double B = bL - aL * psi2 - cL * phi0n;
  double C = -cL * psi0n;
  double R = rL - aL * y2 - cL * y0n;
#pragma unroll
  for (int sp = 0; sp < kMaxPcr; ++sp) {
    const int sh = 1 << sp;
    if (sh < L.Lc) {
      const double Am = from_minus(A, sh, L.Lc), Bm = from_minus(B, sh, L.Lc),
                   Cm = from_minus(C, sh, L.Lc), Rm = from_minus(R, sh, L.Lc);
      const double Ap = from_plus(A, sh, L.Lc), Bp = from_plus(B, sh, L.Lc),
                   Cp = from_plus(C, sh, L.Lc), Rp = from_plus(R, sh, L.Lc);
      const bool vm = L.c >= sh, vp = L.c + sh < L.Lc;
      const double al = vm ? -A / Bm : 0.0;
      const double ga = vp ? -C / Bp : 0.0;
      B = B + (vm ? al * Cm : 0.0) + (vp ? ga * Ap : 0.0);
      R = R + (vm ? al * Rm : 0.0) + (vp ? ga * Rp : 0.0);
      A = vm ? al * Am : 0.0;
      C = vp ? ga * Cp : 0.0;
    }
  }
  const double u = R / B;
  double um = from_minus(u, 1, L.Lc);
  um = (L.c > 0) ? um : 0.0;
#pragma unroll
  for (int k = 0; k < kSK - 1; ++k) z[k] = (k < ne) ? y[k] - fph[k] * um - fps[k] * u : 0.0;
  z[kSK - 1] = full ? u : 0.0;
}

// ------------------------------------------------------------- kernels
#define WIDE_KERNEL(name) \
  template <int OPC, int D> \
  __global__ void __launch_bounds__(kWT) name(WideArgs w)
#define WIDE_SMEM                                        \
  extern __shared__ __align__(16) unsigned char smem[]; \
  __shared__ WideSmem sm;                               \
  double* tl = reinterpret_cast<double*>(smem)

// Factors of the line preconditioner (once per chain).
WIDE_KERNEL(wide_setup_kernel) {
  WIDE_SMEM;
  if (!wide_begin<OPC>(w, sm, tl, true, false)) return;
  double* sv = wide_sv(w);
  SLane L;
  wide_lane<D>(sm.g, L);
  linepre_setup_lane<OPC, D>(sm.g, tl, w.a.dt, w.a.amp, sv, w.ss, sv + SV_S * w.ss, L);
}

// Step transition (point-wise; step j): finish step j-1 (B = x + forcing,
// intermediate store) or load the start vector (j = 1); the residual-mode
// forcing; then either the exact residual b - A target (residual mode, last
// step) or the initial guess. Work-group 0 accounts step j-1 and resets the
// task's step state.
WIDE_KERNEL(wide_step_kernel) {
  WIDE_SMEM;
  if (!wide_begin<OPC>(w, sm, tl, false, false)) return;
  const ChainArgs& a = w.a;
  const GridDev& g = sm.g;
  const int q = a.tasks[blockIdx.y].y;
  const int j = w.j;
  const bool last = (j == a.nsteps), res = a.resmode != 0;
  WideTask* T = w.st + blockIdx.y;
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    if (j == 1) {
      T->kr_sum = T->kr_max = 0;
      T->res_max = 0.0;
      T->flag = 0;
    } else {
      const int it = T->done ? T->it : w.prev_its;
      int fl = T->flag | ((T->done || res) ? 0 : FLAG_NOCONV);
      if (res) {
        fl &= ~(FLAG_NOCONV | FLAG_BREAKDOWN);
        T->res_max = fmax(T->res_max, T->sum[WS_RR0]);
      }
      T->flag = fl;
      T->kr_sum += it;
      T->kr_max = it > T->kr_max ? it : T->kr_max;
    }
    T->done = T->it = T->pend = 0;
    for (int k = 0; k < WR_N; ++k) T->cnt[k] = 0;
  }
  double* sv = wide_sv(w);
  double* X = sv + SV_X * w.ss;
  double* B = sv + SV_B * w.ss;
  const long long off = g.off;
  auto at = [&](const VecRef& r, long long idx) { return r.base + idx * a.slen + off; };
  const double* st = (j == 1 && a.start.base) ? at(a.start, a.start.a * q + a.start.b) : nullptr;
  double* wb = (j == 1 && a.start_wb.base) ? at(a.start_wb, a.start_wb.a * q + a.start_wb.b)
                                           : nullptr;
  const double* fp = (j > 1 && a.forcing.base && !res)
                         ? at(a.forcing, a.forcing.a * q + a.forcing.b + (j - 1)) : nullptr;
  double* is = (j > 1 && a.inter.base) ? at(a.inter, a.inter.a * q + a.inter.b + (j - 1))
                                       : nullptr;
  const double* fj = (res && a.forcing.base) ? at(a.forcing, a.forcing.a * q + a.forcing.b + j)
                                             : nullptr;
  const bool rho = res && last && a.target.base;
  const double* tg = rho ? at(a.target, a.target.a * q + a.target.b) : nullptr;
  const VecRef gr = last ? a.guess_fin : a.guess;
  const double* gx = (!rho && gr.base) ? at(gr, gr.a * q + gr.b + (last ? 0 : j)) : nullptr;
#pragma unroll
  for (int k = 0; k < kWPT; ++k) {
    const int p = blockIdx.x * kWP + k * kWT + threadIdx.x;
    if (p >= g.npts) continue;
    double b;
    if (j == 1) {
      b = st ? st[p] : 0.0;
      if (wb) wb[p] = b;
    } else {
      b = X[p] + (fp ? fp[p] : 0.0);
      if (is) is[p] = b;
    }
    if (fj) b += fj[p];
    if (rho) {
      b -= wide_Ax<OPC, D>(g, tl, a.dt, a.amp, p, [&](int i) { return tg[i]; });
    } else {
      X[p] = gx ? gx[p] : b;
    }
    B[p] = b;
  }
}

// Initial residual of the step (stencil): r = b - A x; BiCGStab also sets
// r^ = p = r. Sums (r, r), (b, b).
template <int OPC, int SOLVER, int D>
__global__ void __launch_bounds__(kWT) wide_init_kernel(WideArgs w) {
  WIDE_SMEM;
  if (!wide_begin<OPC>(w, sm, tl, false, false)) return;
  const ChainArgs& a = w.a;
  const GridDev& g = sm.g;
  double* sv = wide_sv(w);
  const long long ss = w.ss;
  const double* X = sv + SV_X * ss;
  const double* B = sv + SV_B * ss;
  double* R = sv + SV_R * ss;
  double* RH = sv + SV_RH * ss;
  double* P = sv + SV_P * ss;
  double v[2] = {0.0, 0.0};
#pragma unroll
  for (int k = 0; k < kWPT; ++k) {
    const int p = blockIdx.x * kWP + k * kWT + threadIdx.x;
    if (p >= g.npts) continue;
    const double r = B[p] - wide_Ax<OPC, D>(g, tl, a.dt, a.amp, p, [&](int i) { return X[i]; });
    R[p] = r;
    if constexpr (SOLVER == SOLV_BICG) {
      RH[p] = r;
      P[p] = r;
    }
    v[0] += r * r;
    v[1] += B[p] * B[p];
  }
  wide_reduce<2>(w, sm, wide_point_blocks(g), WR_INIT, WS_RR0, v);
}

// ---- BiCGStab, iteration i: K_A(i) [lines], K_B(i), K_C(i) [lines], K_D(i)
// K_A(i): i = 1: h = M^-1 p. i > 1: the end of iteration i-1 (omega: x +=
// omega h, r = s - omega t, sum (r, r)), the direction p = r + beta (p -
// omega v), h = M^-1 p.
WIDE_KERNEL(wide_bicg_a_kernel) {
  WIDE_SMEM;
  if (!wide_begin<OPC>(w, sm, tl, true, true)) return;
  const ChainArgs& a = w.a;
  const GridDev& g = sm.g;
  WideTask* T = w.st + blockIdx.y;
  const double tol2 = a.tol * a.tol;
  const int i = w.i;
  int it, fl;
  double omega = 0.0, beta = 0.0;
  bool pend = false;
  if (i == 1) {
    if (wide_test_init(T, tol2, it, fl)) {
      wide_stop(T, it, fl);
      return;
    }
  } else {
    const double* Dn = wide_dsums(T, i - 1);
    const double ss_ = Dn[2], tt = Dn[1], bb = T->sum[WS_BB];
    if (ss_ <= tol2 * bb) {
      wide_stop(T, i - 1, 0);  // x already holds x + alpha h
      return;
    }
    if (!(tt != 0.0) || isnan_(tt)) {
      wide_stop(T, i - 1, isnan_(tt) ? FLAG_NONFINITE : FLAG_BREAKDOWN);
      return;
    }
    omega = Dn[0] / tt;
    const double rho_o = wide_rho(T, i - 1), rho_n = wide_rho(T, i);
    const double alpha = rho_o / T->sum[WS_RHV];
    if (rho_n == 0.0 || omega == 0.0) {
      pend = true;
    } else {
      beta = (rho_n / rho_o) * (alpha / omega);
    }
  }
  double* sv = wide_sv(w);
  const long long ss = w.ss;
  double* X = sv + SV_X * ss;
  double* R = sv + SV_R * ss;
  double* P = sv + SV_P * ss;
  const double* V = sv + SV_Q * ss;
  const double* S = sv + SV_S * ss;
  const double* Tv = sv + SV_T * ss;
  double* H = sv + SV_D * ss;
  SLane L;
  wide_lane<D>(g, L);
  double pr[kSK], hz[kSK];
  double rr[1] = {0.0};
#pragma unroll
  for (int k = 0; k < kSK; ++k) {
    pr[k] = 0.0;
    if (k >= L.nval) continue;
    const long long p = lane_pt(L, k);
    if (i == 1) {
      pr[k] = P[p];
    } else {
      X[p] += omega * H[p];
      const double r = S[p] - omega * Tv[p];
      R[p] = r;
      rr[0] += r * r;
      const double pn = r + beta * (P[p] - omega * V[p]);
      P[p] = pn;
      pr[k] = pn;
    }
  }
  wide_pre(sv, ss, L, pr, hz);
#pragma unroll
  for (int k = 0; k < kSK; ++k)
    if (k < L.nval) H[lane_pt(L, k)] = hz[k];
  if (i > 1) {
    if (pend && blockIdx.x == 0 && threadIdx.x == 0) T->pend = 1;
    wide_reduce<1>(w, sm, wide_line_blocks(g), WR_RR, WS_RR, rr);
  }
}

// K_B(i): the test of the r update (i > 1); v = A h, sum (r^, v).
WIDE_KERNEL(wide_bicg_b_kernel) {
  WIDE_SMEM;
  if (!wide_begin<OPC>(w, sm, tl, false, true)) return;
  const ChainArgs& a = w.a;
  const GridDev& g = sm.g;
  WideTask* T = w.st + blockIdx.y;
  int it, fl;
  if (w.i > 1 && wide_test_rr(T, a.tol * a.tol, w.i - 1, it, fl)) {
    wide_stop(T, it, fl);
    return;
  }
  double* sv = wide_sv(w);
  const long long ss = w.ss;
  const double* H = sv + SV_D * ss;
  const double* RH = sv + SV_RH * ss;
  double* V = sv + SV_Q * ss;
  double v[1] = {0.0};
#pragma unroll
  for (int k = 0; k < kWPT; ++k) {
    const int p = blockIdx.x * kWP + k * kWT + threadIdx.x;
    if (p >= g.npts) continue;
    const double y = wide_Ax<OPC, D>(g, tl, a.dt, a.amp, p, [&](int m) { return H[m]; });
    V[p] = y;
    v[0] += RH[p] * y;
  }
  wide_reduce<1>(w, sm, wide_point_blocks(g), WR_RHV, WS_RHV, v);
}

// K_C(i): alpha = rho / (r^, v); x += alpha h, s = r - alpha v, h = M^-1 s.
WIDE_KERNEL(wide_bicg_c_kernel) {
  WIDE_SMEM;
  if (!wide_begin<OPC>(w, sm, tl, true, true)) return;
  const GridDev& g = sm.g;
  WideTask* T = w.st + blockIdx.y;
  const double rhv = T->sum[WS_RHV];
  if (!(rhv != 0.0) || isnan_(rhv)) {
    wide_stop(T, w.i, isnan_(rhv) ? FLAG_NONFINITE : FLAG_BREAKDOWN);
    return;
  }
  const double alpha = wide_rho(T, w.i) / rhv;
  double* sv = wide_sv(w);
  const long long ss = w.ss;
  double* X = sv + SV_X * ss;
  const double* R = sv + SV_R * ss;
  const double* V = sv + SV_Q * ss;
  double* S = sv + SV_S * ss;
  double* H = sv + SV_D * ss;
  SLane L;
  wide_lane<D>(g, L);
  double sr[kSK], hz[kSK];
#pragma unroll
  for (int k = 0; k < kSK; ++k) {
    sr[k] = 0.0;
    if (k >= L.nval) continue;
    const long long p = lane_pt(L, k);
    X[p] += alpha * H[p];
    const double s = R[p] - alpha * V[p];
    S[p] = s;
    sr[k] = s;
  }
  wide_pre(sv, ss, L, sr, hz);
#pragma unroll
  for (int k = 0; k < kSK; ++k)
    if (k < L.nval) H[lane_pt(L, k)] = hz[k];
}

// K_D(i): t = A h; sums (t, s), (t, t), (s, s), (r^, s), (r^, t).
WIDE_KERNEL(wide_bicg_d_kernel) {
  WIDE_SMEM;
  if (!wide_begin<OPC>(w, sm, tl, false, true)) return;
  const ChainArgs& a = w.a;
  const GridDev& g = sm.g;
  double* sv = wide_sv(w);
  const long long ss = w.ss;
  const double* H = sv + SV_D * ss;
  const double* S = sv + SV_S * ss;
  const double* RH = sv + SV_RH * ss;
  double* Tv = sv + SV_T * ss;
  double v[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int k = 0; k < kWPT; ++k) {
    const int p = blockIdx.x * kWP + k * kWT + threadIdx.x;
    if (p >= g.npts) continue;
    const double t = wide_Ax<OPC, D>(g, tl, a.dt, a.amp, p, [&](int m) { return H[m]; });
    Tv[p] = t;
    const double s = S[p], rh = RH[p];
    v[0] += t * s;
    v[1] += t * t;
    v[2] += s * s;
    v[3] += rh * s;
    v[4] += rh * t;
  }
  wide_reduce<5>(w, sm, wide_point_blocks(g), WR_D, WS_D + 5 * (w.i & 1), v);
}

// ---- CG, iteration i: K_CA(i) [lines], K_CB(i), K_CC(i)
// K_CA(i): the test of the previous r update; z = M^-1 r, sum (r, z).
WIDE_KERNEL(wide_cg_a_kernel) {
  WIDE_SMEM;
  if (!wide_begin<OPC>(w, sm, tl, true, true)) return;
  const GridDev& g = sm.g;
  WideTask* T = w.st + blockIdx.y;
  int it, fl;
  if (wide_test_next(T, w.a.tol * w.a.tol, w.i, it, fl)) {
    wide_stop(T, it, fl);
    return;
  }
  double* sv = wide_sv(w);
  const long long ss = w.ss;
  const double* R = sv + SV_R * ss;
  double* Z = sv + SV_S * ss;
  SLane L;
  wide_lane<D>(g, L);
  double rv[kSK], zv[kSK];
#pragma unroll
  for (int k = 0; k < kSK; ++k) rv[k] = (k < L.nval) ? R[lane_pt(L, k)] : 0.0;
  wide_pre(sv, ss, L, rv, zv);
  double v[1] = {0.0};
#pragma unroll
  for (int k = 0; k < kSK; ++k)
    if (k < L.nval) {
      Z[lane_pt(L, k)] = zv[k];
      v[0] += rv[k] * zv[k];
    }
  wide_reduce<1>(w, sm, wide_line_blocks(g), WR_RZ, WS_RZ + (w.i & 1), v);
}

// K_CB(i): p_i = z + beta p_{i-1} (the two directions alternate between
// two vectors, so that neighbours read the old one while it is replaced),
// q = A p_i, sum (p, q).
WIDE_KERNEL(wide_cg_b_kernel) {
  WIDE_SMEM;
  if (!wide_begin<OPC>(w, sm, tl, false, true)) return;
  const ChainArgs& a = w.a;
  const GridDev& g = sm.g;
  const WideTask* T = w.st + blockIdx.y;
  const int i = w.i;
  const double beta = (i == 1) ? 0.0 : T->sum[WS_RZ + (i & 1)] / T->sum[WS_RZ + ((i - 1) & 1)];
  double* sv = wide_sv(w);
  const long long ss = w.ss;
  const double* Z = sv + SV_S * ss;
  const double* Po = sv + ((i & 1) ? SV_RH : SV_P) * ss;
  double* Pn = sv + ((i & 1) ? SV_P : SV_RH) * ss;
  double* Q = sv + SV_Q * ss;
  double v[1] = {0.0};
#pragma unroll
  for (int k = 0; k < kWPT; ++k) {
    const int p = blockIdx.x * kWP + k * kWT + threadIdx.x;
    if (p >= g.npts) continue;
    auto pv = [&](int m) { return (i == 1) ? Z[m] : Z[m] + beta * Po[m]; };
    const double y = wide_Ax<OPC, D>(g, tl, a.dt, a.amp, p, pv);
    const double pp = pv(p);
    Pn[p] = pp;
    Q[p] = y;
    v[0] += pp * y;
  }
  wide_reduce<1>(w, sm, wide_point_blocks(g), WR_PQ, WS_PQ, v);
}

// K_CC(i): alpha = (r, z) / (p, q); x += alpha p, r -= alpha q, sum (r, r).
WIDE_KERNEL(wide_cg_c_kernel) {
  WIDE_SMEM;
  if (!wide_begin<OPC>(w, sm, tl, false, true)) return;
  const GridDev& g = sm.g;
  WideTask* T = w.st + blockIdx.y;
  const int i = w.i;
  const double pq = T->sum[WS_PQ];
  if (!(pq != 0.0) || isnan_(pq)) {
    wide_stop(T, i, isnan_(pq) ? FLAG_NONFINITE : FLAG_BREAKDOWN);
    return;
  }
  const double alpha = T->sum[WS_RZ + (i & 1)] / pq;
  double* sv = wide_sv(w);
  const long long ss = w.ss;
  double* X = sv + SV_X * ss;
  double* R = sv + SV_R * ss;
  const double* Pn = sv + ((i & 1) ? SV_P : SV_RH) * ss;
  const double* Q = sv + SV_Q * ss;
  double v[1] = {0.0};
#pragma unroll
  for (int k = 0; k < kWPT; ++k) {
    const int p = blockIdx.x * kWP + k * kWT + threadIdx.x;
    if (p >= g.npts) continue;
    X[p] += alpha * Pn[p];
    const double r = R[p] - alpha * Q[p];
    R[p] = r;
    v[0] += r * r;
  }
  wide_reduce<1>(w, sm, wide_point_blocks(g), WR_RR, WS_RR, v);
}

// The end of the chain (point-wise): the last step's x + forcing (or the
// exact residual formed by the step kernel), fin = v - target, sum
// ||fin||^2; the last work-group to arrive accounts the last step and
// publishes res2, the counters and the status bits.
WIDE_KERNEL(wide_fin_kernel) {
  WIDE_SMEM;
  if (!wide_begin<OPC>(w, sm, tl, false, false)) return;
  const ChainArgs& a = w.a;
  const GridDev& g = sm.g;
  const int q = a.tasks[blockIdx.y].y;
  const bool res = a.resmode != 0;
  const bool rho = res && a.target.base;  // the step kernel formed the residual
  double* sv = wide_sv(w);
  const double* X = sv + SV_X * w.ss;
  const double* B = sv + SV_B * w.ss;
  const long long off = g.off;
  auto at = [&](const VecRef& r, long long idx) { return r.base + idx * a.slen + off; };
  const double* fl = (!rho && !res && a.forcing.base)
                         ? at(a.forcing, a.forcing.a * q + a.forcing.b + a.nsteps) : nullptr;
  double* dst = a.fin.base ? at(a.fin, a.fin.a * q + a.fin.b) : nullptr;
  const double* tg = (!rho && a.target.base) ? at(a.target, a.target.a * q + a.target.b)
                                              : nullptr;
  double v[1] = {0.0};
#pragma unroll
  for (int k = 0; k < kWPT; ++k) {
    const int p = blockIdx.x * kWP + k * kWT + threadIdx.x;
    if (p >= g.npts || !dst) continue;
    double u = rho ? B[p] : X[p] + (fl ? fl[p] : 0.0);
    if (tg) u -= tg[p];
    dst[p] = u;
    v[0] += u * u;
  }
  wide_reduce<1>(w, sm, wide_point_blocks(g), WR_FIN, WS_FIN, v);
  if (!sm.flag || threadIdx.x != 0) return;  // the last work-group of the task
  WideTask* T = w.st + blockIdx.y;
  int flag = T->flag;
  long long kr_sum = T->kr_sum, kr_max = T->kr_max;
  double res_max = T->res_max;
  if (!rho) {  // account the last step
    const int it = T->done ? T->it : w.prev_its;
    flag |= (T->done || res) ? 0 : FLAG_NOCONV;
    if (res) {
      flag &= ~(FLAG_NOCONV | FLAG_BREAKDOWN);
      res_max = fmax(res_max, T->sum[WS_RR0]);
    }
    kr_sum += it;
    kr_max = it > kr_max ? it : kr_max;
  }
  if (a.target.base && a.res2) {
    const double rr = T->sum[WS_FIN];
    a.res2[blockIdx.y] = res ? fmax(rr, res_max) : rr;
  }
  if (a.counters) {
    atomicAdd(&a.counters[CNT_KRYLOV], (unsigned long long)kr_sum);
    atomicMax(&a.counters[CNT_KRYLOV_MAX], (unsigned long long)kr_max);
    atomicAdd(&a.counters[CNT_SOLVES], (unsigned long long)a.nsteps);
    atomicAdd(&a.counters[CNT_WORK], (unsigned long long)kr_sum * (unsigned long long)g.npts);
  }
  if (flag && a.status) atomicOr(a.status, flag);
}

// Poll (one work-group, the range's tasks): the test the next kernel of
// iteration i would make, then the number of tasks still iterating into
// mapped host memory. With the launch skipped, nothing is iterating.
template <int SOLVER>
__global__ void __launch_bounds__(64) wide_poll_kernel(WideArgs w, int ntasks) {
  int busy = 0;
  const bool skipped = w.a.skip && *w.a.skip != 0.0;
  for (int t = threadIdx.x; t < ntasks && !skipped; t += 64) {
    WideTask* T = w.st + t;
    if (T->done) continue;
    int it, fl;
    if (wide_test_next(T, w.a.tol * w.a.tol, w.i, it, fl)) {
      if (fl) T->flag |= fl;
      T->it = it;
      T->done = 1;
    } else {
      ++busy;
    }
  }
  busy = (int)wave_sum((double)busy);
  if (threadIdx.x == 0) {
    __hip_atomic_store(w.host_out, busy, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
    __threadfence_system();
  }
}

#undef WIDE_KERNEL
#undef WIDE_SMEM

}  // namespace ctm
