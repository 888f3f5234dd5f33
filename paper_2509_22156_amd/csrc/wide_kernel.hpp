// The wide streaming solver: the implicit steps of large systems (streaming
// grids, vectors in HBM), every system spread over many work-groups. Built
// for launches whose task count would leave most of the chip idle under the
// one-work-group-per-task streaming kernel (the sequential coarse chain of
// MGRIT, one task per grid; time-sequential stepping), and with its line
// sweeps staged through LDS also the faster choice for the relaxation
// launches of hundreds of tasks. Every Krylov phase is one launch over all
// work-groups of all tasks of the range (grid dimension y = task), and the
// kernel boundaries are the only grid-wide synchronisation: nothing ever
// waits on another work-group, and no kernel needs a device-wide fence. The
// line factors are computed once per grid and launch and shared by the
// grid's tasks.
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
// Sums: a producing kernel stores one partial per work-group; the kernels
// that need the sum add the partials themselves (one wave, in block order,
// so every consumer gets the same value). Point-wise kernels use 256-thread
// work-groups of kWP points; line kernels one wave per work-group, so that
// their uncoalesced line sweeps spread over as many CUs as possible.
#pragma once

#include "stream_kernel.hpp"
#include "wide_map.h"

namespace ctm {

static_assert(kWideSK == kSK, "the wide solver reads the streaming kernel's line factors");
constexpr int kWLT = 64 * kWLW;  // threads per line work-group

__device__ __forceinline__ int wide_point_blocks(const GridDev& g) {
  return (g.npts + kWP - 1) / kWP;
}
__device__ __forceinline__ int wide_line_blocks(const GridDev& g) {
  const int Lc = pow2ceil((stream_seg_len(g) + kSK - 1) / kSK);
  const int waves = (stream_segments(g) + (64 / Lc) - 1) / (64 / Lc);
  return (waves + kWLW - 1) / kWLW;
}

// Work-group placement (wide_map.h): each task's work-groups on one XCD,
// so that the cache lines its blocks share (stencil halos; the neighbouring
// lines of a grid whose stiff axis is not the fastest) are fetched into one
// L2. Any bijection of (task, block) is valid: the kernels depend on it only
// through the blocks' partial-sum slots, which are indexed by the same
// mapped block.
__device__ __forceinline__ bool wide_grouped() { return wide_in_group(blockIdx.y, gridDim.y); }
__device__ __forceinline__ int wide_bx() {
  return wide_map(blockIdx.x, blockIdx.y, gridDim.x, gridDim.y).x;
}
__device__ __forceinline__ int wide_by() {
  return wide_map(blockIdx.x, blockIdx.y, gridDim.x, gridDim.y).y;
}

// Virtual line block: in a last group of fewer than eight tasks (plain
// order), the line blocks of a grid whose stiff axis is not the fastest are
// regrouped per XCD (wide_line_regroup), so that neighbouring lines share
// one L2.
__device__ __forceinline__ int wide_line_vblock(const GridDev& g) {
  const int b = wide_bx();
  if (wide_grouped() || g.sax == g.d - 1) return b;
  return wide_line_regroup(b, wide_line_blocks(g));
}

struct WideSmem {
  double red[2 * 64];
  int flag;  // done broadcast (multi-wave work-groups)
};

// Shared preamble: the launch-level skip, the task's grid and coefficient
// tables, the block range of the grid, and the done flag. The grid
// descriptor is read in place from the task's state (the chain's first
// kernel copies it there), so that the skip flag, the grid and the done flag
// load in parallel instead of through the task list; only the per-axis
// tables of the SEP and VAR classes are staged in LDS (tl_lds), the
// constant-size DRIFT table is read in place and HEAT has none. A
// single-wave work-group reads `done` itself; a larger one broadcasts thread
// 0's read, so that its waves agree. Returns false (uniformly over the
// work-group) when the block has nothing to do.
template <int OPC, int BT>
__device__ __forceinline__ bool wide_begin(const WideArgs& w, WideSmem& sm, double* tl_lds,
                                           bool line, bool check_done, const GridDev*& gp,
                                           const double*& tl) {
  const ChainArgs& a = w.a;
  WideTask* T = w.st + wide_by();
  const double skipv = a.skip ? *a.skip : 0.0;
  gp = &T->g;
  const GridDev& g = *gp;
  int done = 0;
  if constexpr (BT == 64) done = check_done ? T->done : 0;
  if (skipv != 0.0) return false;
  const int nb = line ? wide_line_blocks(g) : wide_point_blocks(g);
  if (wide_bx() >= nb) return false;
  if constexpr (BT > 64) {
    if (threadIdx.x == 0) sm.flag = check_done ? T->done : 0;
  }
  if constexpr (OPC == OPC_SEP || OPC == OPC_VAR) {
    load_tables<OPC, double, BT>(g, a.tab64, a.dt, tl_lds);
    tl = tl_lds;
  } else {
    tl = a.tab64 + g.tab0;
  }
  if constexpr (BT > 64 || OPC == OPC_SEP || OPC == OPC_VAR) __syncthreads();
  if constexpr (BT > 64) done = sm.flag;
  return done == 0;
}

__device__ __forceinline__ double* wide_sv(const WideArgs& w) {
  return w.scratch + (long long)wide_by() * SV_N * w.ss;
}
// Scratch of the task holding this task's line factors.
__device__ __forceinline__ const double* wide_fsv(const WideArgs& w) {
  return w.scratch + (long long)w.st[wide_by()].fsrc * SV_N * w.ss;
}
__device__ __forceinline__ double* wide_part(const WideArgs& w, int slot) {
  return w.part + ((size_t)wide_by() * WS_N + slot) * w.maxblk;
}

// Store this work-group's partials of slots slot0 .. slot0 + NS - 1.
template <int BT, int NS>
__device__ __forceinline__ void wide_put(const WideArgs& w, WideSmem& sm, int slot0,
                                         double (&v)[NS]) {
  RedRing ring{sm.red, 0};
  block_sum<BT / 64, NS, double>(v, ring);
  if (threadIdx.x == 0) {
#pragma unroll
    for (int s = 0; s < NS; ++s) wide_part(w, slot0 + s)[wide_bx()] = v[s];
  }
}

// The sums of NS slots over their producers' nb[s] work-groups: every wave
// adds the partials in block order itself (no LDS, no barrier), so every
// thread gets the same values.
template <int NS>
__device__ __forceinline__ void wide_sums(const WideArgs& w, const int (&slot)[NS],
                                          const int (&nb)[NS], double (&out)[NS]) {
  const int lane = threadIdx.x & 63;
  int nbmax = 0;
#pragma unroll
  for (int s = 0; s < NS; ++s) nbmax = nb[s] > nbmax ? nb[s] : nbmax;
  double acc[NS];
#pragma unroll
  for (int s = 0; s < NS; ++s) acc[s] = 0.0;
  // every slot's loads of a round are issued together, unconditionally (a
  // block index past a slot's producers reads entry 0, which every slot
  // holds, and adds nothing)
  for (int b = lane; b - lane < nbmax; b += 64) {
    double x[NS];
#pragma unroll
    for (int s = 0; s < NS; ++s) x[s] = wide_part(w, slot[s])[b < nb[s] ? b : 0];
#pragma unroll
    for (int s = 0; s < NS; ++s) acc[s] += (b < nb[s]) ? x[s] : 0.0;
  }
#pragma unroll
  for (int s = 0; s < NS; ++s) out[s] = wave_sum(acc[s]);
}

// Stops the task's step (thread 0 of any deciding work-group; idempotent).
__device__ __forceinline__ void wide_stop(WideTask* T, int it, int flag) {
  if (threadIdx.x != 0) return;
  if (flag) atomicOr(&T->flag, flag);
  T->it = it;
  T->done = 1;
}

__device__ __forceinline__ bool isnan_(double x) { return !(x == x); }

// ------------------------------------------------------- stopping tests
// The start of a step (iteration 1): the initial residual.
__device__ __forceinline__ bool wide_test_init(double rr0, double bb, double tol2, int& it,
                                               int& fl) {
  it = 0;
  fl = 0;
  if (isnan_(rr0) || isnan_(bb)) {
    fl = FLAG_NONFINITE;
    return true;
  }
  return rr0 <= tol2 * bb;
}
// After the r update of iteration itd (CG: (r, r); BiCGStab: also a
// breakdown found in the direction update).
__device__ __forceinline__ bool wide_test_rr(double rr, double bb, int pend, double tol2, int itd,
                                             int& it, int& fl) {
  it = itd;
  fl = 0;
  if (isnan_(rr)) {
    fl = FLAG_NONFINITE;
    return true;
  }
  if (rr <= tol2 * bb) return true;
  if (pend) {
    fl = FLAG_BREAKDOWN;
    return true;
  }
  return false;
}

// The BiCGStab scalars a phase needs: (r0, r0), (b, b), (r^, v) and both
// parities of the t-phase sums.
struct BicgSums {
  double rr0, bb, rhv;
  double d[2][5];  // {ts, tt, ss, rhs, rht} of the iterations of each parity
};
__device__ __forceinline__ void bicg_sums(const WideArgs& w, const GridDev& g, BicgSums& S) {
  const int nb = wide_point_blocks(g);
  constexpr int slot[13] = {WS_RR0, WS_BB, WS_RHV, WS_D, WS_D + 1, WS_D + 2, WS_D + 3, WS_D + 4,
                            WS_D + 5, WS_D + 6, WS_D + 7, WS_D + 8, WS_D + 9};
  const int nbs[13] = {nb, nb, nb, nb, nb, nb, nb, nb, nb, nb, nb, nb, nb};
  double v[13];
  wide_sums<13>(w, slot, nbs, v);
  S.rr0 = v[0];
  S.bb = v[1];
  S.rhv = v[2];
#pragma unroll
  for (int m = 0; m < 5; ++m) {
    S.d[0][m] = v[3 + m];
    S.d[1][m] = v[8 + m];
  }
}
// The t-phase sums of iteration k (selected, not indexed: the parity is a
// run-time value and an indexed register array would live in scratch).
__device__ __forceinline__ void bicg_d(const BicgSums& S, int k, double (&D)[5]) {
  const bool odd = (k & 1) != 0;
#pragma unroll
  for (int m = 0; m < 5; ++m) D[m] = odd ? S.d[1][m] : S.d[0][m];
}
// rho_k = (r^, r_{k-1}): rho_1 = (r0, r0); rho_k = rhs - omega rht of k-1.
__device__ __forceinline__ double bicg_rho(const BicgSums& S, int k) {
  if (k == 1) return S.rr0;
  double D[5];
  bicg_d(S, k - 1, D);
  return D[3] - (D[0] / D[1]) * D[4];
}

// ------------------------------------------------------- point-wise helpers
template <int OPC, int D, class F>
__device__ __forceinline__ double wide_Ax(const GridDev& g, const double* tl, double dt,
                                          double amp, int p, F x) {
  PointCoef<OPC, D> c;
  point_coef<OPC, D>(g, tl, dt, amp, p, c);
  double xl[D], xu[D];
#pragma unroll
  for (int i = 0; i < D; ++i) {
    xl[i] = x(stencil_lo(g, c, i, p));
    xu[i] = x(stencil_up(g, c, i, p));
  }
  double v = c.diag * x(p);
#pragma unroll
  for (int i = 0; i < D; ++i) v += c.lo[i] * xl[i] + c.up[i] * xu[i];
  return v;
}

// ------------------------------------------------------- line helpers
// Lane of this thread in the line layout (wave w of the block: virtual wave
// wide_line_vblock * kWLW + w of the task).
template <int D>
__device__ __forceinline__ void wide_lane(const GridDev& g, SLane& L) {
  stream_lane_at<D>(g, wide_line_vblock(g) * kWLW + (threadIdx.x >> 6), threadIdx.x & 63, L);
}
// Point index of unknown k of the lane's chunk (< 2^20: a 32-bit offset).
__device__ __forceinline__ unsigned lane_pt(const SLane& L, int k) {
  return (unsigned)L.base + (unsigned)((L.j0 + k) * L.step);
}
// Loads and stores at a 32-bit element offset from a work-group-uniform
// base, so that the compiler addresses with a scalar base and one 32-bit
// offset register per unknown (shared by every vector), not a 64-bit
// address per load.
__device__ __forceinline__ double ldo(const double* base, unsigned i) {
  return *reinterpret_cast<const double*>(reinterpret_cast<const char*>(base) +
                                          (size_t)(i * 8u));
}
__device__ __forceinline__ void sto(double* base, unsigned i, double v) {
  *reinterpret_cast<double*>(reinterpret_cast<char*>(base) + (size_t)(i * 8u)) = v;
}
__device__ __forceinline__ float ldo(const float* base, unsigned i) {
  return *reinterpret_cast<const float*>(reinterpret_cast<const char*>(base) +
                                         (size_t)(i * 4u));
}

// Line sweeps of a wave. Where the stiff axis is the grid's fastest axis
// (stride 1), the wave's 64 / Lc lines are one contiguous range of at most
// 64 kSK unknowns, and a lane's chunk is kSK consecutive values: read
// directly, every load instruction touches 64 cache lines. For launches of
// many tasks (WideArgs::stage) the wave stages its lines through LDS there:
// coalesced global loads (element m * 64 + lane) into a padded tile (one
// pad slot per chunk, so that the lanes' chunk reads fall in different
// banks), then each lane reads its chunk; stores the other way round.
// Otherwise the lanes read their chunks directly (launches of few tasks are
// latency-bound, and the extra LDS round trip did not pay there).
constexpr int kTileMax = 64 * kSK;                   // unknowns of a wave's lines
constexpr int kTilePad = kTileMax + kTileMax / kSK;  // with one pad per chunk
constexpr int kTileVecs = 2;                         // tile slots (vectors per LDS pass)
__device__ __forceinline__ int tpad(int e) { return e + e / kSK; }

struct WaveTile {
  bool on;      // staged
  unsigned t0;  // first unknown of the wave's lines
  int n;        // unknowns of the wave's lines
  int e0;       // this lane's chunk start inside the range
};
__device__ __forceinline__ WaveTile wave_tile(const WideArgs& w, const GridDev& g,
                                              const SLane& L) {
  WaveTile T;
  // (lines cut into segments are read directly: a wave's segments need
  // not be one contiguous range)
  T.on = w.stage && (g.sax == g.d - 1) && g.nseg == 1;
  const int G = 64 / L.Lc;
  const int line0 = (wide_line_vblock(g) * kWLW + (int)(threadIdx.x >> 6)) * G;
  const int gv = g.nlines - line0 < G ? g.nlines - line0 : G;
  T.t0 = (unsigned)line0 * (unsigned)g.ns;
  T.n = gv * g.ns;
  T.e0 = ((int)(threadIdx.x & 63) / L.Lc) * g.ns + L.j0;
  return T;
}

// out[s][k] = vector s at unknown k of the lane's chunk (0 past nval).
// TE: the vectors' element type (double; float for the line factors, which
// then pass through the wave's tile region as floats).
template <int NV, typename TE = double>
__device__ __forceinline__ void line_gather(const WaveTile& T, const SLane& L,
                                            const TE* const (&v)[NV], double* tile,
                                            TE (&out)[NV][kSK]) {
  if (!T.on) {
#pragma unroll
    for (int k = 0; k < kSK; ++k) {
      const bool ok = k < L.nval;
      const unsigned p = lane_pt(L, k);
#pragma unroll
      for (int s = 0; s < NV; ++s) out[s][k] = ok ? ldo(v[s], p) : (TE)0;
    }
    return;
  }
  TE* tw = reinterpret_cast<TE*>(tile + (threadIdx.x >> 6) * (kTileVecs * kTilePad));
  const int lane = threadIdx.x & 63;
  // every global load first (one round trip), then the vectors pass
  // through the tile kTileVecs at a time (a small tile keeps more
  // work-groups resident per CU)
  TE tmp[NV][kSK];
#pragma unroll
  for (int m = 0; m < kSK; ++m) {
    const int e = m * 64 + lane;
    const bool ok = e < T.n;
#pragma unroll
    for (int s = 0; s < NV; ++s) tmp[s][m] = ok ? ldo(v[s], T.t0 + (unsigned)e) : (TE)0;
  }
#pragma unroll
  for (int s0 = 0; s0 < NV; s0 += kTileVecs) {
#pragma unroll
    for (int m = 0; m < kSK; ++m) {
      const int e = m * 64 + lane;
      if (e < T.n) {
#pragma unroll
        for (int s = s0; s < NV && s < s0 + kTileVecs; ++s)
          tw[(s - s0) * kTilePad + tpad(e)] = tmp[s][m];
      }
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < kSK; ++k) {
      const bool ok = k < L.nval;
#pragma unroll
      for (int s = s0; s < NV && s < s0 + kTileVecs; ++s)
        out[s][k] = ok ? tw[(s - s0) * kTilePad + tpad(T.e0 + k)] : (TE)0;
    }
    __syncthreads();  // the tile is reused by the next pass, gather or scatter
  }
}

// vector s at unknown k of the lane's chunk = in[s][k] (k < nval).
template <int NV>
__device__ __forceinline__ void line_scatter(const WaveTile& T, const SLane& L,
                                             double* const (&v)[NV], double* tile,
                                             const double (&in)[NV][kSK]) {
  if (!T.on) {
#pragma unroll
    for (int k = 0; k < kSK; ++k)
      if (k < L.nval) {
        const unsigned p = lane_pt(L, k);
#pragma unroll
        for (int s = 0; s < NV; ++s) sto(v[s], p, in[s][k]);
      }
    return;
  }
  double* tw = tile + (threadIdx.x >> 6) * (kTileVecs * kTilePad);
  const int lane = threadIdx.x & 63;
#pragma unroll
  for (int s0 = 0; s0 < NV; s0 += kTileVecs) {
#pragma unroll
    for (int k = 0; k < kSK; ++k)
      if (k < L.nval) {
#pragma unroll
        for (int s = s0; s < NV && s < s0 + kTileVecs; ++s)
          tw[(s - s0) * kTilePad + tpad(T.e0 + k)] = in[s][k];
      }
    __syncthreads();
#pragma unroll
    for (int m = 0; m < kSK; ++m) {
      const int e = m * 64 + lane;
      if (e < T.n) {
#pragma unroll
        for (int s = s0; s < NV && s < s0 + kTileVecs; ++s)
          sto(v[s], T.t0 + (unsigned)e, tw[(s - s0) * kTilePad + tpad(e)]);
      }
    }
    __syncthreads();
  }
}

// z = M^-1 r on the chunk of lane L in registers (r and z hold the chunk's
// kSK unknowns; entries past nval are ignored / returned 0). The five factor
// vectors are gathered in one pass. They are stored in FP32 (half the bytes
// and registers; the arithmetic stays FP64): M is then the exact line-block
// solve up to a relative perturbation of the FP32 rounding, a fixed linear
// operator, so the Krylov solve still converges to the FP64 tolerance; only
// its iteration count can change.
__device__ __forceinline__ void wide_pre(const double* fsv, long long ss, const WaveTile& T,
                                         const SLane& L, double* tile, const double (&r)[kSK],
                                         double (&z)[kSK]) {
  auto fv_at = [&](int slot) { return reinterpret_cast<const float*>(fsv + slot * ss); };
  const float* const fv[5] = {fv_at(SV_FM), fv_at(SV_FID), fv_at(SV_FCU), fv_at(SV_FPHI),
                              fv_at(SV_FPSI)};
  float f[5][kSK];
  line_gather<5, float>(T, L, fv, tile, f);
  const float* fm = f[0];
  const float* fid = f[1];
  const float* fcu = f[2];
  const float* fph = f[3];
  const float* fps = f[4];
  const bool full = (L.nval == kSK);
  const int ne = L.nval < kSK - 1 ? L.nval : kSK - 1;
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
#define WIDE_SMEM                                        \
  extern __shared__ __align__(16) unsigned char smem[]; \
  __shared__ WideSmem sm;                               \
  const GridDev* gp = nullptr;                          \
  const double* tl = nullptr;                           \
  double* tl_lds = reinterpret_cast<double*>(smem)

#define WIDE_TILE __shared__ double tile[kWLW * kTileVecs * kTilePad]
static_assert(kWLW * kTileVecs * kTilePad * sizeof(double) + sizeof(WideSmem) <= kWideStaticLds,
              "static LDS of the line kernels");

// Factors of the line preconditioner (once per chain).
template <int OPC, int D>
__global__ void __launch_bounds__(kWLT) wide_setup_kernel(WideArgs w) {
  WIDE_SMEM;
  // the chain's first kernel: the grid comes from the task list, and work-
  // group 0 of each task copies it (and the interval) into the task's state
  // for the kernels that follow
  const ChainArgs& a = w.a;
  if (a.skip && *a.skip != 0.0) return;
  const int2 task = a.tasks[wide_by()];
  const GridDev& g = a.grids[task.x];
  WideTask* T = w.st + wide_by();
  // the factors depend on the grid and the step only: the first task of the
  // launch on this grid computes them, the others read that task's copy
  // (one wave: the lanes scan the earlier tasks, a shuffle tree takes the
  // minimum)
  int fsrc = wide_by();
  for (int t = (int)threadIdx.x; t < wide_by(); t += 64)
    if (a.tasks[t].x == task.x) {
      fsrc = t;
      break;
    }
#pragma unroll
  for (int sh = 32; sh >= 1; sh >>= 1) {
    const int o = __shfl_xor(fsrc, sh, 64);
    fsrc = o < fsrc ? o : fsrc;
  }
  if (wide_bx() == 0) {
    const int* src = reinterpret_cast<const int*>(&g);
    int* dst = reinterpret_cast<int*>(&T->g);
    for (int t = threadIdx.x; t < (int)(sizeof(GridDev) / sizeof(int)); t += kWLT) dst[t] = src[t];
    if (threadIdx.x == 0) {
      T->q = task.y;
      T->fsrc = fsrc;
    }
  }
  if (wide_bx() >= wide_line_blocks(g) || fsrc != wide_by()) return;
  if constexpr (OPC == OPC_SEP || OPC == OPC_VAR) {
    load_tables<OPC, double, kWLT>(g, a.tab64, a.dt, tl_lds);
    tl = tl_lds;
    __syncthreads();
  } else {
    tl = a.tab64 + g.tab0;
  }
  (void)sm;
  (void)gp;
  double* sv = wide_sv(w);
  SLane L;
  wide_lane<D>(g, L);
  linepre_setup_lane<OPC, D, float>(g, tl, a.dt, a.amp, sv, w.ss, sv + SV_S * w.ss, L);
}

// Step transition (point-wise; step j): finish step j-1 (B = x + forcing,
// intermediate store) or load the start vector (j = 1); the residual-mode
// forcing; then either the exact residual b - A target (residual mode, last
// step) or the initial guess. Work-group 0 accounts step j-1 and resets the
// task's step state.
template <int OPC, int D>
__global__ void __launch_bounds__(kWT) wide_step_kernel(WideArgs w) {
  WIDE_SMEM;
  if (!wide_begin<OPC, kWT>(w, sm, tl_lds, false, false, gp, tl)) return;
  const ChainArgs& a = w.a;
  const GridDev& g = *gp;
  const int q = w.st[wide_by()].q;
  const int j = w.j;
  const bool last = (j == a.nsteps), res = a.resmode != 0;
  if (wide_bx() == 0) {
    double rr0 = 0.0;
    if (j > 1 && res) {
      const int slot[1] = {WS_RR0}, nb[1] = {wide_point_blocks(g)};
      double v[1];
      wide_sums<1>(w, slot, nb, v);
      rr0 = v[0];
    }
    if (threadIdx.x == 0) {
      WideTask* T = w.st + wide_by();
      if (j == 1) {
        T->kr_sum = T->kr_max = 0;
        T->res_max = 0.0;
        T->flag = 0;
      } else {
        const int it = T->done ? T->it : w.prev_its;
        int fl = T->flag | ((T->done || res) ? 0 : FLAG_NOCONV);
        if (res) {
          fl &= ~(FLAG_NOCONV | FLAG_BREAKDOWN);
          T->res_max = fmax(T->res_max, rr0);
        }
        T->flag = fl;
        T->kr_sum += it;
        T->kr_max = it > T->kr_max ? it : T->kr_max;
      }
      T->done = T->it = T->pend = 0;
    }
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
  const double tj = a.ft0 + (double)q * a.ftq + (double)j * a.dt;  // time of step j
  const VecRef gr = last ? a.guess_fin : a.guess;
  const double* gx = (!rho && gr.base) ? at(gr, gr.a * q + gr.b + (last ? 0 : j)) : nullptr;
  // (every load before the stores: the vectors may share a base)
  double b0[kWPT], b1[kWPT], xg[kWPT];
#pragma unroll
  for (int k = 0; k < kWPT; ++k) {
    const int p = wide_bx() * kWP + k * kWT + threadIdx.x;
    b0[k] = b1[k] = xg[k] = 0.0;
    if (p >= g.npts) continue;
    const double b = (j == 1) ? (st ? st[p] : 0.0) : X[p] + (fp ? fp[p] : 0.0);
    double bb = b + (fj ? fj[p] : 0.0);
    // manufactured heat problem: (I + dt L) x = v + dt f(t_j)
    if constexpr (OPC == OPC_HEAT) {
      if (a.fkind && !res) bb += a.dt * mms_point<D>(g, p, tj);
    }
    if (rho) bb -= wide_Ax<OPC, D>(g, tl, a.dt, a.amp, p, [&](int i) { return tg[i]; });
    b0[k] = b;
    b1[k] = bb;
    xg[k] = gx ? gx[p] : bb;
  }
#pragma unroll
  for (int k = 0; k < kWPT; ++k) {
    const int p = wide_bx() * kWP + k * kWT + threadIdx.x;
    if (p >= g.npts) continue;
    if (wb) wb[p] = b0[k];
    if (is) is[p] = b0[k];
    if (!rho) X[p] = xg[k];
    B[p] = b1[k];
  }
}

// Initial residual of the step (stencil): r = b - A x; BiCGStab also sets
// r^ = p = r. Partials of (r, r), (b, b).
template <int OPC, int SOLVER, int D>
__global__ void __launch_bounds__(kWT) wide_init_kernel(WideArgs w) {
  WIDE_SMEM;
  if (!wide_begin<OPC, kWT>(w, sm, tl_lds, false, false, gp, tl)) return;
  const ChainArgs& a = w.a;
  const GridDev& g = *gp;
  double* sv = wide_sv(w);
  const long long ss = w.ss;
  const double* X = sv + SV_X * ss;
  const double* B = sv + SV_B * ss;
  double* R = sv + SV_R * ss;
  double* RH = sv + SV_RH * ss;
  double* P = sv + SV_P * ss;
  double v[2] = {0.0, 0.0};
  double rv[kWPT];
#pragma unroll
  for (int k = 0; k < kWPT; ++k) {
    const int p = wide_bx() * kWP + k * kWT + threadIdx.x;
    rv[k] = 0.0;
    if (p >= g.npts) continue;
    const double b = B[p];
    const double r = b - wide_Ax<OPC, D>(g, tl, a.dt, a.amp, p, [&](int i) { return X[i]; });
    rv[k] = r;
    v[0] += r * r;
    v[1] += b * b;
  }
#pragma unroll
  for (int k = 0; k < kWPT; ++k) {
    const int p = wide_bx() * kWP + k * kWT + threadIdx.x;
    if (p >= g.npts) continue;
    R[p] = rv[k];
    if constexpr (SOLVER == SOLV_BICG) {
      RH[p] = rv[k];
      P[p] = rv[k];
    }
  }
  static_assert(WS_BB == WS_RR0 + 1, "slot order");
  wide_put<kWT, 2>(w, sm, WS_RR0, v);
}

// ---- BiCGStab, iteration i: K_A(i) [lines], K_B(i), K_C(i) [lines], K_D(i)
// K_A(i): i = 1: the initial test, h = M^-1 p. i > 1: the end of iteration
// i-1 (tests on (s, s) and (t, t); omega: x += omega h, r = s - omega t,
// partial (r, r)), the direction p = r + beta (p - omega v), h = M^-1 p.
template <int OPC, int D>
__global__ void __launch_bounds__(kWLT) wide_bicg_a_kernel(WideArgs w) {
  WIDE_SMEM;
  WIDE_TILE;
  if (!wide_begin<OPC, kWLT>(w, sm, tl_lds, true, true, gp, tl)) return;
  const ChainArgs& a = w.a;
  const GridDev& g = *gp;
  WideTask* T = w.st + wide_by();
  const double tol2 = a.tol * a.tol;
  const int i = w.i;
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
  const WaveTile Tl = wave_tile(w, g, L);
  // The first pass's loads go out before the sums' loads (they do not
  // depend on them; a stopped task discards them). All loads of a pass are
  // issued before its stores: the vectors share one base, so the compiler
  // cannot move a load above an earlier store.
  double pr[kSK], hz[kSK];
  double rr[1] = {0.0};
  int it, fl;
  if (i == 1) {
    {
      const double* const v1[1] = {P};
      double o[1][kSK];
      line_gather<1>(Tl, L, v1, tile, o);
#pragma unroll
      for (int k = 0; k < kSK; ++k) pr[k] = o[0][k];
    }
    const int slot[2] = {WS_RR0, WS_BB}, nb[2] = {wide_point_blocks(g), wide_point_blocks(g)};
    double v[2];
    wide_sums<2>(w, slot, nb, v);
    if (wide_test_init(v[0], v[1], tol2, it, fl)) {
      wide_stop(T, it, fl);
      return;
    }
  } else {
    const double* const v4[4] = {X, H, S, Tv};
    double o[4][kSK];
    line_gather<4>(Tl, L, v4, tile, o);
    BicgSums Sm;
    bicg_sums(w, g, Sm);
    double Dn[5];
    bicg_d(Sm, i - 1, Dn);
    const double tt = Dn[1];
    if (Dn[2] <= tol2 * Sm.bb) {
      wide_stop(T, i - 1, 0);  // x already holds x + alpha h
      return;
    }
    if (!(tt != 0.0) || isnan_(tt)) {
      wide_stop(T, i - 1, isnan_(tt) ? FLAG_NONFINITE : FLAG_BREAKDOWN);
      return;
    }
    const double omega = Dn[0] / tt;
    const double rho_o = bicg_rho(Sm, i - 1), rho_n = bicg_rho(Sm, i);
    const double alpha = rho_o / Sm.rhv;
    const bool pend = (rho_n == 0.0 || omega == 0.0);
    const double beta = pend ? 0.0 : (rho_n / rho_o) * (alpha / omega);
    if (pend && wide_bx() == 0 && threadIdx.x == 0) T->pend = 1;
    // r = s - omega t, x += omega h; then p = r + beta (p - omega v)
    {
      double st[2][kSK];
#pragma unroll
      for (int k = 0; k < kSK; ++k) {
        const double r = o[2][k] - omega * o[3][k];
        pr[k] = r;
        rr[0] += r * r;
        st[0][k] = o[0][k] + omega * o[1][k];
        st[1][k] = r;
      }
      double* const d2[2] = {X, R};
      line_scatter<2>(Tl, L, d2, tile, st);
    }
    {
      const double* const v2[2] = {P, V};
      double o2[2][kSK], st[1][kSK];
      line_gather<2>(Tl, L, v2, tile, o2);
#pragma unroll
      for (int k = 0; k < kSK; ++k) {
        const double pn = pr[k] + beta * (o2[0][k] - omega * o2[1][k]);
        pr[k] = (k < L.nval) ? pn : 0.0;
        st[0][k] = pn;
      }
      double* const d1[1] = {P};
      line_scatter<1>(Tl, L, d1, tile, st);
    }
  }
  wide_pre(wide_fsv(w), ss, Tl, L, tile, pr, hz);
  {
    double* const d1[1] = {H};
    const double(&st)[1][kSK] = reinterpret_cast<const double(&)[1][kSK]>(hz);
    line_scatter<1>(Tl, L, d1, tile, st);
  }
  if (i > 1) wide_put<kWLT, 1>(w, sm, WS_RR, rr);
}

// K_B(i): the test of the r update (i > 1); v = A h, partial (r^, v).
template <int OPC, int D>
__global__ void __launch_bounds__(kWT) wide_bicg_b_kernel(WideArgs w) {
  WIDE_SMEM;
  if (!wide_begin<OPC, kWT>(w, sm, tl_lds, false, true, gp, tl)) return;
  const ChainArgs& a = w.a;
  const GridDev& g = *gp;
  WideTask* T = w.st + wide_by();
  double* sv = wide_sv(w);
  const long long ss = w.ss;
  const double* H = sv + SV_D * ss;
  const double* RH = sv + SV_RH * ss;
  double* V = sv + SV_Q * ss;
  // (the stencil's loads go out before the sums' loads; a stopped task
  // discards them)
  double v[1] = {0.0};
  double yv[kWPT];
#pragma unroll
  for (int k = 0; k < kWPT; ++k) {
    const int p = wide_bx() * kWP + k * kWT + threadIdx.x;
    yv[k] = 0.0;
    if (p >= g.npts) continue;
    const double y = wide_Ax<OPC, D>(g, tl, a.dt, a.amp, p, [&](int m) { return H[m]; });
    yv[k] = y;
    v[0] += RH[p] * y;
  }
  if (w.i > 1) {
    const int slot[2] = {WS_RR, WS_BB}, nb[2] = {wide_line_blocks(g), wide_point_blocks(g)};
    double sr[2];
    wide_sums<2>(w, slot, nb, sr);
    int it, fl;
    if (wide_test_rr(sr[0], sr[1], T->pend, a.tol * a.tol, w.i - 1, it, fl)) {
      wide_stop(T, it, fl);
      return;
    }
  }
#pragma unroll
  for (int k = 0; k < kWPT; ++k) {
    const int p = wide_bx() * kWP + k * kWT + threadIdx.x;
    if (p < g.npts) V[p] = yv[k];
  }
  wide_put<kWT, 1>(w, sm, WS_RHV, v);
}

// K_C(i): alpha = rho / (r^, v); x += alpha h, s = r - alpha v, h = M^-1 s.
template <int OPC, int D>
__global__ void __launch_bounds__(kWLT) wide_bicg_c_kernel(WideArgs w) {
  WIDE_SMEM;
  WIDE_TILE;
  if (!wide_begin<OPC, kWLT>(w, sm, tl_lds, true, true, gp, tl)) return;
  const GridDev& g = *gp;
  WideTask* T = w.st + wide_by();
  double* sv = wide_sv(w);
  const long long ss = w.ss;
  double* X = sv + SV_X * ss;
  const double* R = sv + SV_R * ss;
  const double* V = sv + SV_Q * ss;
  double* S = sv + SV_S * ss;
  double* H = sv + SV_D * ss;
  SLane L;
  wide_lane<D>(g, L);
  const WaveTile Tl = wave_tile(w, g, L);
  // the data loads go out before the sums' (they do not depend on them; a
  // stopped task discards them), so both share one memory round trip
  const double* const v4[4] = {X, H, R, V};
  double o[4][kSK];
  line_gather<4>(Tl, L, v4, tile, o);
  BicgSums Sm;
  bicg_sums(w, g, Sm);
  const double rhv = Sm.rhv;
  if (!(rhv != 0.0) || isnan_(rhv)) {
    wide_stop(T, w.i, isnan_(rhv) ? FLAG_NONFINITE : FLAG_BREAKDOWN);
    return;
  }
  const double alpha = bicg_rho(Sm, w.i) / rhv;
  double sr[kSK], hz[kSK];
  {
    double st[2][kSK];
#pragma unroll
    for (int k = 0; k < kSK; ++k) {
      const double sk = o[2][k] - alpha * o[3][k];
      sr[k] = sk;
      st[0][k] = o[0][k] + alpha * o[1][k];
      st[1][k] = sk;
    }
    double* const d2[2] = {X, S};
    line_scatter<2>(Tl, L, d2, tile, st);
  }
  wide_pre(wide_fsv(w), ss, Tl, L, tile, sr, hz);
  {
    double* const d1[1] = {H};
    const double(&st)[1][kSK] = reinterpret_cast<const double(&)[1][kSK]>(hz);
    line_scatter<1>(Tl, L, d1, tile, st);
  }
}

// K_D(i): t = A h; partials (t, s), (t, t), (s, s), (r^, s), (r^, t).
template <int OPC, int D>
__global__ void __launch_bounds__(kWT) wide_bicg_d_kernel(WideArgs w) {
  WIDE_SMEM;
  if (!wide_begin<OPC, kWT>(w, sm, tl_lds, false, true, gp, tl)) return;
  const ChainArgs& a = w.a;
  const GridDev& g = *gp;
  double* sv = wide_sv(w);
  const long long ss = w.ss;
  const double* H = sv + SV_D * ss;
  const double* S = sv + SV_S * ss;
  const double* RH = sv + SV_RH * ss;
  double* Tv = sv + SV_T * ss;
  double v[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
  double tv[kWPT];
#pragma unroll
  for (int k = 0; k < kWPT; ++k) {
    const int p = wide_bx() * kWP + k * kWT + threadIdx.x;
    tv[k] = 0.0;
    if (p >= g.npts) continue;
    const double t = wide_Ax<OPC, D>(g, tl, a.dt, a.amp, p, [&](int m) { return H[m]; });
    tv[k] = t;
    const double s = S[p], rh = RH[p];
    v[0] += t * s;
    v[1] += t * t;
    v[2] += s * s;
    v[3] += rh * s;
    v[4] += rh * t;
  }
#pragma unroll
  for (int k = 0; k < kWPT; ++k) {
    const int p = wide_bx() * kWP + k * kWT + threadIdx.x;
    if (p < g.npts) Tv[p] = tv[k];
  }
  wide_put<kWT, 5>(w, sm, WS_D + 5 * (w.i & 1), v);
}

// ---- CG, iteration i: K_CA(i) [lines], K_CB(i), K_CC(i)
// K_CA(i): the test of the previous r update; z = M^-1 r, partial (r, z).
template <int OPC, int D>
__global__ void __launch_bounds__(kWLT) wide_cg_a_kernel(WideArgs w) {
  WIDE_SMEM;
  WIDE_TILE;
  if (!wide_begin<OPC, kWLT>(w, sm, tl_lds, true, true, gp, tl)) return;
  const GridDev& g = *gp;
  WideTask* T = w.st + wide_by();
  const double tol2 = w.a.tol * w.a.tol;
  double* sv = wide_sv(w);
  const long long ss = w.ss;
  const double* R = sv + SV_R * ss;
  double* Z = sv + SV_S * ss;
  SLane L;
  wide_lane<D>(g, L);
  const WaveTile Tl = wave_tile(w, g, L);
  // (the r loads go out before the sums' loads)
  double rv[kSK], zv[kSK];
  {
    const double* const v1[1] = {R};
    double o[1][kSK];
    line_gather<1>(Tl, L, v1, tile, o);
#pragma unroll
    for (int k = 0; k < kSK; ++k) rv[k] = o[0][k];
  }
  {
    const int slot[3] = {WS_RR0, WS_BB, WS_RR};
    const int nb[3] = {wide_point_blocks(g), wide_point_blocks(g),
                       w.i > 1 ? wide_point_blocks(g) : 0};
    double v[3];
    wide_sums<3>(w, slot, nb, v);
    int it, fl;
    const bool stop = (w.i == 1) ? wide_test_init(v[0], v[1], tol2, it, fl)
                                 : wide_test_rr(v[2], v[1], 0, tol2, w.i - 1, it, fl);
    if (stop) {
      wide_stop(T, it, fl);
      return;
    }
  }
  wide_pre(wide_fsv(w), ss, Tl, L, tile, rv, zv);
  double v[1] = {0.0};
#pragma unroll
  for (int k = 0; k < kSK; ++k) v[0] += rv[k] * zv[k];
  {
    double* const d1[1] = {Z};
    const double(&st)[1][kSK] = reinterpret_cast<const double(&)[1][kSK]>(zv);
    line_scatter<1>(Tl, L, d1, tile, st);
  }
  wide_put<kWLT, 1>(w, sm, WS_RZ + (w.i & 1), v);
}

// K_CB(i): p_i = z + beta p_{i-1} (the two directions alternate between
// two vectors, so that neighbours read the old one while it is replaced),
// q = A p_i, partial (p, q).
template <int OPC, int D>
__global__ void __launch_bounds__(kWT) wide_cg_b_kernel(WideArgs w) {
  WIDE_SMEM;
  if (!wide_begin<OPC, kWT>(w, sm, tl_lds, false, true, gp, tl)) return;
  const ChainArgs& a = w.a;
  const GridDev& g = *gp;
  const int i = w.i;
  double beta = 0.0;
  if (i > 1) {
    const int slot[2] = {WS_RZ + (i & 1), WS_RZ + ((i - 1) & 1)};
    const int nb[2] = {wide_line_blocks(g), wide_line_blocks(g)};
    double v[2];
    wide_sums<2>(w, slot, nb, v);
    beta = v[0] / v[1];
  }
  double* sv = wide_sv(w);
  const long long ss = w.ss;
  const double* Z = sv + SV_S * ss;
  // (iteration 1: beta = 0 and the old direction reads z, so that no
  // unwritten vector is read)
  const double* Po = (i == 1) ? Z : sv + ((i & 1) ? SV_RH : SV_P) * ss;
  double* Pn = sv + ((i & 1) ? SV_P : SV_RH) * ss;
  double* Q = sv + SV_Q * ss;
  double v[1] = {0.0};
  double pvv[kWPT], yv[kWPT];
#pragma unroll
  for (int k = 0; k < kWPT; ++k) {
    const int p = wide_bx() * kWP + k * kWT + threadIdx.x;
    pvv[k] = yv[k] = 0.0;
    if (p >= g.npts) continue;
    auto pv = [&](int m) { return Z[m] + beta * Po[m]; };
    const double y = wide_Ax<OPC, D>(g, tl, a.dt, a.amp, p, pv);
    const double pp = pv(p);
    pvv[k] = pp;
    yv[k] = y;
    v[0] += pp * y;
  }
#pragma unroll
  for (int k = 0; k < kWPT; ++k) {
    const int p = wide_bx() * kWP + k * kWT + threadIdx.x;
    if (p >= g.npts) continue;
    Pn[p] = pvv[k];
    Q[p] = yv[k];
  }
  wide_put<kWT, 1>(w, sm, WS_PQ, v);
}

// K_CC(i): alpha = (r, z) / (p, q); x += alpha p, r -= alpha q, partial (r, r).
template <int OPC, int D>
__global__ void __launch_bounds__(kWT) wide_cg_c_kernel(WideArgs w) {
  WIDE_SMEM;
  if (!wide_begin<OPC, kWT>(w, sm, tl_lds, false, true, gp, tl)) return;
  const GridDev& g = *gp;
  WideTask* T = w.st + wide_by();
  const int i = w.i;
  const int slot[2] = {WS_PQ, WS_RZ + (i & 1)};
  const int nb[2] = {wide_point_blocks(g), wide_line_blocks(g)};
  double sc[2];
  wide_sums<2>(w, slot, nb, sc);
  const double pq = sc[0];
  if (!(pq != 0.0) || isnan_(pq)) {
    wide_stop(T, i, isnan_(pq) ? FLAG_NONFINITE : FLAG_BREAKDOWN);
    return;
  }
  const double alpha = sc[1] / pq;
  double* sv = wide_sv(w);
  const long long ss = w.ss;
  double* X = sv + SV_X * ss;
  double* R = sv + SV_R * ss;
  const double* Pn = sv + ((i & 1) ? SV_P : SV_RH) * ss;
  const double* Q = sv + SV_Q * ss;
  double v[1] = {0.0};
  double xv[kWPT], rv[kWPT];
#pragma unroll
  for (int k = 0; k < kWPT; ++k) {
    const int p = wide_bx() * kWP + k * kWT + threadIdx.x;
    xv[k] = rv[k] = 0.0;
    if (p >= g.npts) continue;
    xv[k] = X[p] + alpha * Pn[p];
    const double r = R[p] - alpha * Q[p];
    rv[k] = r;
    v[0] += r * r;
  }
#pragma unroll
  for (int k = 0; k < kWPT; ++k) {
    const int p = wide_bx() * kWP + k * kWT + threadIdx.x;
    if (p >= g.npts) continue;
    X[p] = xv[k];
    R[p] = rv[k];
  }
  wide_put<kWT, 1>(w, sm, WS_RR, v);
}

// The end of the chain (point-wise): the last step's x + forcing (or the
// exact residual formed by the step kernel), fin = v - target, partial
// ||fin||^2.
template <int OPC, int D>
__global__ void __launch_bounds__(kWT) wide_fin_kernel(WideArgs w) {
  WIDE_SMEM;
  if (!wide_begin<OPC, kWT>(w, sm, tl_lds, false, false, gp, tl)) return;
  const ChainArgs& a = w.a;
  const GridDev& g = *gp;
  const int q = w.st[wide_by()].q;
  const bool res = a.resmode != 0;
  const bool rho = res && a.target.base;  // the step kernel formed the residual
  double* sv = wide_sv(w);
  const double* X = sv + SV_X * w.ss;
  const double* B = sv + SV_B * w.ss;
  const long long off = g.off;
  auto at = [&](const VecRef& r, long long idx) { return r.base + idx * a.slen + off; };
  const double* fl = (!res && a.forcing.base)
                         ? at(a.forcing, a.forcing.a * q + a.forcing.b + a.nsteps) : nullptr;
  double* dst = a.fin.base ? at(a.fin, a.fin.a * q + a.fin.b) : nullptr;
  const double* tg = (!rho && a.target.base) ? at(a.target, a.target.a * q + a.target.b)
                                              : nullptr;
  double v[1] = {0.0};
#pragma unroll
  for (int k = 0; k < kWPT; ++k) {
    const int p = wide_bx() * kWP + k * kWT + threadIdx.x;
    if (p >= g.npts || !dst) continue;
    double u = rho ? B[p] : X[p] + (fl ? fl[p] : 0.0);
    if (tg) u -= tg[p];
    dst[p] = u;
    v[0] += u * u;
  }
  wide_put<kWT, 1>(w, sm, WS_FIN, v);
}

// After the chain (one wave per task): account the last step, publish
// res2 (residual mode: the max with the steps' initial residuals), the
// counters and the status bits.
template <int OPC>
__global__ void __launch_bounds__(64) wide_finish_kernel(WideArgs w) {
  WIDE_SMEM;
  if (!wide_begin<OPC, 64>(w, sm, tl_lds, false, false, gp, tl)) return;
  const ChainArgs& a = w.a;
  const GridDev& g = *gp;
  const bool res = a.resmode != 0;
  const bool rho = res && a.target.base;
  const int slot[2] = {WS_FIN, WS_RR0}, nb[2] = {wide_point_blocks(g), wide_point_blocks(g)};
  double v[2];
  wide_sums<2>(w, slot, nb, v);
  if (threadIdx.x != 0) return;
  WideTask* T = w.st + wide_by();
  int flag = T->flag;
  long long kr_sum = T->kr_sum, kr_max = T->kr_max;
  double res_max = T->res_max;
  if (!rho) {  // account the last step
    const int it = T->done ? T->it : w.prev_its;
    flag |= (T->done || res) ? 0 : FLAG_NOCONV;
    if (res) {
      flag &= ~(FLAG_NOCONV | FLAG_BREAKDOWN);
      res_max = fmax(res_max, v[1]);
    }
    kr_sum += it;
    kr_max = it > kr_max ? it : kr_max;
  }
  if (a.target.base && a.res2) a.res2[wide_by()] = res ? fmax(v[0], res_max) : v[0];
  if (a.counters) {
    atomicAdd(&a.counters[CNT_KRYLOV], (unsigned long long)kr_sum);
    atomicMax(&a.counters[CNT_KRYLOV_MAX], (unsigned long long)kr_max);
    atomicAdd(&a.counters[CNT_SOLVES], (unsigned long long)a.nsteps);
    atomicAdd(&a.counters[CNT_WORK], (unsigned long long)kr_sum * (unsigned long long)g.npts);
    atomicAdd(&a.counters[CNT_DOFSTEPS], (unsigned long long)a.nsteps * (unsigned long long)g.npts);
  }
  if (flag && a.status) atomicOr(a.status, flag);
}

// Poll (one wave per task): the test the next kernel of iteration i would
// make first (BiCGStab: the start of K_B(i); CG: the start of K_CA(i)),
// then 1 (still iterating) or 0 into host_out[task] (mapped host memory).
// With the launch skipped, nothing is iterating.
template <int OPC, int SOLVER>
__global__ void __launch_bounds__(64) wide_poll_kernel(WideArgs w) {
  WIDE_SMEM;
  const bool skipped = w.a.skip && *w.a.skip != 0.0;
  int busy = 0;
  if (!skipped && wide_begin<OPC, 64>(w, sm, tl_lds, false, true, gp, tl)) {
    const GridDev& g = *gp;
    const int nbr = (SOLVER == SOLV_BICG) ? wide_line_blocks(g) : wide_point_blocks(g);
    const int slot[3] = {WS_RR0, WS_BB, WS_RR};
    const int nb[3] = {wide_point_blocks(g), wide_point_blocks(g), w.i > 1 ? nbr : 0};
    double v[3];
    wide_sums<3>(w, slot, nb, v);
    WideTask* T = w.st + wide_by();
    int it, fl;
    const double tol2 = w.a.tol * w.a.tol;
    const bool stop = (w.i == 1) ? wide_test_init(v[0], v[1], tol2, it, fl)
                                 : wide_test_rr(v[2], v[1], T->pend, tol2, w.i - 1, it, fl);
    if (stop)
      wide_stop(T, it, fl);
    else
      busy = 1;
  }
  if (threadIdx.x == 0)
    __hip_atomic_store(w.host_out + wide_by(), busy, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
}

#undef WIDE_SMEM
#undef WIDE_TILE

}  // namespace ctm
