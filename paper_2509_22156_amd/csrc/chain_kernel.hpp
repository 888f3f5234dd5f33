// The batched implicit-step kernel ("chain"): one work-group per task
// (component grid g, time interval q). A task loads its start vector into
// registers and applies `nsteps` backward-Euler steps v <- Phi(v) + f_j
// (Section 2, time propagation), each solved matrix-free by preconditioned
// CG or BiCGStab (Section 4.1) with every vector held on chip: the lane's
// own unknowns in registers, one LDS copy of the vector the stencil reads.
// This one kernel carries every time-stepping phase of MGRIT (F-, C- and
// FC-relaxation, the C-point residual, the sequential coarse-level solve;
// Section 2.3.1) and plain time-sequential stepping; the phases differ only
// in which vectors are read and written (see ChainArgs).
//
// Precision: FP64, or mixed: FP64 iterative refinement of each implicit
// step (FP64 residual b - A x) around an FP32 preconditioned Krylov solve of
// the correction.
#pragma once

#include "line_layout.hpp"
#include "manufactured.hpp"

namespace ctm {

template <typename T>
__device__ __forceinline__ bool finite_val(T v) {
  return v == v && v - v == (T)0;
}

// Quotient of two Krylov scalars. FP32 (the inner solves) uses the hardware
// reciprocal (about 1 ulp): the recurrences do not need a correctly rounded
// quotient, and the FP64 refinement around them decides convergence. FP64
// keeps the IEEE division.
template <typename T>
__device__ __forceinline__ T kdiv(T a, T b) {
  if constexpr (sizeof(T) == 4) return a * __builtin_amdgcn_rcpf(b);
  else return a / b;
}

template <int OPC, typename T, int K>
struct Solver {
  const GridDev& g;
  const Lane<K>& L;
  const LineOp<OPC, T, K>& O;
  const PreOf<OPC, T, K>& M;
  T* xl;  // LDS vector (precision T)
};

// y = A x (x written to LDS first; one barrier).
template <int OPC, typename T, int W, int K>
__device__ __forceinline__ void sapply(const Solver<OPC, T, K>& S, const T (&x)[K], T (&y)[K]) {
  if (S.g.d > 1) {  // one-dimensional grids need no neighbour lines
    lds_put<T, K, lds_pitch(W)>(S.L, S.xl, x);
    __syncthreads();
  }
  line_apply<OPC, T, K, lds_pitch(W)>(S.g, S.L, S.O, S.xl, x, y);
}

// Preconditioned CG in the single-reduction form of Chronopoulos and Gear:
// per iteration one preconditioner solve, one stencil apply and one fused
// reduction of (r,z), (Az,z), (r,r). x holds the initial guess (x_zero:
// it is zero and the first apply is skipped). Stops when
// ||b - A x||_2^2 <= tol2 * bb on the recursively updated residual.
// check_first (a guess that may already be converged): test the initial
// residual on its own reduction before the first preconditioner solve.
template <int OPC, typename T, int W, int K>
__device__ __forceinline__ int krylov_pcg(const Solver<OPC, T, K>& S, RedRing& ring, T (&x)[K],
                                          const T (&b)[K], bool x_zero, bool check_first,
                                          T tol2, int maxit, int* flag, T* rr0 = nullptr,
                                          T* rel_end = nullptr) {
  T r[K], z[K], w[K], p[K], s[K];
  if (x_zero) {
#pragma unroll
    for (int k = 0; k < K; ++k) r[k] = b[k];
  } else {
    sapply<OPC, T, W, K>(S, x, w);
#pragma unroll
    for (int k = 0; k < K; ++k) r[k] = b[k] - w[k];
    __syncthreads();  // every wave has read x from LDS before z overwrites it
  }
  if (check_first && !x_zero) {
    T s2[2] = {(T)0, (T)0};
#pragma unroll
    for (int k = 0; k < K; ++k) {
      s2[0] += r[k] * r[k];
      s2[1] += b[k] * b[k];
    }
    block_sum<W, 2, T>(s2, ring);
    if (rr0) *rr0 = s2[0];
    if (!finite_val(s2[0]) || !finite_val(s2[1])) {
      *flag |= FLAG_NONFINITE;
      return 0;
    }
    if (s2[0] <= tol2 * s2[1]) return 0;
  }
  linepre_apply<OPC, T, K, 64 * W>(S.L, S.O, S.M, r, z);
  sapply<OPC, T, W, K>(S, z, w);
  // (r,z), (Az,z), (r,r) and, unless x = 0 (then b = r), (b,b)
  T red[4] = {(T)0, (T)0, (T)0, (T)0};
#pragma unroll
  for (int k = 0; k < K; ++k) {
    red[0] += r[k] * z[k];
    red[1] += w[k] * z[k];
    red[2] += r[k] * r[k];
    red[3] += b[k] * b[k];
  }
  block_sum<W, 4, T>(red, ring);
  if (rr0 && !(check_first && !x_zero)) *rr0 = red[2];
  const T bb = x_zero ? red[2] : red[3];
  if (!finite_val(red[2]) || !finite_val(red[1]) || !finite_val(bb)) {
    *flag |= FLAG_NONFINITE;
    return 0;
  }
  if (red[2] <= tol2 * bb) {
    if (rel_end) *rel_end = red[2] / bb;
    return 0;
  }
  T gamma = red[0];
  T alpha = kdiv(gamma, red[1]);
#pragma unroll
  for (int k = 0; k < K; ++k) {
    p[k] = z[k];
    s[k] = w[k];
  }
  for (int it = 1; it <= maxit; ++it) {
#pragma unroll
    for (int k = 0; k < K; ++k) {
      x[k] += alpha * p[k];
      r[k] -= alpha * s[k];
    }
    linepre_apply<OPC, T, K, 64 * W>(S.L, S.O, S.M, r, z);
    sapply<OPC, T, W, K>(S, z, w);
    T rd[3] = {(T)0, (T)0, (T)0};
#pragma unroll
    for (int k = 0; k < K; ++k) {
      rd[0] += r[k] * z[k];
      rd[1] += w[k] * z[k];
      rd[2] += r[k] * r[k];
    }
    block_sum<W, 3, T>(rd, ring);
    if (!finite_val(rd[2]) || !finite_val(rd[1])) {
      *flag |= FLAG_NONFINITE;
      return it;
    }
    if (rd[2] <= tol2 * bb) {
      if (rel_end) *rel_end = rd[2] / bb;
      return it;
    }
    const T beta = kdiv(rd[0], gamma);
    const T den = rd[1] - beta * kdiv(rd[0], alpha);
    if (den == (T)0 || !finite_val(den)) {
      *flag |= FLAG_BREAKDOWN;
      return it;
    }
    alpha = kdiv(rd[0], den);
    gamma = rd[0];
#pragma unroll
    for (int k = 0; k < K; ++k) {
      p[k] = z[k] + beta * p[k];
      s[k] = w[k] + beta * s[k];
    }
  }
  *flag |= FLAG_NOCONV;
  return maxit;
}

// Right-preconditioned BiCGStab (van der Vorst), shadow residual r^ = r_0.
template <int OPC, typename T, int W, int K>
__device__ __forceinline__ int krylov_pbicgstab(const Solver<OPC, T, K>& S, RedRing& ring,
                                                T (&x)[K], const T (&b)[K], bool x_zero, T tol2,
                                                int maxit, int* flag, T* rr0 = nullptr) {
  T r[K], rh[K], p[K], v[K], s[K], t[K], h[K];
  if (x_zero) {
#pragma unroll
    for (int k = 0; k < K; ++k) r[k] = b[k];
  } else {
    sapply<OPC, T, W, K>(S, x, v);
#pragma unroll
    for (int k = 0; k < K; ++k) r[k] = b[k] - v[k];
  }
  T s1[2] = {(T)0, (T)0};
#pragma unroll
  for (int k = 0; k < K; ++k) {
    rh[k] = r[k];
    p[k] = r[k];
    s1[0] += r[k] * r[k];
    s1[1] += b[k] * b[k];
  }
  block_sum<W, 2, T>(s1, ring);
  if (rr0) *rr0 = s1[0];
  const T bb = x_zero ? s1[0] : s1[1];
  if (!finite_val(s1[0]) || !finite_val(bb)) {
    *flag |= FLAG_NONFINITE;
    return 0;
  }
  if (s1[0] <= tol2 * bb) return 0;
  T rho = s1[0];
  for (int it = 1; it <= maxit; ++it) {
    linepre_apply<OPC, T, K, 64 * W>(S.L, S.O, S.M, p, h);
    sapply<OPC, T, W, K>(S, h, v);
    T s2[1] = {(T)0};
#pragma unroll
    for (int k = 0; k < K; ++k) s2[0] += rh[k] * v[k];
    block_sum<W, 1, T>(s2, ring);
    if (s2[0] == (T)0 || !finite_val(s2[0])) {
      *flag |= finite_val(s2[0]) ? FLAG_BREAKDOWN : FLAG_NONFINITE;
      return it;
    }
    const T alpha = kdiv(rho, s2[0]);
#pragma unroll
    for (int k = 0; k < K; ++k) {
      x[k] += alpha * h[k];
      s[k] = r[k] - alpha * v[k];
    }
    linepre_apply<OPC, T, K, 64 * W>(S.L, S.O, S.M, s, h);
    sapply<OPC, T, W, K>(S, h, t);
    T s3[3] = {(T)0, (T)0, (T)0};
#pragma unroll
    for (int k = 0; k < K; ++k) {
      s3[0] += t[k] * s[k];
      s3[1] += t[k] * t[k];
      s3[2] += s[k] * s[k];
    }
    block_sum<W, 3, T>(s3, ring);
    if (s3[2] <= tol2 * bb) return it;
    if (s3[1] == (T)0 || !finite_val(s3[1])) {
      *flag |= finite_val(s3[1]) ? FLAG_BREAKDOWN : FLAG_NONFINITE;
      return it;
    }
    const T omega = kdiv(s3[0], s3[1]);
    T s4[2] = {(T)0, (T)0};
#pragma unroll
    for (int k = 0; k < K; ++k) {
      x[k] += omega * h[k];
      r[k] = s[k] - omega * t[k];
      s4[0] += r[k] * r[k];
      s4[1] += rh[k] * r[k];
    }
    block_sum<W, 2, T>(s4, ring);
    if (!finite_val(s4[0])) {
      *flag |= FLAG_NONFINITE;
      return it;
    }
    if (s4[0] <= tol2 * bb) return it;
    if (s4[1] == (T)0 || omega == (T)0) {
      *flag |= FLAG_BREAKDOWN;
      return it;
    }
    const T beta = kdiv(s4[1], rho) * kdiv(alpha, omega);
    rho = s4[1];
#pragma unroll
    for (int k = 0; k < K; ++k) p[k] = r[k] + beta * (p[k] - omega * v[k]);
  }
  *flag |= FLAG_NOCONV;
  return maxit;
}

template <int OPC, int SOLVER, typename T, int W, int K>
__device__ __forceinline__ int krylov(const Solver<OPC, T, K>& S, RedRing& ring, T (&x)[K],
                                      const T (&b)[K], bool x_zero, T tol2, int maxit,
                                      int* flag, bool check_first = false, T* rr0 = nullptr,
                                      T* rel_end = nullptr) {
  if constexpr (SOLVER == SOLV_CG)
    return krylov_pcg<OPC, T, W, K>(S, ring, x, b, x_zero, check_first, tol2, maxit, flag, rr0,
                                    rel_end);
  else
    return krylov_pbicgstab<OPC, T, W, K>(S, ring, x, b, x_zero, tol2, maxit, flag, rr0);
}

__device__ __forceinline__ double* vec_at(const VecRef& r, long long idx, long long slen,
                                          long long off) {
  return r.base + idx * slen + off;
}

// A lane's K values in HBM. A lane whose chunk holds fewer than K unknowns
// reads (and writes back) its first unknown in the place of the missing
// ones, so that the K accesses form one block without per-value branches:
// the compiler made each predicated store wait for the previous one to
// complete, a memory round trip per value, measured at up to a third of a
// small task's life. Rewriting the first unknown with its own value is
// harmless; idle lanes (no unknowns) touch nothing.
// gload_raw leaves a copy of the first value in the slots past the chunk's
// end and uses nothing it loads, so that a prefetch does not wait;
// pad_zero then clears those slots where the values are consumed.
template <int K>
__device__ __forceinline__ void gload_raw(const Lane<K>& L, const double* src, double (&v)[K]) {
  if (L.nval > 0) {
#pragma unroll
    for (int k = 0; k < K; ++k) v[k] = src[L.cbase + (long long)(k < L.nval ? k : 0) * L.cstep];
  } else {
#pragma unroll
    for (int k = 0; k < K; ++k) v[k] = 0.0;
  }
}
template <int K>
__device__ __forceinline__ void pad_zero(const Lane<K>& L, double (&v)[K]) {
#pragma unroll
  for (int k = 0; k < K; ++k) v[k] = k < L.nval ? v[k] : 0.0;
}
template <int K>
__device__ __forceinline__ void gload(const Lane<K>& L, const double* src, double (&v)[K]) {
  gload_raw<K>(L, src, v);
  pad_zero<K>(L, v);
}
template <int K>
__device__ __forceinline__ void gstore(const Lane<K>& L, double* dst, const double (&v)[K]) {
  if (L.nval > 0) {
#pragma unroll
    for (int k = 0; k < K; ++k) {
      const bool in = k < L.nval;
      dst[L.cbase + (long long)(in ? k : 0) * L.cstep] = in ? v[k] : v[0];
    }
  }
}

// One implicit step in FP64: x <- (I + dt L)^-1 v (x: the initial guess;
// warm: a guess that may already meet the tolerance).
template <int OPC, int SOLVER, int W, int K>
__device__ __forceinline__ void step_fp64(const Solver<OPC, double, K>& S, RedRing& ring,
                                          const double (&v)[K], double tol2, int maxit,
                                          bool warm, double (&x)[K], int* flag,
                                          long long& kr_sum, long long& kr_max) {
  const int it =
      krylov<OPC, SOLVER, double, W, K>(S, ring, x, v, false, tol2, maxit, flag, warm);
  kr_sum += it;
  kr_max = it > kr_max ? it : kr_max;
}

// One implicit step by FP64 iterative refinement around FP32 Krylov solves.
// Bound on the gap between the true residual of an FP32 CG correction and
// the recursive residual the CG recurrences carry, relative to the norm of
// the right-hand side: the rounding of the right-hand side to FP32, of the
// FP32 operator's coefficients, and of the recurrences over `it` iterations,
// each a small multiple of the FP32 unit roundoff times ||A|| ||d|| (standard
// rounding-error analysis of CG; ||d|| <= 1 since A = I + dt L with L
// symmetric positive semi-definite, so A >= I), with a safety factor of 32.
// `anorm` bounds ||A||_2 (Gershgorin).
__device__ __forceinline__ double cg_gap_bound(int it, double anorm) {
  return 32.0 * 5.9604644775390625e-08 * (double)(it + 3) * anorm;
}

template <int OPC, int SOLVER, int W, int K, class Apply64>
__device__ __forceinline__ void step_mixed(const Apply64& apply64,
                                           const Solver<OPC, float, K>& S32, RedRing& ring,
                                           const double (&v)[K], double tol2, float itol2,
                                           int maxit, int refine_maxit, double (&x)[K],
                                           int* flag, long long& kr_sum, long long& kr_max,
                                           long long& rf_sum, long long& rf_max,
                                           double anorm) {
  bool conv = false;
  int sweeps = 0, its = 0;
  double bb = 0.0;
  for (; sweeps <= refine_maxit; ++sweeps) {
    double rq[K];
    apply64(x, rq);
    double rr[2] = {0.0, 0.0};
#pragma unroll
    for (int k = 0; k < K; ++k) {
      rq[k] = v[k] - rq[k];
      rr[0] += rq[k] * rq[k];
      rr[1] += v[k] * v[k];
    }
    if (sweeps == 0) {
      block_sum<W, 2, double>(rr, ring);
      bb = rr[1];
    } else {
      double r1[1] = {rr[0]};
      block_sum<W, 1, double>(r1, ring);
      rr[0] = r1[0];
    }
    if (!finite_val(rr[0]) || !finite_val(bb)) {
      *flag |= FLAG_NONFINITE;
      break;
    }
    if (rr[0] <= tol2 * bb) {
      conv = true;
      break;
    }
    if (sweeps == refine_maxit) break;
    const double nr = sqrt(rr[0]);
    const double inv = 1.0 / nr;
    float r32[K], d32[K];
#pragma unroll
    for (int k = 0; k < K; ++k) {
      r32[k] = (float)(rq[k] * inv);
      d32[k] = 0.0f;
    }
    // inner target: the reduction the outer test still needs, with a factor
    // of two in hand, (tol ||b|| / 2 ||r||)^2, but never below the FP32
    // floor inner_tol and at least a halving of the residual. A warm-started
    // step that is already close to the tolerance then takes one or two FP32
    // iterations instead of a full solve to inner_tol.
    double t2 = 0.25 * tol2 * bb / rr[0];
    t2 = t2 > (double)itol2 ? t2 : (double)itol2;
    t2 = t2 < 0.25 ? t2 : 0.25;
    int iflag = 0;
    float rel = 1.0f;
    const int it = krylov<OPC, SOLVER, float, W, K>(S32, ring, d32, r32, true, (float)t2, maxit,
                                                    &iflag, false, nullptr, &rel);
    its += it;
    if (iflag & FLAG_NONFINITE) {
      *flag |= FLAG_NONFINITE;
      break;
    }
#pragma unroll
    for (int k = 0; k < K; ++k) x[k] += nr * (double)d32[k];
    // CG on a symmetric operator (anorm > 0): the FP64 residual after the
    // correction is at most nr (sqrt(rel) + gap). Where that bound already
    // meets the tolerance the step ends without computing it; the next
    // step, and the MGRIT residual, start from FP64 residuals as always.
    if constexpr (SOLVER == SOLV_CG) {
      if (anorm > 0.0 && iflag == 0) {
        const double est = nr * (sqrt((double)rel) + cg_gap_bound(it, anorm));
        if (est * est <= tol2 * bb) {
          ++sweeps;
          conv = true;
          break;
        }
      }
    }
  }
  if (!conv) *flag |= FLAG_NOCONV;
  kr_sum += its;
  kr_max = its > kr_max ? its : kr_max;
  rf_sum += sweeps;
  rf_max = sweeps > rf_max ? sweeps : rf_max;
}

// One implicit step as a single FP32 solve from zero (mixed path, loose
// coarse-level tolerance): x <- (I + dt L)^-1 v to relative tolerance itol.
// (Starting from the state one step earlier instead cut the FP32 Krylov
// iterations of the 6-D workload by a quarter but raised its MGRIT
// iterations from 11 to 15: the coarse corrections were worse.)
template <int OPC, int SOLVER, int W, int K>
__device__ __forceinline__ void step_single32(const Solver<OPC, float, K>& S32, RedRing& ring,
                                              const double (&v)[K], float itol2, int maxit,
                                              double (&x)[K], int* flag, long long& kr_sum,
                                              long long& kr_max) {
  float b32[K], d32[K];
#pragma unroll
  for (int k = 0; k < K; ++k) {
    b32[k] = (float)v[k];
    d32[k] = 0.0f;
  }
  const int it = krylov<OPC, SOLVER, float, W, K>(S32, ring, d32, b32, true, itol2, maxit, flag);
#pragma unroll
  for (int k = 0; k < K; ++k) x[k] = (double)d32[k];
  kr_sum += it;
  kr_max = it > kr_max ? it : kr_max;
}

// MODE_FORCED (heat only): the steps add the manufactured-problem forcing;
// a separate instantiation, so that the forcing's transcendental functions
// do not raise the register budget of the plain kernels.
// MODE_RESIDUAL: space-time residual mode of MGRIT. Every step is a fixed
// number of Krylov iterations from the given initial guess (an inexact step
// that refines the previous iterate; in the mixed path one FP32 correction
// solve of that many iterations on the FP64 residual), the forcing is added
// before the step (the coarse equation A_c e_m = e_{m-1} + rho_m), and in
// residual mode (target given) the last step is replaced by the exact
// space-time residual rho = v - A target; the task's residual norm is the
// largest over that and the initial residuals of its other steps.
enum { MODE_PLAIN = 0, MODE_FORCED = 1, MODE_RESIDUAL = 2 };

// Waves per SIMD the compiler must leave room for. gfx950 gives a SIMD 512
// vector registers per lane: a kernel over 256 runs one wave per SIMD, and
// the chain kernels, bound by the latency of their reductions and barriers,
// then idle. The mixed K = 4 kernels of the variable-coefficient operator
// held the FP64 and the FP32 line operator in registers (about 290); with
// most of the FP64 one parked in LDS they need about 190, and the bound
// keeps them at two waves should that grow again (held to 256 before the
// parking they spilled under 40 registers and ran 25% faster than at one
// wave; held to three waves, 168, they spilled over 120 and ran 65% slower).
template <int OPC, bool MIXED, int MODE, int W, int K>
constexpr int chain_min_waves() {
  return (OPC == OPC_VAR && K == 4 && (MIXED || MODE != MODE_RESIDUAL)) ? 2 : 1;
}

template <int OPC, int SOLVER, bool MIXED, int MODE, int W, int K>
__global__ void __launch_bounds__(64 * W)
    __attribute__((amdgpu_waves_per_eu(chain_min_waves<OPC, MIXED, MODE, W, K>())))
    chain_kernel(ChainArgs a, int tabmax) {
  constexpr bool FORCED = (MODE == MODE_FORCED);
  constexpr bool RES = (MODE == MODE_RESIDUAL);
  constexpr int BS = 64 * W;
  extern __shared__ __align__(16) unsigned char smem[];
  // mixed K = 4 variable-coefficient chains keep most of the FP64 line
  // operator in LDS (parked after set-up, loaded for each FP64 residual): it
  // would hold 30 more registers through the FP32 inner solves
  constexpr bool PARK = MIXED && OPC == OPC_VAR && K == 4;
  const ChainSmem lay = chain_smem_layout(W, K, tabmax, MIXED, OPC == OPC_HEAT, a.pcrmax, PARK);
  double* xl64 = reinterpret_cast<double*>(smem);
  double* ocv64 = reinterpret_cast<double*>(smem + lay.ocv);
  float* ocv32 = reinterpret_cast<float*>(ocv64 + MAXD);
  float* xl32 = reinterpret_cast<float*>(smem + lay.x32);
  double* tl64 = reinterpret_cast<double*>(smem + lay.tab);
  float* tl32 = reinterpret_cast<float*>(tl64 + tabmax);
  HeatTab<double, K>* ht64 = reinterpret_cast<HeatTab<double, K>*>(smem + lay.heat);
  HeatTab<float, K>* ht32 = reinterpret_cast<HeatTab<float, K>*>(
      smem + lay.heat + align16(sizeof(HeatTab<double, K>)));
  double* red = reinterpret_cast<double*>(smem + lay.red);
  __shared__ GridDev gs;
  if (a.skip && *a.skip != 0.0) return;  // whole work-group: queued past convergence
  lds_zero_ghosts<double, K>(xl64);
  if constexpr (MIXED) lds_zero_ghosts<float, K>(xl32);

  const int2 task = a.tasks[blockIdx.x];
  const int q = task.y;
  {
    const int* src = reinterpret_cast<const int*>(a.grids + task.x);
    int* dst = reinterpret_cast<int*>(&gs);
    for (int t = threadIdx.x; t < (int)(sizeof(GridDev) / sizeof(int)); t += BS) dst[t] = src[t];
  }
  __syncthreads();
  const GridDev& g = gs;
  load_tables<OPC, double, BS>(g, a.tab64, a.dt, tl64);
  if constexpr (MIXED) load_tables<OPC, float, BS>(g, a.tab64, a.dt, tl32);
  __syncthreads();

  Lane<K> L;
  setup_lane<K>(g, L);
  LineOp<OPC, double, K> O64;
  lineop_setup<OPC, double, K>(g, L, a.dt, a.amp, tl64, ht64, ocv64, O64);
  double* op64 = reinterpret_cast<double*>(smem + lay.op);
  LineOpVarKeep<K> keep64;
  if constexpr (PARK) lineop_park<K, BS>(O64, op64, keep64);

  const long long off = g.off;
  double v[K];
  if (a.start.base) {
    gload<K>(L, vec_at(a.start, a.start.a * q + a.start.b, a.slen, off), v);
  } else {
#pragma unroll
    for (int k = 0; k < K; ++k) v[k] = 0.0;
  }
  if (a.start_wb.base)
    gstore<K>(L, vec_at(a.start_wb, a.start_wb.a * q + a.start_wb.b, a.slen, off), v);

  RedRing ring{red, 0};
  int flag = 0;
  long long kr_sum = 0, kr_max = 0, rf_sum = 0, rf_max = 0;
  const double tol2 = a.tol * a.tol;

  // preconditioner and FP32 operator (mixed) are built once per chain
  PreOf<OPC, double, K> M64;
  LineOp<OPC, float, K> O32;
  PreOf<OPC, float, K> M32;
  if constexpr (MIXED) {
    lineop_setup<OPC, float, K>(g, L, a.dt, a.amp, tl32, ht32, ocv32, O32);
    linepre_setup<OPC, float, K, BS>(L, O32, M32, reinterpret_cast<float*>(smem + lay.pre),
                                     a.pcrmax, &flag);
  } else {
    linepre_setup<OPC, double, K, BS>(L, O64, M64, reinterpret_cast<double*>(smem + lay.pre),
                                      a.pcrmax, &flag);
  }
  if constexpr (OPC == OPC_HEAT && MIXED) __syncthreads();  // FP64 weights visible
  const Solver<OPC, double, K> S64{g, L, O64, M64, xl64};
  const Solver<OPC, float, K> S32{g, L, O32, M32, xl32};
  // y = A x in FP64 (the parked operator is loaded for the apply only)
  auto apply64 = [&](const double (&xin)[K], double (&yout)[K]) {
    if constexpr (PARK) {
      LineOp<OPC, double, K> Ol;
      lineop_unpark<K, BS>(Ol, op64, keep64, ocv64);
      const Solver<OPC, double, K> Sl{g, L, Ol, M64, xl64};
      sapply<OPC, double, W, K>(Sl, xin, yout);
    } else {
      sapply<OPC, double, W, K>(S64, xin, yout);
    }
  };
  const float itol2 = (float)(a.inner_tol * a.inner_tol);
  // ||I + dt L||_2 <= 1 + dt sum_i 4 a_max / h_i^2 (Gershgorin; a_max = 1 for
  // the heat operator, 1 + |amp| for the variable coefficient) for the
  // symmetric operators; 0 (no bound) for the others
  double anorm = 0.0;
  if constexpr (OPC == OPC_HEAT || OPC == OPC_VAR) {
    const double amax = (OPC == OPC_VAR) ? 1.0 + fabs(a.amp) : 1.0;
    double sum = 0.0;
    for (int i = 0; i < g.d; ++i) sum += g.ih2[i];
    anorm = 1.0 + a.dt * 4.0 * amax * sum;
  }
  double res_max = 0.0;  // residual mode: largest squared residual of the task's steps

  // initial guess of step j: the given one (a previous iterate at this time
  // point: guess for j < nsteps, guess_fin for the last step), else the state
  // one step earlier. The FP64 kernels of the operators with per-line
  // coefficients, and the mixed ones that park their FP64 operator, load
  // given guesses one step ahead, so that their memory latency hides behind
  // the solve of the step before (measured: 6% off the 6-D FP64 solve; the
  // heat kernels and the other mixed ones lose a wave of occupancy to the
  // extra registers, or gain nothing, and load at the step).
  constexpr bool kPrefetch = (!MIXED && OPC != OPC_HEAT) || PARK;
  auto guess_of = [&](int j) -> const VecRef& { return j == a.nsteps ? a.guess_fin : a.guess; };
  auto guess_at = [&](int j) {
    const VecRef& r = guess_of(j);
    return vec_at(r, r.a * q + r.b + (j == a.nsteps ? 0 : j), a.slen, off);
  };
  double gnext[K];
  if constexpr (kPrefetch) {
    if (guess_of(1).base) gload_raw<K>(L, guess_at(1), gnext);
  }
  for (int j = 1; j <= a.nsteps; ++j) {
    // The state after step j - 1 (still in v) is written to `inter` here, at
    // the start of step j rather than at the end of step j - 1. A wait for a
    // load also waits for every store issued before it, and the prefetched
    // guess is waited for as soon as a step ends: stored there, the state
    // cost a full write round trip per step. Stored after that wait and
    // before the next prefetch, it completes during the solve. The kernels
    // that load the guess at the step store first, so that the store and
    // the load overlap.
    const bool put = a.inter.base && j > 1;
    auto put_prev = [&]() {
      gstore<K>(L, vec_at(a.inter, a.inter.a * q + a.inter.b + (j - 1), a.slen, off), v);
    };
    if constexpr (!kPrefetch) {
      if (put) put_prev();
    }
    // heat (few registers in use): the forcing of this step is loaded
    // before the solve, so that its latency hides behind it
    constexpr bool kEarly = (OPC == OPC_HEAT);
    double f[K];
    if (kEarly && a.forcing.base)
      gload<K>(L, vec_at(a.forcing, a.forcing.a * q + a.forcing.b + j, a.slen, off), f);
    double x[K];
    const bool last = (j == a.nsteps);
    const VecRef& gr = guess_of(j);
    if (gr.base) {
      if constexpr (kPrefetch) {
#pragma unroll
        for (int k = 0; k < K; ++k) x[k] = gnext[k];
        pad_zero<K>(L, x);
      } else {
        gload<K>(L, guess_at(j), x);
      }
    } else {
#pragma unroll
      for (int k = 0; k < K; ++k) x[k] = v[k];
    }
    if constexpr (kPrefetch) {
      // the prefetched guess has arrived before the stores issue
      // (s_waitcnt vmcnt(0), on every path): left to itself the compiler
      // orders the copy of the guess after the stores, and its wait then
      // includes theirs
      __builtin_amdgcn_s_waitcnt(0x0F70);
      if (put) put_prev();
      if (!last && guess_of(j + 1).base) gload_raw<K>(L, guess_at(j + 1), gnext);
    }
    // manufactured heat problem: the step solves (I + dt L) x = v + dt f(t_j)
    if constexpr (FORCED) {
      double fj[K];
      mms_forcing<K>(g, L, a.ft0 + (double)q * a.ftq + (double)j * a.dt, fj);
#pragma unroll
      for (int k = 0; k < K; ++k) v[k] += a.dt * fj[k];
    }
    if constexpr (RES) {
      if (a.forcing.base) {  // before the step
        if (!kEarly)
          gload<K>(L, vec_at(a.forcing, a.forcing.a * q + a.forcing.b + j, a.slen, off), f);
#pragma unroll
        for (int k = 0; k < K; ++k) v[k] += f[k];
      }
      if (last && a.target.base) {
        // exact space-time residual at the C-point: rho = v - A target
        double tg[K], y[K];
        gload<K>(L, vec_at(a.target, a.target.a * q + a.target.b, a.slen, off), tg);
        apply64(tg, y);
#pragma unroll
        for (int k = 0; k < K; ++k) v[k] = (k < L.nval) ? v[k] - y[k] : 0.0;
      } else {
        // fixed-count inexact step from the previous iterate; its initial
        // residual enters the task's residual norm
        double r0 = 0.0;
        int it;
        if constexpr (MIXED) {
          // x += d, A d = v - A x solved in FP32 by a.maxit iterations
          double rq[K];
          apply64(x, rq);
          double rr[1] = {0.0};
          float r32[K], d32[K];
#pragma unroll
          for (int k = 0; k < K; ++k) {
            rq[k] = v[k] - rq[k];
            rr[0] += rq[k] * rq[k];
            r32[k] = 0.0f;
            d32[k] = 0.0f;
          }
          block_sum<W, 1, double>(rr, ring);
          r0 = rr[0];
          it = 0;
          if (r0 > 0.0 && finite_val(r0)) {
            // the residual is normalised before rounding to FP32
            const double nr = sqrt(r0), inv = 1.0 / nr;
#pragma unroll
            for (int k = 0; k < K; ++k) r32[k] = (float)(rq[k] * inv);
            int iflag = 0;
            // FP32 stops at inner_tol (its own noise floor) if it gets
            // there before a.maxit iterations
            it = krylov<OPC, SOLVER, float, W, K>(S32, ring, d32, r32, true, itol2, a.maxit,
                                                  &iflag);
            flag |= iflag & FLAG_NONFINITE;
#pragma unroll
            for (int k = 0; k < K; ++k) x[k] += nr * (double)d32[k];
          } else if (!finite_val(r0)) {
            flag |= FLAG_NONFINITE;
          }
        } else {
          it = krylov<OPC, SOLVER, double, W, K>(S64, ring, x, v, false, 0.0, a.maxit, &flag,
                                                 gr.base != nullptr, &r0);
        }
        // an inexact step ends where it ends: the iteration limit, or a
        // vanishing BiCGStab denominator once the step's residual is ~0,
        // leaves a valid iterate (the space-time residual test decides)
        flag &= ~(FLAG_NOCONV | FLAG_BREAKDOWN);
        kr_sum += it;
        kr_max = it > kr_max ? it : kr_max;
        res_max = r0 > res_max ? r0 : res_max;
#pragma unroll
        for (int k = 0; k < K; ++k) v[k] = x[k];
      }
    } else {
      if constexpr (MIXED) {
        if (a.single32)
          step_single32<OPC, SOLVER, W, K>(S32, ring, v, itol2, a.maxit, x, &flag, kr_sum,
                                           kr_max);
        else
          step_mixed<OPC, SOLVER, W, K>(apply64, S32, ring, v, tol2, itol2, a.maxit,
                                        a.refine_maxit, x, &flag, kr_sum, kr_max, rf_sum, rf_max,
                                        anorm);
      } else {
        step_fp64<OPC, SOLVER, W, K>(S64, ring, v, tol2, a.maxit, gr.base != nullptr, x, &flag,
                                     kr_sum, kr_max);
      }
      if (a.forcing.base) {
        if (!kEarly)
          gload<K>(L, vec_at(a.forcing, a.forcing.a * q + a.forcing.b + j, a.slen, off), f);
#pragma unroll
        for (int k = 0; k < K; ++k) v[k] = x[k] + f[k];
      } else {
#pragma unroll
        for (int k = 0; k < K; ++k) v[k] = x[k];
      }
    }
  }

  // statistics: counter i from lane i (the values are uniform over the
  // work-group), so that the task ends with two atomic instructions rather
  // than a chain of single-lane ones, each waiting for the one before; ahead
  // of the final stores, whose data registers they would otherwise wait for
  if (a.counters && threadIdx.x < CNT_N) {
    const int t = threadIdx.x;
    const unsigned long long npts = (unsigned long long)g.npts;
    unsigned long long val = 0;
    switch (t) {
      case CNT_KRYLOV: val = (unsigned long long)kr_sum; break;
      case CNT_KRYLOV_MAX: val = (unsigned long long)kr_max; break;
      case CNT_REFINE: val = (unsigned long long)rf_sum; break;
      case CNT_REFINE_MAX: val = (unsigned long long)rf_max; break;
      case CNT_SOLVES: val = (unsigned long long)a.nsteps; break;
      case CNT_WORK: val = (unsigned long long)kr_sum * npts; break;
      case CNT_DOFSTEPS: val = (unsigned long long)a.nsteps * npts; break;
      default: break;
    }
    if (t == CNT_KRYLOV_MAX || t == CNT_REFINE_MAX) {
      if (MIXED || t == CNT_KRYLOV_MAX) atomicMax(&a.counters[t], val);
    } else if (val != 0) {
      atomicAdd(&a.counters[t], val);
    }
  }
  if (threadIdx.x == 0 && flag && a.status) atomicOr(a.status, flag);

  if (a.fin.base) {
    double* dst = vec_at(a.fin, a.fin.a * q + a.fin.b, a.slen, off);
    if (a.target.base) {
      double rr[1] = {0.0};
      if constexpr (RES) {  // v holds the exact residual already
#pragma unroll
        for (int k = 0; k < K; ++k) rr[0] += v[k] * v[k];
      } else {
        double tg[K];
        gload<K>(L, vec_at(a.target, a.target.a * q + a.target.b, a.slen, off), tg);
#pragma unroll
        for (int k = 0; k < K; ++k) {
          v[k] = (k < L.nval) ? v[k] - tg[k] : 0.0;
          rr[0] += v[k] * v[k];
        }
      }
      gstore<K>(L, dst, v);
      block_sum<W, 1, double>(rr, ring);
      if (RES) rr[0] = rr[0] > res_max ? rr[0] : res_max;
      if (threadIdx.x == 0 && a.res2) a.res2[blockIdx.x] = rr[0];
    } else {
      gstore<K>(L, dst, v);
    }
  }

}

template <int OPC, int SOLVER>
hipError_t launch_chain_t(bool mixed, int shape, const ChainArgs& a, int ntasks, size_t smem,
                          int tabmax, hipStream_t s) {
  if (ntasks <= 0) return hipSuccess;
  // the manufactured forcing exists for the heat operator only, and residual
  // mode does not combine with it; residual mode runs in both precisions
  const bool forced = (OPC == OPC_HEAT) && a.fkind;
  constexpr int kF = (OPC == OPC_HEAT) ? MODE_FORCED : MODE_PLAIN;
  if (a.resmode && forced) return hipErrorInvalidValue;
#define CTM_CASE(IDX, W, K)                                                                  \
  case IDX:                                                                                  \
    if (a.resmode) {                                                                         \
      if (mixed)                                                                             \
        hipLaunchKernelGGL((chain_kernel<OPC, SOLVER, true, MODE_RESIDUAL, W, K>),           \
                           dim3(ntasks), dim3(64 * W), smem, s, a, tabmax);                  \
      else                                                                                   \
        hipLaunchKernelGGL((chain_kernel<OPC, SOLVER, false, MODE_RESIDUAL, W, K>),          \
                           dim3(ntasks), dim3(64 * W), smem, s, a, tabmax);                  \
    } else if (forced) {                                                                     \
      if (mixed)                                                                             \
        hipLaunchKernelGGL((chain_kernel<OPC, SOLVER, true, kF, W, K>), dim3(ntasks),        \
                           dim3(64 * W), smem, s, a, tabmax);                                \
      else                                                                                   \
        hipLaunchKernelGGL((chain_kernel<OPC, SOLVER, false, kF, W, K>), dim3(ntasks),       \
                           dim3(64 * W), smem, s, a, tabmax);                                \
    } else if (mixed) {                                                                      \
      hipLaunchKernelGGL((chain_kernel<OPC, SOLVER, true, MODE_PLAIN, W, K>), dim3(ntasks),  \
                         dim3(64 * W), smem, s, a, tabmax);                                  \
    } else {                                                                                 \
      hipLaunchKernelGGL((chain_kernel<OPC, SOLVER, false, MODE_PLAIN, W, K>), dim3(ntasks), \
                         dim3(64 * W), smem, s, a, tabmax);                                  \
    }                                                                                        \
    break;
  switch (shape) {
    CTM_CASE(0, 1, 4)
    CTM_CASE(1, 2, 4)
    CTM_CASE(2, 4, 4)
    CTM_CASE(3, 8, 4)
    CTM_CASE(4, 16, 4)
    CTM_CASE(5, 1, 8)
    CTM_CASE(6, 2, 8)
    CTM_CASE(7, 4, 8)
    CTM_CASE(8, 8, 8)
    CTM_CASE(9, 16, 8)
    default:
      return hipErrorInvalidValue;
  }
#undef CTM_CASE
  return hipGetLastError();
}

}  // namespace ctm
