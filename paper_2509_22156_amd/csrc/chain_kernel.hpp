// The batched implicit-step kernel ("chain"): one work-group per task
// (component grid g, time interval q). A task loads its start vector into
// registers and applies `nsteps` backward-Euler steps v <- Phi(v) + f_j, each
// solved matrix-free by CG or BiCGStab with all vectors held on chip
// (registers for the thread's own points, one LDS copy of the vector the
// stencil reads). This single kernel carries every time-stepping phase:
// MGRIT F-, C- and FC-relaxation, the C-point residual, the sequential
// coarse-level solve and plain time-sequential stepping; they differ only
// in which vectors are read and written (see ChainArgs).
//
// Precision: FP64, or mixed: FP64 iterative refinement of each implicit
// step (FP64 residual b - A x), with the correction solved by FP32 Krylov.
#pragma once

#include "device_common.hpp"

namespace ctm {

enum { FLAG_NOCONV = 1 << CTM_ERR_NOCONV, FLAG_BREAKDOWN = 1 << CTM_ERR_BREAKDOWN,
       FLAG_NONFINITE = 1 << CTM_ERR_NONFINITE };

template <typename T>
__device__ __forceinline__ bool finite_val(T v) {
  return v == v && v - v == (T)0;
}

// Unpreconditioned CG (Section 4.1, symmetric operators) on the work-group.
// x holds the initial guess; stops when ||b - A x||_2^2 <= tol2 * bb on the
// recursively updated residual. Returns the iteration count; *flag gets
// FLAG_NOCONV / FLAG_NONFINITE on failure.
template <int OPC, typename T, int W, int K>
__device__ __forceinline__ int krylov_cg(const GridDev& g, const Pts<K>& P,
                                         const Stencil<OPC, T, K>& S, const T* tab, T* xl,
                                         RedRing& ring, T (&x)[K], const T (&b)[K], T bb,
                                         T tol2, int maxit, int* flag) {
  T r[K], p[K], q[K];
#pragma unroll
  for (int k = 0; k < K; ++k)
    if (P.p[k] >= 0) xl[P.p[k]] = x[k];
  __syncthreads();
  stencil_apply<OPC, T, K>(g, P, S, tab, xl, x, q);
  T s1[1] = {(T)0};
#pragma unroll
  for (int k = 0; k < K; ++k) {
    r[k] = b[k] - q[k];
    p[k] = r[k];
    s1[0] += r[k] * r[k];
  }
  block_sum<W, 1, T>(s1, ring);
  T rr = s1[0];
  if (!finite_val(rr)) {
    *flag |= FLAG_NONFINITE;
    return 0;
  }
  if (rr <= tol2 * bb) return 0;
  for (int it = 1; it <= maxit; ++it) {
#pragma unroll
    for (int k = 0; k < K; ++k)
      if (P.p[k] >= 0) xl[P.p[k]] = p[k];
    __syncthreads();
    stencil_apply<OPC, T, K>(g, P, S, tab, xl, p, q);
    T s2[1] = {(T)0};
#pragma unroll
    for (int k = 0; k < K; ++k) s2[0] += p[k] * q[k];
    block_sum<W, 1, T>(s2, ring);
    const T alpha = rr / s2[0];
    T s3[1] = {(T)0};
#pragma unroll
    for (int k = 0; k < K; ++k) {
      x[k] += alpha * p[k];
      r[k] -= alpha * q[k];
      s3[0] += r[k] * r[k];
    }
    block_sum<W, 1, T>(s3, ring);
    const T rn = s3[0];
    if (!finite_val(rn)) {
      *flag |= FLAG_NONFINITE;
      return it;
    }
    if (rn <= tol2 * bb) return it;
    const T beta = rn / rr;
    rr = rn;
#pragma unroll
    for (int k = 0; k < K; ++k) p[k] = r[k] + beta * p[k];
  }
  *flag |= FLAG_NOCONV;
  return maxit;
}

// Unpreconditioned BiCGStab (van der Vorst; Section 4.1, non-symmetric
// operators), shadow residual r^ = r_0.
template <int OPC, typename T, int W, int K>
__device__ __forceinline__ int krylov_bicgstab(const GridDev& g, const Pts<K>& P,
                                               const Stencil<OPC, T, K>& S, const T* tab, T* xl,
                                               RedRing& ring, T (&x)[K], const T (&b)[K],
                                               T bb, T tol2, int maxit, int* flag) {
  T r[K], rh[K], p[K], v[K], s[K], t[K];
#pragma unroll
  for (int k = 0; k < K; ++k)
    if (P.p[k] >= 0) xl[P.p[k]] = x[k];
  __syncthreads();
  stencil_apply<OPC, T, K>(g, P, S, tab, xl, x, v);
  T s1[1] = {(T)0};
#pragma unroll
  for (int k = 0; k < K; ++k) {
    r[k] = b[k] - v[k];
    rh[k] = r[k];
    p[k] = r[k];
    s1[0] += r[k] * r[k];
  }
  block_sum<W, 1, T>(s1, ring);
  T rr = s1[0];
  if (!finite_val(rr)) {
    *flag |= FLAG_NONFINITE;
    return 0;
  }
  if (rr <= tol2 * bb) return 0;
  T rho = rr;
  for (int it = 1; it <= maxit; ++it) {
#pragma unroll
    for (int k = 0; k < K; ++k)
      if (P.p[k] >= 0) xl[P.p[k]] = p[k];
    __syncthreads();
    stencil_apply<OPC, T, K>(g, P, S, tab, xl, p, v);
    T s2[1] = {(T)0};
#pragma unroll
    for (int k = 0; k < K; ++k) s2[0] += rh[k] * v[k];
    block_sum<W, 1, T>(s2, ring);
    if (s2[0] == (T)0 || !finite_val(s2[0])) {
      *flag |= finite_val(s2[0]) ? FLAG_BREAKDOWN : FLAG_NONFINITE;
      return it;
    }
    const T alpha = rho / s2[0];
#pragma unroll
    for (int k = 0; k < K; ++k) s[k] = r[k] - alpha * v[k];
#pragma unroll
    for (int k = 0; k < K; ++k)
      if (P.p[k] >= 0) xl[P.p[k]] = s[k];
    __syncthreads();
    stencil_apply<OPC, T, K>(g, P, S, tab, xl, s, t);
    T s3[3] = {(T)0, (T)0, (T)0};
#pragma unroll
    for (int k = 0; k < K; ++k) {
      s3[0] += t[k] * s[k];
      s3[1] += t[k] * t[k];
      s3[2] += s[k] * s[k];
    }
    block_sum<W, 3, T>(s3, ring);
    if (s3[2] <= tol2 * bb) {
#pragma unroll
      for (int k = 0; k < K; ++k) x[k] += alpha * p[k];
      return it;
    }
    if (s3[1] == (T)0 || !finite_val(s3[1])) {
      *flag |= finite_val(s3[1]) ? FLAG_BREAKDOWN : FLAG_NONFINITE;
      return it;
    }
    const T omega = s3[0] / s3[1];
    T s4[2] = {(T)0, (T)0};
#pragma unroll
    for (int k = 0; k < K; ++k) {
      x[k] += alpha * p[k] + omega * s[k];
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
    const T beta = (s4[1] / rho) * (alpha / omega);
    rho = s4[1];
#pragma unroll
    for (int k = 0; k < K; ++k) p[k] = r[k] + beta * (p[k] - omega * v[k]);
  }
  *flag |= FLAG_NOCONV;
  return maxit;
}

template <int OPC, int SOLVER, typename T, int W, int K>
__device__ __forceinline__ int krylov(const GridDev& g, const Pts<K>& P,
                                      const Stencil<OPC, T, K>& S, const T* tab, T* xl,
                                      RedRing& ring, T (&x)[K], const T (&b)[K], T bb, T tol2,
                                      int maxit, int* flag) {
  if constexpr (SOLVER == SOLV_CG)
    return krylov_cg<OPC, T, W, K>(g, P, S, tab, xl, ring, x, b, bb, tol2, maxit, flag);
  else
    return krylov_bicgstab<OPC, T, W, K>(g, P, S, tab, xl, ring, x, b, bb, tol2, maxit, flag);
}

__device__ __forceinline__ double* vec_at(const VecRef& r, long long idx, long long slen,
                                          long long off) {
  return r.base + idx * slen + off;
}

template <int OPC, int SOLVER, bool MIXED, int W, int K>
__global__ void __launch_bounds__(64 * W) chain_kernel(ChainArgs a, int tabmax) {
  constexpr int BS = 64 * W;
  constexpr int CAP = BS * K;
  extern __shared__ __align__(16) unsigned char smem[];
  double* xl64 = reinterpret_cast<double*>(smem);
  float* xl32 = reinterpret_cast<float*>(smem);
  double* tl64 = reinterpret_cast<double*>(smem + CAP * sizeof(double));
  float* tl32 = reinterpret_cast<float*>(tl64 + tabmax);
  const size_t tab_bytes =
      (size_t)tabmax * sizeof(double) + (MIXED ? (size_t)tabmax * sizeof(float) : 0);
  double* red = reinterpret_cast<double*>(smem + CAP * sizeof(double) +
                                          ((tab_bytes + 15) & ~size_t(15)));
  __shared__ GridDev gs;

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

  Pts<K> P;
  setup_points<BS, K>(g, P);
  Stencil<OPC, double, K> S64;
  stencil_setup<OPC, double, K>(g, P, a.dt, a.amp, tl64, S64);
  Stencil<OPC, float, K> S32;
  if constexpr (MIXED) stencil_setup<OPC, float, K>(g, P, a.dt, a.amp, tl32, S32);

  const long long off = g.off;
  double v[K];
  if (a.start.base) {
    const double* src = vec_at(a.start, a.start.a * q + a.start.b, a.slen, off);
#pragma unroll
    for (int k = 0; k < K; ++k) v[k] = (P.p[k] >= 0) ? src[P.p[k]] : 0.0;
  } else {
#pragma unroll
    for (int k = 0; k < K; ++k) v[k] = 0.0;
  }
  if (a.start_wb.base) {
    double* dst = vec_at(a.start_wb, a.start_wb.a * q + a.start_wb.b, a.slen, off);
#pragma unroll
    for (int k = 0; k < K; ++k)
      if (P.p[k] >= 0) dst[P.p[k]] = v[k];
  }

  RedRing ring{red, 0};
  int flag = 0;
  long long kr_sum = 0, kr_max = 0, rf_sum = 0, rf_max = 0;
  const double tol2 = a.tol * a.tol;

  for (int j = 1; j <= a.nsteps; ++j) {
    double bbv[1] = {0.0};
#pragma unroll
    for (int k = 0; k < K; ++k) bbv[0] += v[k] * v[k];
    block_sum<W, 1, double>(bbv, ring);
    const double bb = bbv[0];
    double x[K];
    if (!finite_val(bb)) {
      flag |= FLAG_NONFINITE;
#pragma unroll
      for (int k = 0; k < K; ++k) x[k] = v[k];
    } else if (bb == 0.0) {
#pragma unroll
      for (int k = 0; k < K; ++k) x[k] = 0.0;
    } else if constexpr (!MIXED) {
#pragma unroll
      for (int k = 0; k < K; ++k) x[k] = v[k];
      const int it = krylov<OPC, SOLVER, double, W, K>(g, P, S64, tl64, xl64, ring, x, v,
                                                       bb, tol2, a.maxit, &flag);
      kr_sum += it;
      kr_max = it > kr_max ? it : kr_max;
    } else {
      // FP64 iterative refinement around an FP32 Krylov correction solve
#pragma unroll
      for (int k = 0; k < K; ++k) x[k] = v[k];
      const float itol2 = (float)(a.inner_tol * a.inner_tol);
      bool conv = false;
      int sweeps = 0, its = 0;
      for (; sweeps <= a.refine_maxit; ++sweeps) {
        double rq[K];
#pragma unroll
        for (int k = 0; k < K; ++k)
          if (P.p[k] >= 0) xl64[P.p[k]] = x[k];
        __syncthreads();
        stencil_apply<OPC, double, K>(g, P, S64, tl64, xl64, x, rq);
        double rr[1] = {0.0};
#pragma unroll
        for (int k = 0; k < K; ++k) {
          rq[k] = v[k] - rq[k];
          rr[0] += rq[k] * rq[k];
        }
        block_sum<W, 1, double>(rr, ring);
        if (!finite_val(rr[0])) {
          flag |= FLAG_NONFINITE;
          break;
        }
        if (rr[0] <= tol2 * bb) {
          conv = true;
          break;
        }
        if (sweeps == a.refine_maxit) break;
        const double nr = sqrt(rr[0]);
        const double inv = 1.0 / nr;
        float r32[K], d32[K];
        float bb32 = 0.0f;
#pragma unroll
        for (int k = 0; k < K; ++k) {
          r32[k] = (float)(rq[k] * inv);
          d32[k] = 0.0f;
          bb32 += r32[k] * r32[k];
        }
        float bbs[1] = {bb32};
        block_sum<W, 1, float>(bbs, ring);
        int iflag = 0;
        const int it = krylov<OPC, SOLVER, float, W, K>(g, P, S32, tl32, xl32, ring, d32,
                                                        r32, bbs[0], itol2, a.maxit, &iflag);
        its += it;
        if (iflag & FLAG_NONFINITE) {
          flag |= FLAG_NONFINITE;
          break;
        }
#pragma unroll
        for (int k = 0; k < K; ++k) x[k] += nr * (double)d32[k];
      }
      if (!conv) flag |= FLAG_NOCONV;
      kr_sum += its;
      kr_max = its > kr_max ? its : kr_max;
      rf_sum += sweeps;
      rf_max = sweeps > rf_max ? sweeps : rf_max;
    }
    if (a.forcing.base) {
      const double* f = vec_at(a.forcing, a.forcing.a * q + a.forcing.b + j, a.slen, off);
#pragma unroll
      for (int k = 0; k < K; ++k) v[k] = x[k] + ((P.p[k] >= 0) ? f[P.p[k]] : 0.0);
    } else {
#pragma unroll
      for (int k = 0; k < K; ++k) v[k] = x[k];
    }
    if (a.inter.base && j < a.nsteps) {
      double* dst = vec_at(a.inter, a.inter.a * q + a.inter.b + j, a.slen, off);
#pragma unroll
      for (int k = 0; k < K; ++k)
        if (P.p[k] >= 0) dst[P.p[k]] = v[k];
    }
  }

  if (a.fin.base) {
    double* dst = vec_at(a.fin, a.fin.a * q + a.fin.b, a.slen, off);
    if (a.target.base) {
      const double* tg = vec_at(a.target, a.target.a * q + a.target.b, a.slen, off);
      double rr[1] = {0.0};
#pragma unroll
      for (int k = 0; k < K; ++k) {
        if (P.p[k] >= 0) {
          const double r = v[k] - tg[P.p[k]];
          dst[P.p[k]] = r;
          rr[0] += r * r;
        }
      }
      block_sum<W, 1, double>(rr, ring);
      if (threadIdx.x == 0 && a.res2) a.res2[blockIdx.x] = rr[0];
    } else {
#pragma unroll
      for (int k = 0; k < K; ++k)
        if (P.p[k] >= 0) dst[P.p[k]] = v[k];
    }
  }

  if (threadIdx.x == 0) {
    if (a.counters) {
      atomicAdd(&a.counters[CNT_KRYLOV], (unsigned long long)kr_sum);
      atomicMax(&a.counters[CNT_KRYLOV_MAX], (unsigned long long)kr_max);
      atomicAdd(&a.counters[CNT_REFINE], (unsigned long long)rf_sum);
      atomicMax(&a.counters[CNT_REFINE_MAX], (unsigned long long)rf_max);
      atomicAdd(&a.counters[CNT_SOLVES], (unsigned long long)a.nsteps);
      atomicAdd(&a.counters[CNT_WORK], (unsigned long long)kr_sum * (unsigned long long)g.npts);
    }
    if (flag && a.status) atomicOr(a.status, flag);
  }
}

template <int OPC, int SOLVER>
hipError_t launch_chain_t(bool mixed, int shape, const ChainArgs& a, int ntasks, size_t smem,
                          int tabmax, hipStream_t s) {
  if (ntasks <= 0) return hipSuccess;
#define CTM_CASE(IDX, W, K)                                                                   \
  case IDX:                                                                                   \
    if (mixed)                                                                                \
      hipLaunchKernelGGL((chain_kernel<OPC, SOLVER, true, W, K>), dim3(ntasks), dim3(64 * W), \
                         smem, s, a, tabmax);                                                 \
    else                                                                                      \
      hipLaunchKernelGGL((chain_kernel<OPC, SOLVER, false, W, K>), dim3(ntasks),              \
                         dim3(64 * W), smem, s, a, tabmax);                                   \
    break;
  switch (shape) {
    CTM_CASE(0, 1, 1)
    CTM_CASE(1, 1, 2)
    CTM_CASE(2, 1, 4)
    CTM_CASE(3, 2, 4)
    CTM_CASE(4, 4, 4)
    CTM_CASE(5, 4, 8)
    CTM_CASE(6, 8, 8)
    CTM_CASE(7, 16, 8)
    default:
      return hipErrorInvalidValue;
  }
#undef CTM_CASE
  return hipGetLastError();
}

}  // namespace ctm
