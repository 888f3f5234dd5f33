// Device helpers shared by the kernels: wave64 reductions, point decoding
// and the (2d+1)-point stencils of the system matrix I + dt L_l.
#pragma once

#include "ctm_internal.h"

namespace ctm {

// ---------------------------------------------------------------- reductions
// DPP moves within a row of 16 lanes; quad_perm and row rotations only, so
// every source lane is valid.
template <int CTRL>
__device__ __forceinline__ unsigned dpp32(unsigned v) {
  return (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, CTRL, 0xF, 0xF, false);
}
template <int CTRL>
__device__ __forceinline__ float dpp(float v) {
  return __builtin_bit_cast(float, dpp32<CTRL>(__builtin_bit_cast(unsigned, v)));
}
template <int CTRL>
__device__ __forceinline__ double dpp(double v) {
  const uint64_t u = __builtin_bit_cast(uint64_t, v);
  const unsigned lo = dpp32<CTRL>((unsigned)u);
  const unsigned hi = dpp32<CTRL>((unsigned)(u >> 32));
  return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}
__device__ __forceinline__ float readlane(float v, int l) {
  return __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), l));
}
__device__ __forceinline__ double readlane(double v, int l) {
  const uint64_t u = __builtin_bit_cast(uint64_t, v);
  const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)u, l);
  const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(u >> 32), l);
  return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}

// DPP move with a row mask: rows outside `ROWMASK` receive 0.
template <int CTRL, int ROWMASK>
__device__ __forceinline__ unsigned dpp32m(unsigned v) {
  return (unsigned)__builtin_amdgcn_update_dpp(0, (int)v, CTRL, ROWMASK, 0xF, false);
}
template <int CTRL, int ROWMASK>
__device__ __forceinline__ float dppm(float v) {
  return __builtin_bit_cast(float, dpp32m<CTRL, ROWMASK>(__builtin_bit_cast(unsigned, v)));
}
template <int CTRL, int ROWMASK>
__device__ __forceinline__ double dppm(double v) {
  const uint64_t u = __builtin_bit_cast(uint64_t, v);
  const unsigned lo = dpp32m<CTRL, ROWMASK>((unsigned)u);
  const unsigned hi = dpp32m<CTRL, ROWMASK>((unsigned)(u >> 32));
  return __builtin_bit_cast(double, ((uint64_t)hi << 32) | lo);
}

// Sum over the 64 lanes of a wave; every lane gets the same value. Row sums
// by quad permutes and row rotations, then the row broadcasts add row 0 into
// row 1, row 2 into row 3 and rows 0-1 into row 3; lane 63 holds the total.
template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
  v += dpp<0xB1>(v);   // quad_perm [1,0,3,2]
  v += dpp<0x4E>(v);   // quad_perm [2,3,0,1]
  v += dpp<0x124>(v);  // row_ror:4
  v += dpp<0x128>(v);  // row_ror:8
  v += dppm<0x142, 0xA>(v);  // row_bcast:15 into rows 1 and 3
  v += dppm<0x143, 0xC>(v);  // row_bcast:31 into rows 2 and 3
  return readlane(v, 63);
}

// Two LDS slot arrays for cross-wave sums, used strictly alternately: the
// barrier of every call then separates a slot's reads from its next writes.
struct RedRing {
  double* base;  // 2 * 64 doubles
  int phase;
};

// Sum of NV (<= 4) values over the work-group of W (<= 16) waves; every
// thread gets the same result (partials added in wave order).
template <int W, int NV, typename T>
__device__ __forceinline__ void block_sum(T (&v)[NV], RedRing& ring) {
#pragma unroll
  for (int i = 0; i < NV; ++i) v[i] = wave_sum(v[i]);
  if constexpr (W > 1) {
    T* slots = reinterpret_cast<T*>(ring.base + (ring.phase & 1) * 64);
    ring.phase ^= 1;
    const int wave = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
#pragma unroll
      for (int i = 0; i < NV; ++i) slots[i * W + wave] = v[i];
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < NV; ++i) {
      T s = slots[i * W];
#pragma unroll
      for (int w = 1; w < W; ++w) s += slots[i * W + w];
      v[i] = s;
    }
  }
}

// ------------------------------------------------------------- point layout
// Each thread owns the points p = threadIdx.x + k * 64W, k < K (strided, so
// a wave touches consecutive points: coalesced global and conflict-free LDS
// access). Coordinates are packed into one word; mk holds the neighbour
// flags: bit 2i = has a lower neighbour on axis i, bit 2i+1 = upper.
template <int K>
struct Pts {
  int p[K];
  unsigned cw[K];
  unsigned mk[K];
};

template <int BS, int K>
__device__ __forceinline__ void setup_points(const GridDev& g, Pts<K>& P) {
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const int p = (int)threadIdx.x + k * BS;
    unsigned cw = 0, mk = 0;
    if (p < g.npts) {
      int rem = p;
#pragma unroll
      for (int i = MAXD - 1; i >= 0; --i) {
        if (i < g.d) {
          const int n = g.n[i];
          const int j = rem % n;
          rem /= n;
          cw |= (unsigned)j << g.boff[i];
          mk |= (unsigned)(j > 0) << (2 * i);
          mk |= (unsigned)(j < n - 1) << (2 * i + 1);
        }
      }
      P.p[k] = p;
    } else {
      P.p[k] = -1;
    }
    P.cw[k] = cw;
    P.mk[k] = mk;
  }
}

__device__ __forceinline__ int coord_of(const GridDev& g, unsigned cw, int i) {
  return (int)((cw >> g.boff[i]) & (unsigned)g.bmask[i]);
}

// --------------------------------------------------------------- stencils
// Per-chain constants of the system matrix A = I + dt L_l in precision T.
//  HEAT: A x = (1 + 2 dt sum_i h_i^-2) x_p - sum_i dt h_i^-2 (x_{p-e_i} + x_{p+e_i})
//  SEP:  A x = (1 + sum_i dt D_i[j_i]) x_p + sum_i dt (Lo_i[j_i] x_{p-e_i} + Up_i[j_i] x_{p+e_i})
//        with the 1-D tables (Lo, D, Up) of L, held in LDS already scaled by dt
//  VAR:  A x = x_p + sum_i dt h_i^-2 (a_up (x_p - x_{p+e_i}) + a_dn (x_p - x_{p-e_i})),
//        a = 1 + amp sm_i[face] prod_{k != i} sn_k[j_k] from LDS sine tables
// Missing neighbours (boundary ghosts) contribute zero.
template <int OPC, typename T, int K>
struct Stencil {
  T diag;        // HEAT
  T c[MAXD];     // HEAT, VAR: dt / h_i^2
  T amp;         // VAR
  T sdiag[K];    // SEP: per-point diagonal
};

template <int OPC, typename T, int K>
__device__ __forceinline__ void stencil_setup(const GridDev& g, const Pts<K>& P, double dt,
                                              double amp, const T* tab, Stencil<OPC, T, K>& S) {
  double s = 0.0;
#pragma unroll
  for (int i = 0; i < MAXD; ++i) {
    const double ci = (i < g.d) ? dt * g.ih2[i] : 0.0;
    S.c[i] = (T)ci;
    s += 2.0 * ci;
  }
  S.diag = (T)(1.0 + s);
  S.amp = (T)amp;
  if constexpr (OPC == OPC_SEP) {
#pragma unroll
    for (int k = 0; k < K; ++k) {
      T acc = (T)1;
#pragma unroll
      for (int i = 0; i < MAXD; ++i) {
        if (i < g.d && P.p[k] >= 0) {
          const int j = coord_of(g, P.cw[k], i);
          acc += tab[g.tab[i] + g.n[i] + j];
        }
      }
      S.sdiag[k] = acc;
    }
  }
}

// y = A x for the thread's points; xl is x in LDS (all points of the grid).
template <int OPC, typename T, int K>
__device__ __forceinline__ void stencil_apply(const GridDev& g, const Pts<K>& P,
                                              const Stencil<OPC, T, K>& S, const T* tab,
                                              const T* xl, const T (&x)[K], T (&y)[K]) {
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const int p = P.p[k];
    if (p < 0) {
      y[k] = (T)0;
      continue;
    }
    const unsigned mk = P.mk[k];
    const T xs = x[k];
    if constexpr (OPC == OPC_HEAT) {
      T acc = S.diag * xs;
#pragma unroll
      for (int i = 0; i < MAXD; ++i) {
        if (i < g.d) {
          const int st = g.stride[i];
          const bool lo = (mk >> (2 * i)) & 1u;
          const bool hi = (mk >> (2 * i + 1)) & 1u;
          T xm = xl[lo ? p - st : p];
          T xp = xl[hi ? p + st : p];
          xm = lo ? xm : (T)0;
          xp = hi ? xp : (T)0;
          acc -= S.c[i] * (xm + xp);
        }
      }
      y[k] = acc;
    } else if constexpr (OPC == OPC_SEP) {
      T acc = S.sdiag[k] * xs;
#pragma unroll
      for (int i = 0; i < MAXD; ++i) {
        if (i < g.d) {
          const int st = g.stride[i];
          const int j = coord_of(g, P.cw[k], i);
          const T* t = tab + g.tab[i];
          const bool lo = (mk >> (2 * i)) & 1u;
          const bool hi = (mk >> (2 * i + 1)) & 1u;
          T xm = xl[lo ? p - st : p];
          T xp = xl[hi ? p + st : p];
          xm = lo ? xm : (T)0;
          xp = hi ? xp : (T)0;
          acc += t[j] * xm + t[2 * g.n[i] + j] * xp;
        }
      }
      y[k] = acc;
    } else {
      // products of the node sines of all axes but i, by prefix/suffix products
      T sn[MAXD];
#pragma unroll
      for (int i = 0; i < MAXD; ++i)
        sn[i] = (i < g.d) ? tab[g.tab[i] + coord_of(g, P.cw[k], i)] : (T)1;
      T pre[MAXD], suf[MAXD];
      T run = (T)1;
#pragma unroll
      for (int i = 0; i < MAXD; ++i) {
        pre[i] = run;
        run *= sn[i];
      }
      run = (T)1;
#pragma unroll
      for (int i = MAXD - 1; i >= 0; --i) {
        suf[i] = run;
        run *= sn[i];
      }
      T acc = xs;
#pragma unroll
      for (int i = 0; i < MAXD; ++i) {
        if (i < g.d) {
          const int st = g.stride[i];
          const int j = coord_of(g, P.cw[k], i);
          const T* sm = tab + g.tab[i] + g.n[i];
          const T e = pre[i] * suf[i];
          const T a_dn = (T)1 + S.amp * sm[j] * e;
          const T a_up = (T)1 + S.amp * sm[j + 1] * e;
          const bool lo = (mk >> (2 * i)) & 1u;
          const bool hi = (mk >> (2 * i + 1)) & 1u;
          T xm = xl[lo ? p - st : p];
          T xp = xl[hi ? p + st : p];
          xm = lo ? xm : (T)0;
          xp = hi ? xp : (T)0;
          acc += S.c[i] * (a_up * (xs - xp) + a_dn * (xs - xm));
        }
      }
      y[k] = acc;
    }
  }
}

// Copy the grid's coefficient tables into LDS in precision T. SEP tables are
// coefficients of L and are scaled by dt here; VAR tables are sines.
template <int OPC, typename T, int BS>
__device__ __forceinline__ void load_tables(const GridDev& g, const double* tab64, double dt,
                                            T* tl) {
  if constexpr (OPC == OPC_HEAT) return;
  const double scale = (OPC == OPC_SEP) ? dt : 1.0;
  for (int t = threadIdx.x; t < g.tabsz; t += BS) tl[t] = (T)(tab64[g.tab0 + t] * scale);
}

}  // namespace ctm
