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

// Status bits a solver kernel ORs into ChainArgs::status.
enum { FLAG_NOCONV = 1 << CTM_ERR_NOCONV, FLAG_BREAKDOWN = 1 << CTM_ERR_BREAKDOWN,
       FLAG_NONFINITE = 1 << CTM_ERR_NONFINITE,
       FLAG_INVALID = 1 << CTM_ERR_INVALID };

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
