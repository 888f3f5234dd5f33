// Auxiliary kernels: initial value sampling, standalone stencil apply,
// combination gather / combine-then-project, norms and vector updates of
// the MGRIT driver, and the dispatch of the chain kernel instantiations.
#include <algorithm>

#include "line_layout.hpp"
#include "manufactured.hpp"

namespace ctm {

hipError_t launch_chain_heat_cg(bool, int, const ChainArgs&, int, size_t, int, hipStream_t);
hipError_t launch_chain_heat_bicg(bool, int, const ChainArgs&, int, size_t, int, hipStream_t);
hipError_t launch_chain_sep_bicg(bool, int, const ChainArgs&, int, size_t, int, hipStream_t);
hipError_t launch_chain_var_cg(bool, int, const ChainArgs&, int, size_t, int, hipStream_t);
hipError_t launch_chain_var_bicg(bool, int, const ChainArgs&, int, size_t, int, hipStream_t);
hipError_t launch_chain_drift_bicg(bool, int, const ChainArgs&, int, size_t, int, hipStream_t);

hipError_t launch_chain(int opc, int solver, bool mixed, int shape, const ChainArgs& a,
                        int ntasks, size_t smem, int tabmax, hipStream_t s) {
  if (opc == OPC_HEAT && solver == SOLV_CG)
    return launch_chain_heat_cg(mixed, shape, a, ntasks, smem, tabmax, s);
  if (opc == OPC_HEAT && solver == SOLV_BICG)
    return launch_chain_heat_bicg(mixed, shape, a, ntasks, smem, tabmax, s);
  if (opc == OPC_SEP && solver == SOLV_BICG)
    return launch_chain_sep_bicg(mixed, shape, a, ntasks, smem, tabmax, s);
  if (opc == OPC_VAR && solver == SOLV_CG)
    return launch_chain_var_cg(mixed, shape, a, ntasks, smem, tabmax, s);
  if (opc == OPC_VAR && solver == SOLV_BICG)
    return launch_chain_var_bicg(mixed, shape, a, ntasks, smem, tabmax, s);
  if (opc == OPC_DRIFT && solver == SOLV_BICG)
    return launch_chain_drift_bicg(mixed, shape, a, ntasks, smem, tabmax, s);
  return hipErrorInvalidValue;
}

// ------------------------------------------------------------ initial value
// u0 at the unknowns of grid blockIdx.y: sum_r w_r prod_i F[r][i][J_i], with
// J_i = (j_i + j0) 2^{n - l_i} the index of the node on the finest 1-D grid.
__global__ void initial_state_kernel(const GridDev* __restrict__ grids, int nlev, int terms,
                                     const double* __restrict__ icw,
                                     const double* __restrict__ icf, double* __restrict__ out) {
  const GridDev& g = grids[blockIdx.y];
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= g.npts) return;
  const int F = (1 << nlev) + 1;
  int J[MAXD];
  int rem = p;
#pragma unroll
  for (int i = MAXD - 1; i >= 0; --i) {
    J[i] = 0;
    if (i < g.d) {
      const int j = rem % g.n[i];
      rem /= g.n[i];
      J[i] = (j + g.j0) << (nlev - g.lev[i]);
    }
  }
  double u = 0.0;
  for (int r = 0; r < terms; ++r) {
    double t = icw[r];
#pragma unroll
    for (int i = 0; i < MAXD; ++i)
      if (i < g.d) t *= icf[((size_t)r * g.d + i) * F + J[i]];
    u += t;
  }
  out[g.off + p] = u;
}

hipError_t launch_initial_state(const GridDev* grids, int G, int maxpts, int nlev, int terms,
                                const double* icw, const double* icf, double* out,
                                hipStream_t s) {
  dim3 grid((maxpts + 255) / 256, G);
  hipLaunchKernelGGL(initial_state_kernel, grid, dim3(256), 0, s, grids, nlev, terms, icw, icf,
                     out);
  return hipGetLastError();
}

__global__ void mms_initial_kernel(const GridDev* __restrict__ grids, double t,
                                   double* __restrict__ out) {
  const GridDev& g = grids[blockIdx.y];
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= g.npts) return;
  double x[MAXD];
  int rem = p;
  for (int i = g.d - 1; i >= 0; --i) {
    const int j = rem % g.n[i];
    rem /= g.n[i];
    x[i] = g.lo[i] + (double)(j + g.j0) * g.h[i];
  }
  out[g.off + p] = mms_exact(x, g.d, t);
}

hipError_t launch_mms_initial(const GridDev* grids, int G, int maxpts, double t, double* out,
                              hipStream_t s) {
  dim3 grid((maxpts + 255) / 256, G);
  hipLaunchKernelGGL(mms_initial_kernel, grid, dim3(256), 0, s, grids, t, out);
  return hipGetLastError();
}

// ---------------------------------------------------------- stencil apply
// y = (I + dt L_l) x on every grid, one work-group per grid, FP64, in the
// same line layout and with the same device stencil the solvers use.
template <int OPC, int W, int K>
__global__ void __launch_bounds__(64 * W)
    apply_kernel(const GridDev* __restrict__ grids, const double* __restrict__ tab64, double amp,
                 double dt, const double* __restrict__ x, double* __restrict__ y,
                 int tabmax) {
  constexpr int BS = 64 * W;
  extern __shared__ __align__(16) unsigned char smem[];
  const ChainSmem lay = chain_smem_layout(W, K, tabmax, false, OPC == OPC_HEAT, -1);
  double* xl = reinterpret_cast<double*>(smem);
  double* tl = reinterpret_cast<double*>(smem + lay.tab);
  HeatTab<double, K>* ht = reinterpret_cast<HeatTab<double, K>*>(smem + lay.heat);
  __shared__ GridDev gs;
  lds_zero_ghosts<double, K>(xl);
  {
    const int* src = reinterpret_cast<const int*>(grids + blockIdx.x);
    int* dst = reinterpret_cast<int*>(&gs);
    for (int t = threadIdx.x; t < (int)(sizeof(GridDev) / sizeof(int)); t += BS) dst[t] = src[t];
  }
  __syncthreads();
  const GridDev& g = gs;
  load_tables<OPC, double, BS>(g, tab64, dt, tl);
  __syncthreads();
  Lane<K> L;
  setup_lane<K>(g, L);
  LineOp<OPC, double, K> O;
  lineop_setup<OPC, double, K>(g, L, dt, amp, tl, ht,
                               reinterpret_cast<double*>(smem + lay.ocv), O);
  __syncthreads();  // constant-coefficient and uniform-coupling tables written
  double xs[K], ys[K];
#pragma unroll
  for (int k = 0; k < K; ++k)
    xs[k] = (k < L.nval) ? x[g.off + L.cbase + (long long)k * L.cstep] : 0.0;
  lds_put<double, K, lds_pitch(W)>(L, xl, xs);
  __syncthreads();
  line_apply<OPC, double, K, lds_pitch(W)>(g, L, O, xl, xs, ys);
#pragma unroll
  for (int k = 0; k < K; ++k)
    if (k < L.nval) y[g.off + L.cbase + (long long)k * L.cstep] = ys[k];
}

template <int OPC>
static hipError_t launch_apply_t(int shape, const GridDev* grids, int G, const double* tab64,
                                 double amp, double dt, int tabmax, const double* x, double* y,
                                 hipStream_t s) {
  const size_t smem =
      chain_smem_layout(kShapes[shape].W, kShapes[shape].K, tabmax, false, OPC == OPC_HEAT, -1)
          .total;
#define CTM_ACASE(IDX, W, K)                                                                   \
  case IDX:                                                                                    \
    hipLaunchKernelGGL((apply_kernel<OPC, W, K>), dim3(G), dim3(64 * W), smem, s, grids, tab64, \
                       amp, dt, x, y, tabmax);                                                   \
    break;
  switch (shape) {
    CTM_ACASE(0, 1, 4)
    CTM_ACASE(1, 2, 4)
    CTM_ACASE(2, 4, 4)
    CTM_ACASE(3, 8, 4)
    CTM_ACASE(4, 16, 4)
    CTM_ACASE(5, 1, 8)
    CTM_ACASE(6, 2, 8)
    CTM_ACASE(7, 4, 8)
    CTM_ACASE(8, 8, 8)
    CTM_ACASE(9, 16, 8)
    default:
      return hipErrorInvalidValue;
  }
#undef CTM_ACASE
  return hipGetLastError();
}

hipError_t launch_apply(int opc, int shape, const GridDev* grids, int G, const double* tab64,
                        double amp, double dt, int tabmax, const double* x, double* y,
                        hipStream_t s) {
  if (G <= 0) return hipSuccess;
  switch (opc) {
    case OPC_HEAT:
      return launch_apply_t<OPC_HEAT>(shape, grids, G, tab64, amp, dt, tabmax, x, y, s);
    case OPC_SEP:
      return launch_apply_t<OPC_SEP>(shape, grids, G, tab64, amp, dt, tabmax, x, y, s);
    case OPC_VAR:
      return launch_apply_t<OPC_VAR>(shape, grids, G, tab64, amp, dt, tabmax, x, y, s);
    case OPC_DRIFT:
      return launch_apply_t<OPC_DRIFT>(shape, grids, G, tab64, amp, dt, tabmax, x, y, s);
  }
  return hipErrorInvalidValue;
}

// --------------------------------------------------------------- gather
// (I_g u_g)(x): d-linear interpolation on grid g with zero values at the
// Dirichlet boundary nodes and at the implicit node hi of a lattice axis.
__device__ double interp_grid(const GridDev& g, const double* __restrict__ u, const double* x) {
  int base = 0;
  int cidx[MAXD];
  double w[MAXD];
  unsigned ok0 = 0, ok1 = 0;  // corner 0 / corner 1 along axis i is an unknown
#pragma unroll
  for (int i = 0; i < MAXD; ++i) {
    cidx[i] = 0;
    w[i] = 0.0;
    if (i < g.d) {
      const double t = (x[i] - g.lo[i]) / g.h[i];
      const int top = (1 << g.lev[i]) - 1;
      int J = (int)floor(t);
      J = J < 0 ? 0 : (J > top ? top : J);
      w[i] = t - (double)J;
      const int u0i = J - g.j0;
      cidx[i] = u0i;
      if (u0i >= 0 && u0i < g.n[i]) ok0 |= 1u << i;
      if (u0i + 1 >= 0 && u0i + 1 < g.n[i]) ok1 |= 1u << i;
      base += u0i * g.stride[i];
    }
  }
  double acc = 0.0;
  const int ncorner = 1 << g.d;
  for (int c = 0; c < ncorner; ++c) {
    double wt = 1.0;
    int idx = base;
    bool valid = true;
#pragma unroll
    for (int i = 0; i < MAXD; ++i) {
      if (i < g.d) {
        const int bit = (c >> (g.d - 1 - i)) & 1;
        wt *= bit ? w[i] : 1.0 - w[i];
        idx += bit * g.stride[i];
        valid = valid && (((bit ? ok1 : ok0) >> i) & 1u);
      }
    }
    if (valid && wt != 0.0) acc += wt * u[g.off + idx];
  }
  return acc;
}

// The combination at arbitrary points, out[j] = sum_g coef_g (I_g u_g)(x_j).
// One work-group per kGatherThreads points. It walks the grids in packed
// order, a stage at a time: a stage is a run of consecutive grids whose
// unknowns fit kGatherStage doubles (built by the host at plan creation),
// read from HBM as one contiguous, coalesced slice into one of two LDS
// buffers; the next stage is loaded into registers while the current one
// is interpolated, one barrier per stage. A grid larger than a stage is a
// stage of its own and is read from HBM directly. (Before: every thread
// read its 2^d corners of every grid from HBM itself, scattered over a
// cache line per lane, 29 ms for 1e5 points and the 1,709 grids of the
// 6-D workload.)
constexpr int kGatherThreads = 256;
constexpr int kGatherStage = 4096;
constexpr int kGatherPer = kGatherStage / kGatherThreads;

// (I_g u_g)(x) from the grid's values vals[0 .. npts): the same d-linear
// interpolant as interp_grid, with the 2^D corner weights and offsets
// factored into two tensor halves (axes 0 .. D/2-1 and the rest); a corner
// outside the grid's unknowns gets weight 0 and a clamped offset, so the
// corner loop has no branches.
template <int D>
__device__ __forceinline__ double interp_split(const GridDev& g, const double* vals,
                                               const double (&x)[D]) {
  constexpr int DA = D / 2, DB = D - DA;
  double w0[D], w1[D];
  int o0[D], o1[D];
#pragma unroll
  for (int i = 0; i < D; ++i) {
    const double t = (x[i] - g.lo[i]) / g.h[i];
    const int top = (1 << g.lev[i]) - 1;
    int J = (int)floor(t);
    J = J < 0 ? 0 : (J > top ? top : J);
    const double w = t - (double)J;
    const int u0 = J - g.j0;
    const bool ok0 = u0 >= 0 && u0 < g.n[i];
    const bool ok1 = u0 + 1 >= 0 && u0 + 1 < g.n[i];
    w0[i] = ok0 ? 1.0 - w : 0.0;
    w1[i] = ok1 ? w : 0.0;
    o0[i] = (ok0 ? u0 : 0) * g.stride[i];
    o1[i] = (ok1 ? u0 + 1 : 0) * g.stride[i];
  }
  double wa[1 << DA], wb[1 << DB];
  int ia[1 << DA], ib[1 << DB];
#pragma unroll
  for (int c = 0; c < (1 << DA); ++c) {
    double wt = 1.0;
    int o = 0;
#pragma unroll
    for (int i = 0; i < DA; ++i) {
      const bool bit = (c >> i) & 1;
      wt *= bit ? w1[i] : w0[i];
      o += bit ? o1[i] : o0[i];
    }
    wa[c] = wt;
    ia[c] = o;
  }
#pragma unroll
  for (int c = 0; c < (1 << DB); ++c) {
    double wt = 1.0;
    int o = 0;
#pragma unroll
    for (int i = 0; i < DB; ++i) {
      const bool bit = (c >> i) & 1;
      wt *= bit ? w1[DA + i] : w0[DA + i];
      o += bit ? o1[DA + i] : o0[DA + i];
    }
    wb[c] = wt;
    ib[c] = o;
  }
  double acc = 0.0;
#pragma unroll
  for (int b = 0; b < (1 << DB); ++b) {
    double sa = 0.0;
#pragma unroll
    for (int c = 0; c < (1 << DA); ++c) sa += wa[c] * vals[ia[c] + ib[b]];
    acc += wb[b] * sa;
  }
  return acc;
}

template <int D>
__global__ void __launch_bounds__(kGatherThreads)
    gather_kernel(const GridDev* __restrict__ grids, const int2* __restrict__ stages, int nstage,
                  const double* __restrict__ u, const double* __restrict__ pts, long long npts,
                  double* __restrict__ out) {
  __shared__ double buf[2][kGatherStage];
  const long long j = (long long)blockIdx.x * kGatherThreads + threadIdx.x;
  const bool live = j < npts;
  double x[D];
#pragma unroll
  for (int i = 0; i < D; ++i) x[i] = live ? pts[j * D + i] : 0.0;
  // a stage's slice of u: its first grid's offset and its length
  auto slice = [&](int s, long long& o, long long& n) {
    const int2 r = stages[s];
    o = grids[r.x].off;
    n = grids[r.y - 1].off + grids[r.y - 1].npts - o;
  };
  double pre[kGatherPer];
  auto fetch = [&](int s) {
    long long o, n;
    slice(s, o, n);
#pragma unroll
    for (int k = 0; k < kGatherPer; ++k) {
      const long long e = threadIdx.x + (long long)k * kGatherThreads;
      pre[k] = 0.0;
      if (n <= kGatherStage && e < n) pre[k] = u[o + e];
    }
  };
  fetch(0);
  double acc = 0.0;
  for (int s = 0; s < nstage; ++s) {
    double* cur = buf[s & 1];
    long long o, n;
    slice(s, o, n);
    const bool staged = n <= kGatherStage;
    if (staged) {
#pragma unroll
      for (int k = 0; k < kGatherPer; ++k) {
        const int e = threadIdx.x + k * kGatherThreads;
        if (e < n) cur[e] = pre[k];
      }
    }
    // the stage is in LDS; every thread is past its reads of this buffer's
    // previous stage (two stages back, before the last barrier)
    __syncthreads();
    if (s + 1 < nstage) fetch(s + 1);
    // two loops, so that each reads through a pointer of known address
    // space (LDS reads; a pointer that may be either becomes flat loads,
    // each waiting for the next stage's loads in flight)
    const int2 r = stages[s];
    if (staged) {
      for (int gi = r.x; gi < r.y; ++gi) {
        const GridDev& g = grids[gi];
        acc += g.coef * interp_split<D>(g, cur + (g.off - o), x);
      }
    } else {
      for (int gi = r.x; gi < r.y; ++gi) {
        const GridDev& g = grids[gi];
        acc += g.coef * interp_split<D>(g, u + g.off, x);
      }
    }
  }
  if (live) out[j] = acc;
}

hipError_t launch_gather(const GridDev* grids, const int2* stages, int nstage, int d,
                         const double* u, const double* pts, long long npts, double* out,
                         hipStream_t s) {
  if (npts <= 0) return hipSuccess;
  if (nstage <= 0) return hipErrorInvalidValue;
  const dim3 grid((unsigned)((npts + kGatherThreads - 1) / kGatherThreads)), block(kGatherThreads);
  switch (d) {
#define CTM_GATHER(D)                                                                        \
  case D:                                                                                    \
    hipLaunchKernelGGL(gather_kernel<D>, grid, block, 0, s, grids, stages, nstage, u, pts,   \
                       npts, out);                                                           \
    break;
    CTM_GATHER(1)
    CTM_GATHER(2)
    CTM_GATHER(3)
    CTM_GATHER(4)
    CTM_GATHER(5)
    CTM_GATHER(6)
    CTM_GATHER(7)
    CTM_GATHER(8)
#undef CTM_GATHER
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

int gather_stage_capacity() { return kGatherStage; }

// Combine-then-project: the combination evaluated at the unknowns of every
// grid (packed index -> grid by binary search over the offsets).
__global__ void project_kernel(const GridDev* __restrict__ grids,
                               const long long* __restrict__ offsets, int G, long long slen,
                               const double* __restrict__ u, double* __restrict__ out) {
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= slen) return;
  int lo = 0, hi = G - 1;
  while (lo < hi) {
    const int mid = (lo + hi + 1) >> 1;
    if (offsets[mid] <= e) lo = mid;
    else hi = mid - 1;
  }
  const GridDev& tg = grids[lo];
  int rem = (int)(e - tg.off);
  double x[MAXD];
#pragma unroll
  for (int i = MAXD - 1; i >= 0; --i) {
    x[i] = 0.0;
    if (i < tg.d) {
      const int j = rem % tg.n[i];
      rem /= tg.n[i];
      x[i] = tg.lo[i] + (double)(j + tg.j0) * tg.h[i];
    }
  }
  double acc = 0.0;
  for (int gi = 0; gi < G; ++gi) {
    const GridDev& g = grids[gi];
    acc += g.coef * interp_grid(g, u, x);
  }
  out[e] = acc;
}

hipError_t launch_project(const GridDev* grids, const long long* offsets, int G, long long slen,
                          const double* u, double* out, hipStream_t s) {
  if (slen <= 0) return hipSuccess;
  hipLaunchKernelGGL(project_kernel, dim3((unsigned)((slen + 255) / 256)), dim3(256), 0, s, grids,
                     offsets, G, slen, u, out);
  return hipGetLastError();
}

// ----------------------------------------------------- hierarchical basis
// 1-D passes along each axis of the grid: a node J at level k (an odd
// multiple of 2^(l-k)) has the parents J -/+ 2^(l-k); its surplus is its
// value minus their mean (zero at the Dirichlet boundary and at the lattice
// node hi). Forward: levels finest first; inverse: coarsest first. Nodes of
// one level only read coarser ones, so a level is one parallel pass.
template <bool INV>
__global__ void __launch_bounds__(256)
    hier_kernel(const GridDev* __restrict__ grids, int lattice, const double* in,
                double* out) {
  extern __shared__ double buf[];
  __shared__ GridDev gs;
  {
    const int* src = reinterpret_cast<const int*>(grids + blockIdx.x);
    int* dst = reinterpret_cast<int*>(&gs);
    for (int t = threadIdx.x; t < (int)(sizeof(GridDev) / sizeof(int)); t += 256) dst[t] = src[t];
  }
  __syncthreads();
  const GridDev& g = gs;
  const int npts = g.npts;
  for (int p = threadIdx.x; p < npts; p += 256) buf[p] = in[g.off + p];
  __syncthreads();
  const int j0 = lattice ? 0 : 1;
  for (int i = 0; i < g.d; ++i) {
    const int li = g.lev[i], ni = g.n[i], sti = g.stride[i];
    for (int step = 0; step < li; ++step) {
      const int k = INV ? 1 + step : li - step;
      const int st = 1 << (li - k);
      for (int p = threadIdx.x; p < npts; p += 256) {
        const int J = (p / sti) % ni + j0;
        if ((J & (2 * st - 1)) != st) continue;
        const int jl = J - st - j0, jr = J + st - j0;  // parents as unknown indices
        const double vl = (jl >= 0) ? buf[p - st * sti] : 0.0;
        const double vr = (jr < ni) ? buf[p + st * sti] : 0.0;
        const double m = 0.5 * (vl + vr);
        buf[p] = INV ? buf[p] + m : buf[p] - m;
      }
      __syncthreads();
    }
  }
  for (int p = threadIdx.x; p < npts; p += 256) out[g.off + p] = buf[p];
}

hipError_t launch_hierarchize(const GridDev* grids, int G, int maxpts, bool lattice,
                              bool inverse, const double* in, double* out, hipStream_t s) {
  if (G <= 0) return hipSuccess;
  const size_t smem = (size_t)maxpts * sizeof(double);
  if (inverse)
    hipLaunchKernelGGL(hier_kernel<true>, dim3(G), dim3(256), smem, s, grids, (int)lattice, in,
                       out);
  else
    hipLaunchKernelGGL(hier_kernel<false>, dim3(G), dim3(256), smem, s, grids, (int)lattice, in,
                       out);
  return hipGetLastError();
}

__global__ void __launch_bounds__(256)
    hier_combine_kernel(const int* __restrict__ off, const int* __restrict__ idx,
                        const double* __restrict__ coef, int nodes,
                        const double* __restrict__ uh, double* __restrict__ sg) {
  const int s = blockIdx.x * 256 + threadIdx.x;
  if (s >= nodes) return;
  double acc = 0.0;
  for (int e = off[s]; e < off[s + 1]; ++e) acc += coef[e] * uh[idx[e]];
  sg[s] = acc;
}

hipError_t launch_hier_combine(const int* off, const int* idx, const double* coef, int nodes,
                               const double* uh, double* sg, hipStream_t s) {
  if (nodes <= 0) return hipSuccess;
  hipLaunchKernelGGL(hier_combine_kernel, dim3((nodes + 255) / 256), dim3(256), 0, s, off, idx,
                     coef, nodes, uh, sg);
  return hipGetLastError();
}

__global__ void __launch_bounds__(256)
    hier_scatter_kernel(const int* __restrict__ node, long long slen,
                        const double* __restrict__ sg, double* __restrict__ out) {
  const long long p = (long long)blockIdx.x * 256 + threadIdx.x;
  if (p < slen) out[p] = sg[node[p]];
}

hipError_t launch_hier_scatter(const int* node, long long slen, const double* sg, double* out,
                               hipStream_t s) {
  if (slen <= 0) return hipSuccess;
  hipLaunchKernelGGL(hier_scatter_kernel, dim3((unsigned)((slen + 255) / 256)), dim3(256), 0, s,
                     node, slen, sg, out);
  return hipGetLastError();
}

// ----------------------------------------------------------- reductions
__global__ void __launch_bounds__(256)
    grid_norms2_kernel(const GridDev* __restrict__ grids, const double* __restrict__ u,
                       double* __restrict__ out) {
  __shared__ double slots[2 * 64];
  const GridDev& g = grids[blockIdx.x];
  double s = 0.0;
  for (int p = threadIdx.x; p < g.npts; p += 256) {
    const double v = u[g.off + p];
    s += v * v;
  }
  double v[1] = {s};
  RedRing ring{slots, 0};
  block_sum<4, 1, double>(v, ring);
  if (threadIdx.x == 0) out[blockIdx.x] = v[0];
}

hipError_t launch_grid_norms2(const GridDev* grids, int G, const double* u, double* out,
                              hipStream_t s) {
  if (G <= 0) return hipSuccess;
  hipLaunchKernelGGL(grid_norms2_kernel, dim3(G), dim3(256), 0, s, grids, u, out);
  return hipGetLastError();
}

// The MGRIT residual test: max over tasks t of sqrt(res2[t] /
// norm2[grid(t)]) (norm2 = 0 -> 1; NaN wins), in two passes: up to
// kResBlocks work-groups each reduce a strided share of the tasks into
// part[], then one work-group reduces part[] and records the iteration.
// (One work-group over all tasks took 0.74 ms per iteration for the
// 218,752 tasks of the 6-D workload, alone on the critical path.) The max
// is exact, so the result does not depend on the split.
__device__ __forceinline__ double nanmax(double a, double b) { return (b > a || b != b) ? b : a; }

__device__ __forceinline__ double block_max256(double m, double* sm) {
  sm[threadIdx.x] = m;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) sm[threadIdx.x] = nanmax(sm[threadIdx.x], sm[threadIdx.x + w]);
    __syncthreads();
  }
  return sm[0];
}

__global__ void __launch_bounds__(256)
    residual_part_kernel(const int2* __restrict__ tasks, int ntasks,
                         const double* __restrict__ res2, const double* __restrict__ norm2,
                         double* __restrict__ part) {
  __shared__ double sm[256];
  double m = 0.0;
  for (int t = blockIdx.x * 256 + threadIdx.x; t < ntasks; t += gridDim.x * 256) {
    const double n2 = norm2[tasks[t].x];
    m = nanmax(m, sqrt(res2[t] / (n2 > 0.0 ? n2 : 1.0)));
  }
  const double r = block_max256(m, sm);
  if (threadIdx.x == 0) part[blockIdx.x] = r;
}

__global__ void __launch_bounds__(256)
    residual_max_kernel(const double* __restrict__ part, int nparts, double* __restrict__ mg,
                        double* __restrict__ host_mg, int it, double tol,
                        const int* __restrict__ status) {
  __shared__ double sm[256];
  double m = 0.0;
  for (int b = threadIdx.x; b < nparts; b += 256) m = nanmax(m, part[b]);
  const double res = block_max256(m, sm);
  if (threadIdx.x == 0) {
    if (mg[0] == 0.0) {
      mg[2 * it] = res;
      const bool nonfinite = (res != res) || ((*status >> CTM_ERR_NONFINITE) & 1);
      if (res <= tol || nonfinite) mg[0] = (double)it;
    }
    mg[2 * it + 1] = mg[0];
    if (host_mg) {  // pinned host mirror, read by the host after this iteration's event
      host_mg[2 * it] = mg[2 * it];
      host_mg[2 * it + 1] = mg[2 * it + 1];
    }
  }
}

hipError_t launch_residual_max(const int2* tasks, int ntasks, const double* res2,
                               const double* norm2, double* part, double* mg, double* host_mg,
                               int it, double tol, const int* status, hipStream_t s) {
  const int nb = ntasks <= 0 ? 1 : std::min(kResBlocks, (ntasks + 255) / 256);
  hipLaunchKernelGGL(residual_part_kernel, dim3(nb), dim3(256), 0, s, tasks, ntasks, res2, norm2,
                     part);
  hipLaunchKernelGGL(residual_max_kernel, dim3(1), dim3(256), 0, s, part, nb, mg, host_mg, it,
                     tol, status);
  return hipGetLastError();
}

// ------------------------------------------------------------ vector ops
// Vector index q runs over blockIdx.y, gridDim.y, ... < nvec (the grid's y
// extent is capped at 65,535).
constexpr int kMaxGridY = 65535;

__global__ void vec_add_kernel(VecRef dst, VecRef x, VecRef y, int nvec, long long slen,
                               const double* skip) {
  if (skip && *skip != 0.0) return;
  const long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= slen) return;
  for (long long q = blockIdx.y; q < nvec; q += gridDim.y) {
    double v = x.base[(x.a * q + x.b) * slen + e];
    if (y.base) v += y.base[(y.a * q + y.b) * slen + e];
    dst.base[(dst.a * q + dst.b) * slen + e] = v;
  }
}

hipError_t launch_vec_add(VecRef dst, VecRef x, VecRef y, int nvec, long long slen,
                          hipStream_t s, const double* skip) {
  if (nvec <= 0 || slen <= 0) return hipSuccess;
  const unsigned gy = (unsigned)(nvec < kMaxGridY ? nvec : kMaxGridY);
  hipLaunchKernelGGL(vec_add_kernel, dim3((unsigned)((slen + 255) / 256), gy), dim3(256), 0, s,
                     dst, x, y, nvec, slen, skip);
  return hipGetLastError();
}

__global__ void class_vec_add_kernel(const int2* __restrict__ tasks,
                                     const GridDev* __restrict__ grids, VecRef dst, VecRef x,
                                     VecRef y, int nvec, long long slen, const double* skip) {
  if (skip && *skip != 0.0) return;
  const GridDev& g = grids[tasks[blockIdx.x].x];
  const long long base = g.off;
  for (long long q = blockIdx.y; q < nvec; q += gridDim.y) {
    double* d = dst.base + (dst.a * q + dst.b) * slen + base;
    const double* xs = x.base ? x.base + (x.a * q + x.b) * slen + base : nullptr;
    const double* ys = y.base ? y.base + (y.a * q + y.b) * slen + base : nullptr;
    for (int e = threadIdx.x; e < g.npts; e += blockDim.x)
      d[e] = (xs ? xs[e] : 0.0) + (ys ? ys[e] : 0.0);
  }
}

hipError_t launch_class_vec_add(const int2* tasks, int ntasks, const GridDev* grids, VecRef dst,
                                VecRef x, VecRef y, int nvec, long long slen, hipStream_t s,
                                const double* skip) {
  if (ntasks <= 0 || nvec <= 0) return hipSuccess;
  const unsigned gy = (unsigned)(nvec < kMaxGridY ? nvec : kMaxGridY);
  hipLaunchKernelGGL(class_vec_add_kernel, dim3((unsigned)ntasks, gy), dim3(256), 0, s, tasks,
                     grids, dst, x, y, nvec, slen, skip);
  return hipGetLastError();
}

__global__ void fill_zero_kernel(double* p, long long n, const double* skip) {
  if (skip && *skip != 0.0) return;
  for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < n;
       e += (long long)gridDim.x * blockDim.x)
    p[e] = 0.0;
}

hipError_t launch_fill_zero(double* p, long long n, hipStream_t s, const double* skip) {
  if (n <= 0) return hipSuccess;
  long long blocks = (n + 255) / 256;
  if (blocks > 65536) blocks = 65536;
  hipLaunchKernelGGL(fill_zero_kernel, dim3((unsigned)blocks), dim3(256), 0, s, p, n, skip);
  return hipGetLastError();
}

}  // namespace ctm
