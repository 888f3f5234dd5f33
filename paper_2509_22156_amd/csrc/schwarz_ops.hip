// Device set-up and standalone application of the two-level overlapping
// Schwarz preconditioner (Section 2.1.2): the Galerkin restrictions of the
// step matrix A = I + dt L to every subdomain and to the coarse space,
// assembled from the streaming kernel's point coefficients and inverted in
// place by Gauss-Jordan elimination with partial pivoting, one work-group
// per matrix.
#include "stream_kernel.hpp"

namespace ctm {

namespace {

constexpr int kSetupThreads = 256;

__device__ __forceinline__ void copy_grid(const GridDev* grids, int g, GridDev& gs) {
  const int* src = reinterpret_cast<const int*>(grids + g);
  int* dst = reinterpret_cast<int*>(&gs);
  for (int t = threadIdx.x; t < (int)(sizeof(GridDev) / sizeof(int)); t += blockDim.x)
    dst[t] = src[t];
}

// Local row of grid point q in a subdomain: binary search of the (point,
// row) pairs sorted by point; -1 when q is outside.
__device__ __forceinline__ int local_row(const int* srt, int n, int q) {
  int lo = 0, hi = n - 1;
  while (lo <= hi) {
    const int mid = (lo + hi) >> 1;
    const int pm = srt[2 * mid];
    if (pm == q) return srt[2 * mid + 1];
    if (pm < q)
      lo = mid + 1;
    else
      hi = mid - 1;
  }
  return -1;
}

// R_i A R_i^T of subdomain blockIdx.x (owner grid sub_grid[i]) into its
// slot of linv, column-major.
template <int OPC, int D>
__global__ void __launch_bounds__(kSetupThreads)
    schwarz_local_kernel(const GridDev* __restrict__ grids, const double* __restrict__ tab64,
                         double amp, double dt, SchwarzView v, double* linv,
                         const int* __restrict__ sub_grid) {
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ GridDev gs;
  double* tl = reinterpret_cast<double*>(smem);
  const long long k = blockIdx.x;
  copy_grid(grids, sub_grid[k], gs);
  __syncthreads();
  load_tables<OPC, double, kSetupThreads>(gs, tab64, dt, tl);
  const SchwarzSub sb = v.sub[k];
  const int n = sb.n;
  double* M = linv + sb.inv;
  for (long long e = threadIdx.x; e < (long long)n * n; e += kSetupThreads) M[e] = 0.0;
  __syncthreads();
  const int* idx = v.ints + sb.idx;
  const int* srt = v.ints + sb.srt;
  for (int r = threadIdx.x; r < n; r += kSetupThreads) {
    const int p = idx[r];
    PointCoef<OPC, D> c;
    point_coef<OPC, D>(gs, tl, dt, amp, p, c);
    M[(long long)r * n + r] = c.diag;
#pragma unroll
    for (int i = 0; i < D; ++i) {
      if (i >= gs.d) continue;
      const int ql = stencil_lo(gs, c, i, p), qu = stencil_up(gs, c, i, p);
      if (ql != p) {
        const int col = local_row(srt, n, ql);
        if (col >= 0) M[(long long)col * n + r] = c.lo[i];
      }
      if (qu != p) {
        const int col = local_row(srt, n, qu);
        if (col >= 0) M[(long long)col * n + r] = c.up[i];
      }
    }
  }
}

// R_0 A R_0^T of grid blockIdx.x into its slot of cinv, column-major; row a
// (coarse block a) is summed by one thread over the block's points.
template <int OPC, int D>
__global__ void __launch_bounds__(kSetupThreads)
    schwarz_coarse_kernel(const GridDev* __restrict__ grids, const double* __restrict__ tab64,
                          double amp, double dt, SchwarzView v, double* cinv) {
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ GridDev gs;
  double* tl = reinterpret_cast<double*>(smem);
  const int g = blockIdx.x;
  copy_grid(grids, g, gs);
  __syncthreads();
  load_tables<OPC, double, kSetupThreads>(gs, tab64, dt, tl);
  const SchwarzGrid sg = v.grid[g];
  const int nb = sg.nblk;
  double* M = cinv + sg.cinv;
  for (long long e = threadIdx.x; e < (long long)nb * nb; e += kSetupThreads) M[e] = 0.0;
  __syncthreads();
  const int* cord = v.ints + sg.cord;
  const int* cblk = v.ints + sg.cblk;
  const int* bst = v.ints + sg.bst;
  for (int a = threadIdx.x; a < nb; a += kSetupThreads) {
    for (int pos = bst[a]; pos < bst[a + 1]; ++pos) {
      const int p = cord[pos];
      PointCoef<OPC, D> c;
      point_coef<OPC, D>(gs, tl, dt, amp, p, c);
      M[(long long)a * nb + a] += c.diag;
#pragma unroll
      for (int i = 0; i < D; ++i) {
        if (i >= gs.d) continue;
        const int ql = stencil_lo(gs, c, i, p), qu = stencil_up(gs, c, i, p);
        if (ql != p) M[(long long)cblk[ql] * nb + a] += c.lo[i];
        if (qu != p) M[(long long)cblk[qu] * nb + a] += c.up[i];
      }
    }
  }
}

// In-place inverse of matrix blockIdx.x (kind 0: subdomain records, kind 1:
// grids' coarse matrices), column-major n x n, by Gauss-Jordan elimination
// with partial pivoting: step k takes the largest |entry| of column k at or
// below the diagonal as pivot (row swap), then every entry is updated from
// the old pivot row and column (kept in LDS); the row swaps become column
// swaps of the result, undone in reverse order at the end. A zero or
// non-finite pivot sets the breakdown bit and leaves the matrix.
// LDS: 2 nmax doubles + nmax ints.
__global__ void __launch_bounds__(kSetupThreads)
    gauss_jordan_kernel(SchwarzView v, double* base, int kind, int* status) {
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ double bv[kSetupThreads];
  __shared__ int bi[kSetupThreads];
  long long off;
  int n;
  if (kind == 0) {
    off = v.sub[blockIdx.x].inv;
    n = v.sub[blockIdx.x].n;
  } else {
    off = v.grid[blockIdx.x].cinv;
    n = v.grid[blockIdx.x].nblk;
  }
  double* M = base + off;
  double* colk = reinterpret_cast<double*>(smem);
  double* rowk = colk + n;
  int* perm = reinterpret_cast<int*>(rowk + n);
  const int t = threadIdx.x;
  for (int k = 0; k < n; ++k) {
    // pivot: largest magnitude in column k, rows k..n-1 (lowest row on ties)
    double best = -1.0;
    int bidx = k;
    for (int r = k + t; r < n; r += kSetupThreads) {
      const double a = fabs(M[(long long)k * n + r]);
      if (a > best) {
        best = a;
        bidx = r;
      }
    }
    bv[t] = best;
    bi[t] = bidx;
    __syncthreads();
    for (int w = kSetupThreads / 2; w > 0; w >>= 1) {
      if (t < w) {
        const double o = bv[t + w];
        const int oi = bi[t + w];
        if (o > bv[t] || (o == bv[t] && oi < bi[t])) {
          bv[t] = o;
          bi[t] = oi;
        }
      }
      __syncthreads();
    }
    const double pmag = bv[0];
    const int piv = bi[0];
    __syncthreads();
    if (!(pmag > 0.0) || !(pmag < 1e300)) {  // zero or not finite: uniform exit
      if (t == 0) atomicOr(status, FLAG_BREAKDOWN);
      return;
    }
    if (piv != k) {
      for (int c = t; c < n; c += kSetupThreads) {
        const double a = M[(long long)c * n + k];
        M[(long long)c * n + k] = M[(long long)c * n + piv];
        M[(long long)c * n + piv] = a;
      }
      __syncthreads();
    }
    for (int r = t; r < n; r += kSetupThreads) colk[r] = M[(long long)k * n + r];
    for (int c = t; c < n; c += kSetupThreads) rowk[c] = M[(long long)c * n + k];
    if (t == 0) perm[k] = piv;
    __syncthreads();
    const double ipv = 1.0 / rowk[k];
    for (long long e = t; e < (long long)n * n; e += kSetupThreads) {
      const int r = (int)(e % n), c = (int)(e / n);
      double val;
      if (r == k)
        val = (c == k) ? ipv : rowk[c] * ipv;
      else
        val = (c == k) ? -colk[r] * ipv : M[e] - colk[r] * rowk[c] * ipv;
      M[e] = val;
    }
    __syncthreads();
  }
  for (int k = n - 1; k >= 0; --k) {
    const int p = perm[k];
    if (p != k) {
      for (int r = t; r < n; r += kSetupThreads) {
        const double a = M[(long long)k * n + r];
        M[(long long)k * n + r] = M[(long long)p * n + r];
        M[(long long)p * n + r] = a;
      }
    }
    __syncthreads();
  }
}

// y = C x on grid blockIdx.x (ctm_precond_apply): x copied to the grid's
// scratch residual slot, the preconditioner applied into its direction
// slot, the result copied out.
template <int OPC, int D>
__global__ void __launch_bounds__(kStreamThreads)
    schwarz_apply_kernel(const GridDev* __restrict__ grids, const double* __restrict__ tab64,
                         double amp, double dt, int tabmax, SchwarzView v,
                         const double* __restrict__ x, double* __restrict__ y, double* scratch,
                         long long ss) {
  extern __shared__ __align__(16) unsigned char smem[];
  __shared__ GridDev gs;
  double* tl = reinterpret_cast<double*>(smem);
  copy_grid(grids, blockIdx.x, gs);
  __syncthreads();
  load_tables<OPC, double, kStreamThreads>(gs, tab64, dt, tl);
  double* sv = scratch + (long long)blockIdx.x * SV_N * ss;
  double* R = sv + SV_R * ss;
  double* Z = sv + SV_S * ss;
  for (int p = threadIdx.x; p < gs.npts; p += kStreamThreads) R[p] = x[gs.off + p];
  __syncthreads();
  schwarz_apply<OPC, D>(gs, tl, dt, amp, v, v.grid[blockIdx.x], tl + tabmax, sv, ss, R, Z,
                        nullptr);
  for (int p = threadIdx.x; p < gs.npts; p += kStreamThreads) y[gs.off + p] = Z[p];
}

template <int OPC, int D>
hipError_t setup_t(const GridDev* grids, int G, const double* tab64, double amp, double dt,
                   int tabmax, const SchwarzView& v, double* linv, double* cinv,
                   const int* sub_grid, long long nsub, int nmax_sub, int* status,
                   hipStream_t s) {
  const size_t tsm = (size_t)tabmax * sizeof(double);
  hipLaunchKernelGGL((schwarz_local_kernel<OPC, D>), dim3((unsigned)nsub), dim3(kSetupThreads),
                     tsm, s, grids, tab64, amp, dt, v, linv, sub_grid);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((schwarz_coarse_kernel<OPC, D>), dim3((unsigned)G), dim3(kSetupThreads), tsm,
                     s, grids, tab64, amp, dt, v, cinv);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  SchwarzView lv = v;
  lv.linv = linv;
  lv.cinv = cinv;
  auto gj_lds = [](int n) { return (size_t)n * (2 * sizeof(double) + sizeof(int)); };
  hipLaunchKernelGGL(gauss_jordan_kernel, dim3((unsigned)nsub), dim3(kSetupThreads),
                     gj_lds(nmax_sub), s, lv, linv, 0, status);
  if ((e = hipGetLastError()) != hipSuccess) return e;
  hipLaunchKernelGGL(gauss_jordan_kernel, dim3((unsigned)G), dim3(kSetupThreads),
                     gj_lds(v.nbmax), s, lv, cinv, 1, status);
  return hipGetLastError();
}

template <int OPC, int D>
hipError_t apply_t(const GridDev* grids, int G, const double* tab64, double amp, double dt,
                   int tabmax, const SchwarzView& v, const double* x, double* y,
                   double* scratch, long long ss, hipStream_t s) {
  const size_t smem = ((size_t)tabmax + 3 * (size_t)v.nbmax) * sizeof(double);
  hipLaunchKernelGGL((schwarz_apply_kernel<OPC, D>), dim3((unsigned)G), dim3(kStreamThreads), smem,
                     s, grids, tab64, amp, dt, tabmax, v, x, y, scratch, ss);
  return hipGetLastError();
}

template <int D>
hipError_t setup_d(int opc, const GridDev* grids, int G, const double* tab64, double amp,
                   double dt, int tabmax, const SchwarzView& v, double* linv, double* cinv,
                   const int* sub_grid, long long nsub, int nmax_sub, int* status,
                   hipStream_t s) {
  switch (opc) {
    case OPC_HEAT:
      return setup_t<OPC_HEAT, D>(grids, G, tab64, amp, dt, tabmax, v, linv, cinv, sub_grid,
                                  nsub, nmax_sub, status, s);
    case OPC_SEP:
      return setup_t<OPC_SEP, D>(grids, G, tab64, amp, dt, tabmax, v, linv, cinv, sub_grid, nsub,
                                 nmax_sub, status, s);
    case OPC_VAR:
      return setup_t<OPC_VAR, D>(grids, G, tab64, amp, dt, tabmax, v, linv, cinv, sub_grid, nsub,
                                 nmax_sub, status, s);
    case OPC_DRIFT:
      return setup_t<OPC_DRIFT, D>(grids, G, tab64, amp, dt, tabmax, v, linv, cinv, sub_grid,
                                   nsub, nmax_sub, status, s);
    default:
      return hipErrorInvalidValue;
  }
}

template <int D>
hipError_t apply_d(int opc, const GridDev* grids, int G, const double* tab64, double amp,
                   double dt, int tabmax, const SchwarzView& v, const double* x, double* y,
                   double* scratch, long long ss, hipStream_t s) {
  switch (opc) {
    case OPC_HEAT:
      return apply_t<OPC_HEAT, D>(grids, G, tab64, amp, dt, tabmax, v, x, y, scratch, ss, s);
    case OPC_SEP:
      return apply_t<OPC_SEP, D>(grids, G, tab64, amp, dt, tabmax, v, x, y, scratch, ss, s);
    case OPC_VAR:
      return apply_t<OPC_VAR, D>(grids, G, tab64, amp, dt, tabmax, v, x, y, scratch, ss, s);
    case OPC_DRIFT:
      return apply_t<OPC_DRIFT, D>(grids, G, tab64, amp, dt, tabmax, v, x, y, scratch, ss, s);
    default:
      return hipErrorInvalidValue;
  }
}

}  // namespace

hipError_t launch_schwarz_setup(int opc, int d, const GridDev* grids, int G, const double* tab64,
                                double amp, double dt, int tabmax, const SchwarzView& v,
                                double* linv, double* cinv, const int* sub_grid,
                                long long nsub_total, int nmax_sub, int* status,
                                hipStream_t s) {
  if (G <= 0 || nsub_total <= 0) return hipSuccess;
  if (d < 1 || d > MAXD) return hipErrorInvalidValue;
  if (d <= 2)
    return setup_d<2>(opc, grids, G, tab64, amp, dt, tabmax, v, linv, cinv, sub_grid, nsub_total,
                      nmax_sub, status, s);
  if (d <= 4)
    return setup_d<4>(opc, grids, G, tab64, amp, dt, tabmax, v, linv, cinv, sub_grid, nsub_total,
                      nmax_sub, status, s);
  return setup_d<MAXD>(opc, grids, G, tab64, amp, dt, tabmax, v, linv, cinv, sub_grid,
                       nsub_total, nmax_sub, status, s);
}

hipError_t launch_schwarz_apply(int opc, int solver, int d, const GridDev* grids, int G,
                                const double* tab64, double amp, double dt, int tabmax,
                                const SchwarzView& v, const double* x, double* y,
                                double* scratch, long long ss, hipStream_t s) {
  (void)solver;  // the view carries the form (balanced with CG)
  if (G <= 0) return hipSuccess;
  if (d < 1 || d > MAXD) return hipErrorInvalidValue;
  if (d <= 2) return apply_d<2>(opc, grids, G, tab64, amp, dt, tabmax, v, x, y, scratch, ss, s);
  if (d <= 4) return apply_d<4>(opc, grids, G, tab64, amp, dt, tabmax, v, x, y, scratch, ss, s);
  return apply_d<MAXD>(opc, grids, G, tab64, amp, dt, tabmax, v, x, y, scratch, ss, s);
}

}  // namespace ctm
