// Instantiations of the streaming kernel (every operator class, Krylov
// method and dimension bound D in {2, 4, 8}) and of its point-wise apply.
#include "stream_kernel.hpp"

namespace ctm {

namespace {

template <int D>
hipError_t launch_stream_d(int opc, int solver, const ChainArgs& a, int ntasks, int tabmax,
                           double* scratch, long long ss, hipStream_t s) {
  const bool cg = (solver == SOLV_CG);
  switch (opc) {
    case OPC_HEAT:
      return cg ? launch_stream_t<OPC_HEAT, SOLV_CG, D>(a, ntasks, tabmax, scratch, ss, s)
                : launch_stream_t<OPC_HEAT, SOLV_BICG, D>(a, ntasks, tabmax, scratch, ss, s);
    case OPC_VAR:
      return cg ? launch_stream_t<OPC_VAR, SOLV_CG, D>(a, ntasks, tabmax, scratch, ss, s)
                : launch_stream_t<OPC_VAR, SOLV_BICG, D>(a, ntasks, tabmax, scratch, ss, s);
    case OPC_SEP:
      return launch_stream_t<OPC_SEP, SOLV_BICG, D>(a, ntasks, tabmax, scratch, ss, s);
    case OPC_DRIFT:
      return launch_stream_t<OPC_DRIFT, SOLV_BICG, D>(a, ntasks, tabmax, scratch, ss, s);
    default:
      return hipErrorInvalidValue;
  }
}

template <int D>
hipError_t launch_stream_apply_d(int opc, const GridDev* grids, int G, const double* tab64,
                                 double amp, double dt, size_t smem, const double* x, double* y,
                                 hipStream_t s) {
  const dim3 grid(G), block(kStreamThreads);
  switch (opc) {
    case OPC_HEAT:
      hipLaunchKernelGGL((stream_apply_kernel<OPC_HEAT, D>), grid, block, smem, s, grids, tab64,
                         amp, dt, x, y);
      break;
    case OPC_SEP:
      hipLaunchKernelGGL((stream_apply_kernel<OPC_SEP, D>), grid, block, smem, s, grids, tab64,
                         amp, dt, x, y);
      break;
    case OPC_VAR:
      hipLaunchKernelGGL((stream_apply_kernel<OPC_VAR, D>), grid, block, smem, s, grids, tab64,
                         amp, dt, x, y);
      break;
    case OPC_DRIFT:
      hipLaunchKernelGGL((stream_apply_kernel<OPC_DRIFT, D>), grid, block, smem, s, grids,
                         tab64, amp, dt, x, y);
      break;
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace

hipError_t launch_stream(int opc, int solver, int d, const ChainArgs& a, int ntasks, int tabmax,
                         double* scratch, long long ss, hipStream_t s) {
  if (d < 1 || d > MAXD) return hipErrorInvalidValue;
  if (d <= 2) return launch_stream_d<2>(opc, solver, a, ntasks, tabmax, scratch, ss, s);
  if (d <= 4) return launch_stream_d<4>(opc, solver, a, ntasks, tabmax, scratch, ss, s);
  return launch_stream_d<MAXD>(opc, solver, a, ntasks, tabmax, scratch, ss, s);
}

hipError_t launch_stream_apply(int opc, int d, const GridDev* grids, int G, const double* tab64,
                               double amp, double dt, int tabmax, const double* x, double* y,
                               hipStream_t s) {
  if (G <= 0) return hipSuccess;
  if (d < 1 || d > MAXD) return hipErrorInvalidValue;
  const size_t smem = (size_t)tabmax * sizeof(double);
  if (d <= 2) return launch_stream_apply_d<2>(opc, grids, G, tab64, amp, dt, smem, x, y, s);
  if (d <= 4) return launch_stream_apply_d<4>(opc, grids, G, tab64, amp, dt, smem, x, y, s);
  return launch_stream_apply_d<MAXD>(opc, grids, G, tab64, amp, dt, smem, x, y, s);
}

}  // namespace ctm
