// Instantiations of the streaming kernel (every operator class and Krylov
// method) and of its point-wise apply.
#include "stream_kernel.hpp"

namespace ctm {

hipError_t launch_stream(int opc, int solver, const ChainArgs& a, int ntasks, int tabmax,
                         double* scratch, long long ss, hipStream_t s) {
  const bool cg = (solver == SOLV_CG);
  switch (opc) {
    case OPC_HEAT:
      return cg ? launch_stream_t<OPC_HEAT, SOLV_CG>(a, ntasks, tabmax, scratch, ss, s)
                : launch_stream_t<OPC_HEAT, SOLV_BICG>(a, ntasks, tabmax, scratch, ss, s);
    case OPC_VAR:
      return cg ? launch_stream_t<OPC_VAR, SOLV_CG>(a, ntasks, tabmax, scratch, ss, s)
                : launch_stream_t<OPC_VAR, SOLV_BICG>(a, ntasks, tabmax, scratch, ss, s);
    case OPC_SEP:
      return launch_stream_t<OPC_SEP, SOLV_BICG>(a, ntasks, tabmax, scratch, ss, s);
    case OPC_DRIFT:
      return launch_stream_t<OPC_DRIFT, SOLV_BICG>(a, ntasks, tabmax, scratch, ss, s);
    default:
      return hipErrorInvalidValue;
  }
}

hipError_t launch_stream_apply(int opc, const GridDev* grids, int G, const double* tab64,
                               double amp, double dt, int tabmax, const double* x, double* y,
                               hipStream_t s) {
  if (G <= 0) return hipSuccess;
  const size_t smem = (size_t)tabmax * sizeof(double);
  const dim3 grid(G), block(kStreamThreads);
  switch (opc) {
    case OPC_HEAT:
      hipLaunchKernelGGL(stream_apply_kernel<OPC_HEAT>, grid, block, smem, s, grids, tab64, amp,
                         dt, x, y);
      break;
    case OPC_SEP:
      hipLaunchKernelGGL(stream_apply_kernel<OPC_SEP>, grid, block, smem, s, grids, tab64, amp,
                         dt, x, y);
      break;
    case OPC_VAR:
      hipLaunchKernelGGL(stream_apply_kernel<OPC_VAR>, grid, block, smem, s, grids, tab64, amp,
                         dt, x, y);
      break;
    case OPC_DRIFT:
      hipLaunchKernelGGL(stream_apply_kernel<OPC_DRIFT>, grid, block, smem, s, grids, tab64, amp,
                         dt, x, y);
      break;
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

}  // namespace ctm
