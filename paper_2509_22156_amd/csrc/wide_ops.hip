// Instantiations of the wide streaming solver's kernels (every operator
// class, Krylov method and dimension bound D in {2, 4, 8}) and their
// dispatch by kind.
#include "wide_kernel.hpp"

namespace ctm {

namespace {

template <int OPC, int SOLVER, int D>
hipError_t wide_t(int kind, const WideArgs& w, dim3 grid, size_t smem, hipStream_t s) {
  const dim3 block(kWT), lblock(kWLT);
  switch (kind) {
    case WK_SETUP:
      hipLaunchKernelGGL((wide_setup_kernel<OPC, D>), grid, lblock, smem, s, w);
      break;
    case WK_STEP:
      hipLaunchKernelGGL((wide_step_kernel<OPC, D>), grid, block, smem, s, w);
      break;
    case WK_INIT:
      hipLaunchKernelGGL((wide_init_kernel<OPC, SOLVER, D>), grid, block, smem, s, w);
      break;
    case WK_FIN:
      hipLaunchKernelGGL((wide_fin_kernel<OPC, D>), grid, block, smem, s, w);
      break;
    case WK_FINISH:
      hipLaunchKernelGGL((wide_finish_kernel<OPC>), grid, dim3(64), smem, s, w);
      break;
    case WK_POLL:
      hipLaunchKernelGGL((wide_poll_kernel<OPC, SOLVER>), grid, dim3(64), smem, s, w);
      break;
    default:
      if constexpr (SOLVER == SOLV_BICG) {
        switch (kind) {
          case WK_BA:
            hipLaunchKernelGGL((wide_bicg_a_kernel<OPC, D>), grid, lblock, smem, s, w);
            break;
          case WK_BB:
            hipLaunchKernelGGL((wide_bicg_b_kernel<OPC, D>), grid, block, smem, s, w);
            break;
          case WK_BC:
            hipLaunchKernelGGL((wide_bicg_c_kernel<OPC, D>), grid, lblock, smem, s, w);
            break;
          case WK_BD:
            hipLaunchKernelGGL((wide_bicg_d_kernel<OPC, D>), grid, block, smem, s, w);
            break;
          default:
            return hipErrorInvalidValue;
        }
      } else {
        switch (kind) {
          case WK_CA:
            hipLaunchKernelGGL((wide_cg_a_kernel<OPC, D>), grid, lblock, smem, s, w);
            break;
          case WK_CB:
            hipLaunchKernelGGL((wide_cg_b_kernel<OPC, D>), grid, block, smem, s, w);
            break;
          case WK_CC:
            hipLaunchKernelGGL((wide_cg_c_kernel<OPC, D>), grid, block, smem, s, w);
            break;
          default:
            return hipErrorInvalidValue;
        }
      }
  }
  return hipGetLastError();
}

template <int D>
hipError_t wide_d(int opc, int solver, int kind, const WideArgs& w, dim3 grid, size_t smem,
                  hipStream_t s) {
  const bool cg = (solver == SOLV_CG);
  switch (opc) {
    case OPC_HEAT:
      return cg ? wide_t<OPC_HEAT, SOLV_CG, D>(kind, w, grid, smem, s)
                : wide_t<OPC_HEAT, SOLV_BICG, D>(kind, w, grid, smem, s);
    case OPC_VAR:
      return cg ? wide_t<OPC_VAR, SOLV_CG, D>(kind, w, grid, smem, s)
                : wide_t<OPC_VAR, SOLV_BICG, D>(kind, w, grid, smem, s);
    case OPC_SEP:
      return cg ? hipErrorInvalidValue : wide_t<OPC_SEP, SOLV_BICG, D>(kind, w, grid, smem, s);
    case OPC_DRIFT:
      return cg ? hipErrorInvalidValue
                : wide_t<OPC_DRIFT, SOLV_BICG, D>(kind, w, grid, smem, s);
    default:
      return hipErrorInvalidValue;
  }
}

}  // namespace

hipError_t launch_wide(int opc, int solver, int d, int kind, const WideArgs& w, dim3 grid,
                       int tabmax, hipStream_t s) {
  if (d < 1 || d > MAXD) return hipErrorInvalidValue;
  if (grid.x == 0 || grid.y == 0) return hipSuccess;
  const size_t smem = (size_t)tabmax * sizeof(double);
  if (d <= 2) return wide_d<2>(opc, solver, kind, w, grid, smem, s);
  if (d <= 4) return wide_d<4>(opc, solver, kind, w, grid, smem, s);
  return wide_d<MAXD>(opc, solver, kind, w, grid, smem, s);
}

}  // namespace ctm
