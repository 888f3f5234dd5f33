// Instantiation of the chain kernel for one operator class and Krylov method.
#include "chain_kernel.hpp"

namespace ctm {
hipError_t launch_chain_drift_bicg(bool mixed, int shape, const ChainArgs& a, int ntasks,
                                   size_t smem, int tabmax, hipStream_t s) {
  return launch_chain_t<OPC_DRIFT, SOLV_BICG>(mixed, shape, a, ntasks, smem, tabmax, s);
}
}  // namespace ctm
