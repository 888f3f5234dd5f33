// Launchers of the device kernels for the host-only sanitizer build of the
// plan and driver code: every one reports that no device is present. The
// entry points under test never reach a launch on a host without a GPU
// (plan creation stops at its first device allocation), so these only have
// to link.
#include "ctm_internal.h"

namespace ctm {
#define CTM_STUB(...) { return hipErrorNoDevice; }
hipError_t launch_chain(int, int, bool, int, const ChainArgs&, int, size_t, int, hipStream_t) CTM_STUB()
hipError_t launch_stream(int, int, int, const ChainArgs&, int, int, double*, long long, hipStream_t) CTM_STUB()
hipError_t launch_stream_apply(int, int, const GridDev*, int, const double*, double, double, int,
                               const double*, double*, hipStream_t) CTM_STUB()
hipError_t launch_wide(int, int, int, int, const WideArgs&, dim3, int, hipStream_t) CTM_STUB()
hipError_t launch_initial_state(const GridDev*, int, int, int, int, const double*, const double*,
                                double*, hipStream_t) CTM_STUB()
hipError_t launch_mms_initial(const GridDev*, int, int, double, double*, hipStream_t) CTM_STUB()
hipError_t launch_apply(int, int, const GridDev*, int, const double*, double, double, int,
                        const double*, double*, hipStream_t) CTM_STUB()
hipError_t launch_gather(const GridDev*, const int2*, int, int, const double*, const double*,
                         long long, double*, hipStream_t) CTM_STUB()
int gather_stage_capacity() { return 4096; }
hipError_t launch_project(const GridDev*, const long long*, int, long long, const double*, double*,
                          hipStream_t) CTM_STUB()
hipError_t launch_hierarchize(const GridDev*, int, int, bool, bool, const double*, double*,
                              hipStream_t) CTM_STUB()
hipError_t launch_hier_combine(const int*, const int*, const double*, int, const double*, double*,
                               hipStream_t) CTM_STUB()
hipError_t launch_hier_scatter(const int*, long long, const double*, double*, hipStream_t) CTM_STUB()
hipError_t launch_grid_norms2(const GridDev*, int, const double*, double*, hipStream_t) CTM_STUB()
hipError_t launch_residual_max(const int2*, int, const double*, const double*, double*, double*,
                               double*, int, double, const int*, hipStream_t) CTM_STUB()
hipError_t launch_vec_add(VecRef, VecRef, VecRef, int, long long, hipStream_t, const double*) CTM_STUB()
hipError_t launch_class_vec_add(const int2*, int, const GridDev*, VecRef, VecRef, VecRef, int,
                                long long, hipStream_t, const double*) CTM_STUB()
hipError_t launch_fill_zero(double*, long long, hipStream_t, const double*) CTM_STUB()
hipError_t launch_schwarz_setup(int, int, const GridDev*, int, const double*, double, double, int,
                                const SchwarzView&, double*, double*, const int*, long long, int,
                                int*, hipStream_t) CTM_STUB()
hipError_t launch_schwarz_apply(int, int, int, const GridDev*, int, const double*, double, double,
                                int, const SchwarzView&, const double*, double*, double*,
                                long long, hipStream_t) CTM_STUB()
}  // namespace ctm
