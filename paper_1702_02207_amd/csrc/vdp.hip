// Coupled Van der Pol chains, FP32 without a force (the integrator is in
// vdp_run.h); the forced FP32 kernels are in vdp_forced.hip.

#include "vdp_run.h"

namespace osc {

extern template osc_status vdp_launch_as<float, true>(const VdpLaunch<float> &, hipStream_t);
template osc_status vdp_launch_as<float, false>(const VdpLaunch<float> &, hipStream_t);
template osc_status vdp_launch<float>(const VdpLaunch<float> &, hipStream_t);

}  // namespace osc
