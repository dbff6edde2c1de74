// Coupled Van der Pol chains, FP32 with a harmonic force (the integrator is
// in vdp_run.h).

#include "vdp_run.h"

namespace osc {

template osc_status vdp_launch_as<float, true>(const VdpLaunch<float> &, hipStream_t);

}  // namespace osc
