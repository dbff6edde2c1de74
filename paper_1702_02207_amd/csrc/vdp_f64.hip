// Coupled Van der Pol chains, FP64 (the integrator is in vdp_run.h).

#include "vdp_run.h"

namespace osc {

template osc_status vdp_launch<double>(const VdpLaunch<double> &, hipStream_t);

}  // namespace osc
