// Van der Pol chain entry points beside vdp_launch (osc_internal.h): the
// resident real-time kernel (resident.hip).

#pragma once

#include <cstdint>

#include "osc_internal.h"

namespace osc {

// one kernel for a whole periodic run of Van der Pol chains (s <= 1024),
// released tick by tick as the free and driven resident kernels are
template <typename T>
osc_status vdp_resident_launch(const VdpLaunch<T> &a, const ResidentRun<T> &r, hipStream_t st);
// its workgroups (0 when s is beyond the register layouts)
template <typename T>
int64_t vdp_resident_blocks(const VdpLaunch<T> &a);

}  // namespace osc
