// hmc_zone_h2.hip -- the lane-shift zone solve for h = 2 (5^3 voxels), the workloads' zone
// size, in a translation unit of its own: the build schedules it with the AMDGPU
// register-pressure trackers (the same instructions in another order, 254 registers, no
// spills; 128^3 workload: 5.62 -> 5.24 ms per colour launch); it slows the h = 1 instance,
// which keeps the options of hmc_zone.hip, and the h = 3 one, which has a unit of its own.
#include "hmc_zone_kernels.h"

namespace hmc {

hipError_t launch_zone_lane_h2(int waves, dim3 grid, dim3 block, hipStream_t stream, const ZoneArgs& a)
{
    switch (waves) {
        case 1: hipLaunchKernelGGL((k_zone_lane<2, 1>), grid, block, 0, stream, a); return hipSuccess;
        case 2: hipLaunchKernelGGL((k_zone_lane<2, 2>), grid, block, 0, stream, a); return hipSuccess;
        case 4: hipLaunchKernelGGL((k_zone_lane<2, 4>), grid, block, 0, stream, a); return hipSuccess;
        default: return hipErrorInvalidValue;   // (a launch error is left for the caller's hipGetLastError)
    }
}

}  // namespace hmc
