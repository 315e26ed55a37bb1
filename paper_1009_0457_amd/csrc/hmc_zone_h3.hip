// hmc_zone_h3.hip -- the lane-shift zone solve for h = 3 (7^3 voxels) in a translation unit of
// its own: the build schedules it with the iterative maximum-occupancy strategy (the same
// instructions in another order; 128^3 workload, 400 relaxation steps: 37.4 -> 35.6 ms per
// colour launch), which the other zone sizes do not gain from.
#include "hmc_zone_kernels.h"

namespace hmc {

hipError_t launch_zone_lane_h3(int waves, dim3 grid, dim3 block, hipStream_t stream, const ZoneArgs& a)
{
    switch (waves) {
        case 1: hipLaunchKernelGGL((k_zone_lane<3, 1>), grid, block, 0, stream, a); return hipSuccess;
        case 2: hipLaunchKernelGGL((k_zone_lane<3, 2>), grid, block, 0, stream, a); return hipSuccess;
        case 4: hipLaunchKernelGGL((k_zone_lane<3, 4>), grid, block, 0, stream, a); return hipSuccess;
        default: return hipErrorInvalidValue;   // (a launch error is left for the caller's hipGetLastError)
    }
}

}  // namespace hmc
