// hmc_zone.hip -- the zone-solve pass launcher: picks the kernel (hmc_zone_kernels.h) for
// the zone size and variant and launches it over the colour's trial list.
#include "hmc_zone_kernels.h"

namespace hmc {

hipError_t launch_zone_pass(hmc_ctx_s* c, int colour, hmc_trial_record* rec)
{
    ZoneArgs a;
    a.spins = c->d.spins;
    a.Ctab = c->d.Ctab;
    a.Stab = c->d.Stab;
    a.sigma = c->d.sigma;
    a.reps = c->d.reps;
    a.list = c->d.list;
    a.count = c->d.counters + kListCount + colour;
    a.acc = c->d.accept;
    a.rec = rec;
    a.stats = c->d.stats;
    a.nonfinite = c->d.counters + kNonFinite;
    a.nr = c->p.zone_steps;
    a.order = c->block_order;
    a.plane = c->total_sites;
    a.alpha = (float)c->p.zone_alpha;
    a.beta = (float)c->p.zone_beta;
    const int h = c->p.zone_h;
    // automatic: lane shifts for h >= 1 (at h = 3, 1.67e6 solves/s against 3.75e5 for a
    // wavefront per trial, 128^3 workload, n_r = 400); node columns for h = 0
    const int v = c->p.zone_variant;
    const bool laneshift = (v == 0 && h >= 1) || v == 3 || v == 4 || v == 5;
    const bool column = !laneshift && ((v == 0 && h <= 2) || v == 2);
    const int tok = prof_begin(c, kProfZone);
    if (laneshift) {
        const int waves = v == 4 ? 2 : v == 5 ? 4 : 1;
        const int tw = h == 1 ? LaneShiftShape<1>::TW : h == 2 ? LaneShiftShape<2>::TW : LaneShiftShape<3>::TW;
        const int per_wg = tw * waves;
        int64_t g = (c->max_list + per_wg - 1) / per_wg;
        // many more work-groups than resident slots: a work-group takes at most a group or
        // two, and the hardware's dispatch balances the tail (measured: 8192 -> 65536
        // work-groups, 5.85 -> 5.72 ms per 128^3 colour launch; a grid of exactly the
        // resident slots with static striding was slower, 6.39 ms)
        const int64_t cap = 65536;
        if (g > cap) g = cap;
        if (g < 1) g = 1;
        const dim3 grid((unsigned)g), block(64 * waves);
#define HMC_LANE(HH, WW) hipLaunchKernelGGL((k_zone_lane<HH, WW>), grid, block, 0, c->stream, a)
        switch (h * 8 + waves) {
            case 9: HMC_LANE(1, 1); break;
            case 10: HMC_LANE(1, 2); break;
            case 12: HMC_LANE(1, 4); break;
            case 17:
            case 18:
            case 20:
                if (launch_zone_lane_h2(waves, grid, block, c->stream, a) != hipSuccess) return hipErrorInvalidValue;
                break;
            case 25:
            case 26:
            case 28:
                if (launch_zone_lane_h3(waves, grid, block, c->stream, a) != hipSuccess) return hipErrorInvalidValue;
                break;
            default: return hipErrorInvalidValue;
        }
#undef HMC_LANE
    } else if (column) {
        const int nn = 2 * h + 2, per_wg = 256 / (nn * nn);
        int64_t g = (c->max_list + per_wg - 1) / per_wg;
        const int64_t cap = 256 * 2 * 4;   // a few resident work-groups per CU
        if (g > cap) g = cap;
        if (g < 1) g = 1;
        const dim3 grid((unsigned)g), block(256);
        switch (h) {
            case 0: hipLaunchKernelGGL(k_zone_col<0>, grid, block, 0, c->stream, a); break;
            case 1: hipLaunchKernelGGL(k_zone_col<1>, grid, block, 0, c->stream, a); break;
            case 2: hipLaunchKernelGGL(k_zone_col<2>, grid, block, 0, c->stream, a); break;
            default: return hipErrorInvalidValue;   // h = 3 does not fit two work-groups per CU

        }
    } else {
        int64_t g = c->max_list;
        if (g > 256 * 40) g = 256 * 40;
        if (g < 1) g = 1;
        const dim3 grid((unsigned)g), block(64);
        switch (h) {
            case 0: hipLaunchKernelGGL(k_zone<0>, grid, block, 0, c->stream, a); break;
            case 1: hipLaunchKernelGGL(k_zone<1>, grid, block, 0, c->stream, a); break;
            case 2: hipLaunchKernelGGL(k_zone<2>, grid, block, 0, c->stream, a); break;
            case 3: hipLaunchKernelGGL(k_zone<3>, grid, block, 0, c->stream, a); break;
            default: return hipErrorInvalidValue;
        }
    }
    prof_end(c, tok);
    return hipGetLastError();
}

}  // namespace hmc
