"""Launch-shape autotuner for the HMC library.

Two shapes are tunable and independent of each other:

* the zone-solve kernel (``zone_variant``): chosen on a live context by timing one profiled
  sweep per candidate (the sweeps double as warm-up; every variant computes the same solves
  in a different FP32 rounding order, within the zone tolerance);
* the tile depth of the explicit global step (``refresh_tile_z``): fixed when a context is
  created, so candidates are timed on throw-away contexts built by the caller.

Scores are kernel times from the library's HIP-event profiling, normalised per zone solve or
per explicit step, so they do not depend on how many trials happened to be real flips.
"""
from __future__ import annotations

TILE_DEPTHS = (1, 2, 4, 8, 16, 32)


# zone_variant -> (kernel, trials per work-group as a multiple of one wavefront's)
ZONE_SHAPES = {1: ("one wavefront per trial", 1), 2: ("node columns, 256-lane work-group", 1),
               3: ("lane shifts", 1), 4: ("lane shifts", 2), 5: ("lane shifts", 4)}


def zone_variants_for(zone_h: int) -> list[int]:
    """Kernels and work-group shapes the library accepts for this zone half-width (see
    ``hmc_params.zone_variant``): the lane-shift kernel with one, two or four wavefronts (of
    whole trials) per work-group, the node-column kernel and the one-wavefront-per-trial one."""
    out = [1]
    if zone_h <= 2:
        out.append(2)
    if zone_h >= 1:
        out += [3, 4, 5]
    return out


def tune_zone_variant(ctx, zone_h: int, sweeps: int = 1, candidates=None) -> dict:
    """Time ``sweeps`` sweeps of each candidate kernel on ``ctx`` (a Lattice or Batch that is
    ready to sweep) and leave the fastest selected.  Returns {"best": v, "ms_per_solve": {...}}."""
    cands = list(candidates) if candidates is not None else zone_variants_for(zone_h)
    score = {}
    for v in cands:
        ctx.set_zone_variant(v)
        ctx.reset_stats()
        ctx.kernel_times()
        ctx.set_profiling(True)
        ctx.sweep(sweeps)
        ctx.set_profiling(False)
        zt = ctx.kernel_times()["zone"]
        solves = ctx.stats()["zone_solves"]
        score[v] = zt["total_ms"] / solves if solves else float("inf")
    best = min(score, key=score.get)
    ctx.set_zone_variant(best)
    ctx.reset_stats()
    return {"best": best, "ms_per_solve": {str(k): v for k, v in score.items()},
            "shapes": {str(k): {"kernel": ZONE_SHAPES[k][0], "wavefronts_per_group": ZONE_SHAPES[k][1]} for k in score}}


def tune_tile_depth(build, steps: int = 20, depths=TILE_DEPTHS) -> dict:
    """``build(tile_z)`` returns a context with orientations, spins and a load set.  Each is
    cold-started, timed over ``steps`` profiled explicit steps and closed.  Returns
    {"best": tz, "ms_per_step": {...}}."""
    score = {}
    for tz in depths:
        ctx = build(tz)
        try:
            ctx.stress_refresh(steps, True)
            ctx.kernel_times()
            ctx.set_profiling(True)
            ctx.stress_refresh(steps, False)
            ctx.set_profiling(False)
            ks = ctx.kernel_times()["refresh_step"]
            score[tz] = ks["total_ms"] / max(1, ks["launches"])
        finally:
            ctx.close()
    best = min(score, key=score.get)
    return {"best": best, "ms_per_step": {str(k): v for k, v in score.items()}}
