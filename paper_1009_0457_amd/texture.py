"""Texture measures of Sec. 7 for runs whose orientations are rotations about one axis.

Host-side post-processing of spin fields read back from the library (no lattice work).
With orientations phi = 0, 1, ..., 90 degrees about z and the load along x, cubic symmetry
makes E(phi) = E(90 - phi): 0 and 90 degrees are the softest orientations along x, 45 the
stiffest (Sec. 7, Fig. 2).  A texture is described by the signed deviation of each
orientation from the nearest soft one, in [-45, 45] degrees.

* ``gaussian_density``: the orientation density of Eq. (text_evl), a Gaussian of variance
  parameter g(t) on [-45, 45] normalised by the error function;
* ``fit_g``: g of one texture snapshot by least squares of the measured orientation fractions
  against the density at each orientation's deviation (normalised over the orientations
  present, the discrete form of the Erf normalisation);
* ``fit_variance_law``: tau and beta of g(t) = beta sigma^2 exp(-t / tau), the solution of
  Eq. (varn_eqn), by least squares on log g;
* ``young_x`` / ``young_phi``: the Gaussian fit of x = E / C11 of Eq. (young_gau) and its
  inverse, Eq. (inv_young), which maps orientation densities to Young's-modulus densities.
"""
from __future__ import annotations

import math

import numpy as np

__all__ = ["signed_deviation", "orientation_fractions", "gaussian_density", "fit_g", "fit_variance_law",
           "young_x", "young_phi", "modulus_ratio", "soft_fraction", "mean_abs_deviation",
           "texture_run", "orientation_energy_profile", "single_crystal_energy"]


def signed_deviation(phi_deg):
    """Deviation from the nearest soft orientation (0 or 90 degrees), in [-45, 45]."""
    phi = np.asarray(phi_deg, float)
    return np.where(phi <= 45.0, phi, phi - 90.0)


def orientation_fractions(spins, Q):
    """Volume fraction of each of the Q orientations (one count per site)."""
    c = np.bincount(np.asarray(spins).ravel(), minlength=Q).astype(float)
    return c / c.sum()


def gaussian_density(phi_deg, g):
    """Eq. (text_evl): exp(-phi^2 / 2g^2) / (g sqrt(2 pi) Erf(45 / (sqrt(2) g)))."""
    phi = np.asarray(phi_deg, float)
    return np.exp(-phi ** 2 / (2.0 * g * g)) / (g * math.sqrt(2.0 * math.pi) * math.erf(45.0 / (math.sqrt(2.0) * g)))


def _model_fractions(dev, g):
    f = gaussian_density(dev, g)
    return f / f.sum()


def fit_g(phi_deg, fractions, g_max=1.0e4):
    """Least-squares g of Eq. (text_evl) for one snapshot; returns g_max for a texture that
    is flat (or leans towards the stiff orientations) within the data."""
    from scipy.optimize import minimize_scalar

    dev = signed_deviation(phi_deg)
    F = np.asarray(fractions, float)
    F = F / F.sum()

    def cost(lg):
        return float(((F - _model_fractions(dev, math.exp(lg))) ** 2).sum())

    lo, hi = math.log(0.5), math.log(g_max)
    grid = np.linspace(lo, hi, 200)
    k = int(np.argmin([cost(x) for x in grid]))
    a, b = grid[max(k - 1, 0)], grid[min(k + 1, grid.size - 1)]
    if a == b:
        return math.exp(a)
    r = minimize_scalar(cost, bounds=(a, b), method="bounded", options={"xatol": 1e-10})
    return math.exp(r.x)


def fit_variance_law(t, g, sigma_MPa):
    """tau and beta of g(t) = beta sigma^2 exp(-t/tau) (Eq. varn_eqn's solution) by least
    squares of log g on t.  tau is in the units of t; tau = inf when g does not fall."""
    t = np.asarray(t, float)
    lg = np.log(np.asarray(g, float))
    slope, icpt = np.polyfit(t, lg, 1)
    tau = -1.0 / slope if slope < -1e-12 else math.inf
    return tau, math.exp(icpt) / sigma_MPa ** 2


def young_x(phi_deg, a=0.388, b=16.40, c=0.541):
    """Eq. (young_gau): x = E / C11 = a exp(-(phi - 45)^2 / 2b^2) + c (Sec. 7's constants)."""
    phi = np.asarray(phi_deg, float)
    return a * np.exp(-(phi - 45.0) ** 2 / (2.0 * b * b)) + c


def young_phi(x, a=0.388, b=16.40, c=0.541):
    """Eq. (inv_young): the orientation in [0, 45] degrees with modulus ratio x."""
    x = np.asarray(x, float)
    return 45.0 - np.sqrt(-2.0 * b * b * np.log((x - c) / a))


def modulus_ratio(euler, C=(250.8, 150.0, 123.5), axis=0):
    """x = E / C11 of every orientation along a lab axis (0 = x): E = 1 / S'_aa of the rotated
    compliance, from the library's per-grain tables (Sec. 5, Eq. stiffrot)."""
    from . import hmc as H

    _, S = H.hmc_grain_tables(euler, *C)
    return 1.0 / S[:, axis, axis] / C[0]


def soft_fraction(phi_deg, fractions, within_deg=10.0):
    """Volume fraction within within_deg of a soft orientation."""
    return float(np.asarray(fractions)[np.abs(signed_deviation(phi_deg)) <= within_deg].sum())


def mean_abs_deviation(phi_deg, fractions):
    """Volume-weighted mean |deviation| from the nearest soft orientation (22.75 degrees for
    a flat texture over 0..90 in 1-degree steps)."""
    F = np.asarray(fractions, float)
    return float((np.abs(signed_deviation(phi_deg)) * F).sum() / F.sum())


def texture_run(K=100, runs=10, *, Q=91, coarsen_steps=100, kT=2.6, load_MPa=30.0, substeps=75,
                refresh_steps=200, neighbors=26, zone_h=2, zone_steps=200, lambda_scale=1.0, screen=True,
                record_every=5, C=(250.8, 150.0, 123.5), seed=300, philox_seed=400, profile=False,
                tile_z=0, euler=None, material_points=1, keep_start=False, device="cuda:0"):
    """Sec. 7's texture experiment as one fused batch of ``runs`` replicas on the library.

    Every site starts as an independent random choice among Q orientations (``euler``, Q Bunge
    triples; by default the rotations about z by 0..90 degrees); the lattice
    coarsens for ``coarsen_steps`` sweeps without load; then, for sub-load i = 1..substeps,
    the uniaxial load i/substeps * load_MPa along x is set, the stress field is relaxed to its
    quasi-static state (a cold start of cold_steps the first time, then warm refreshes of
    refresh_steps) and one sweep follows.  ``lambda_scale`` multiplies the elastic-to-MC
    energy scale of every replica; 0 runs the same schedule without any load (the control).
    ``material_points`` = 8 relaxes the stress field with 2 x 2 x 2 material points per
    background cell (the paper's MPM arrangement) instead of one per voxel.

    Returns a dict: t (sweeps since the end of coarsening, every record_every), fractions
    (len(t), runs, Q) volume fractions per orientation, the library's counters, the wall
    time of the loaded phase (seconds, spin read-backs included), with ``profile`` the
    library's kernel times of that phase and with ``keep_start`` the coarsened spins of every
    run (start_spins: a list of K^3 int32 arrays)."""
    import time

    from . import hmc as H
    from .synth import texture_run_inputs

    common = H.hmc_default_params(K, neighbors, zone_h)
    common.zone_steps = zone_steps
    common.refresh_steps = refresh_steps
    common.refresh_every = 1 << 30          # refreshes are explicit, once per sub-load
    common.zone_screen = 1 if screen else 0
    common.C11, common.C12, common.C44 = C
    common.refresh_tile_z = tile_z          # 0: the library's automatic depth
    common.material_points = material_points   # each replica's relaxation constants follow it
    reps = []
    for r in range(runs):
        rep = H.hmc_default_replica(common, K, Q)
        rep.kT = kT
        rep.lambda_el *= lambda_scale
        rep.seed = philox_seed + r
        reps.append(rep)
    b = H.Batch(common, reps, device=device)
    try:
        for r, (eu, q0) in enumerate(texture_run_inputs(K, runs, Q, seed, euler)):
            b.set_replica(r, eu, q0)
        b.sweep(coarsen_steps)

        def snapshot():
            return np.stack([orientation_fractions(b.get_spins(r).cpu().numpy(), Q) for r in range(runs)])

        starts = [b.get_spins(r).cpu().numpy() for r in range(runs)] if keep_start else None
        ts, fr = [0], [snapshot()]
        b.reset_stats()
        if profile:
            b.kernel_times()
            b.set_profiling(True)
        t0 = time.perf_counter()
        for i in range(1, substeps + 1):
            if lambda_scale != 0.0:
                b.set_load([load_MPa * i / substeps, 0.0, 0.0, 0.0, 0.0, 0.0])
                b.stress_refresh(-1, i == 1)
            b.sweep(1)
            if i % record_every == 0 or i == substeps:
                ts.append(i)
                fr.append(snapshot())
        b.synchronize()
        wall = time.perf_counter() - t0
        st = b.stats()
        kt = None
        if profile:
            b.set_profiling(False)
            kt = b.kernel_times()
    finally:
        b.close()
    return {"t": np.array(ts), "fractions": np.array(fr), "stats": st, "wall_s": wall, "kernel_times": kt,
            "start_spins": starts}


def orientation_energy_profile(spins, euler, load_MPa, K, C=(250.8, 150.0, 123.5), n_steps=2000, ckpt_every=50,
                               device="cuda:0"):
    """The elastic driving force of every orientation of a polycrystal under uniaxial tension
    along x, from the adjoint of the global solve (extension 3).

    For orientations that are rotations about z (Bunge (phi, 0, 0)) on an increasing grid of
    phi, the adjoint gives dU/dphi_q summed over the sites of orientation q.  Under stress
    control the envelope identity makes it sum_v 1/2 sigma_v . (dS_q/dphi) sigma_v, so its value
    per site, F_q, is the slope of the orientation's stored energy density w(phi) =
    1/2 sigma . S(phi) sigma as the surrounding polycrystal loads it.  Integrating F over phi
    gives w up to a constant; w_q - <w> (volume-weighted mean) is the energy a site gains by
    taking orientation q, the term that drives the soft orientations' growth in Eqs. (1ddri)
    and (varn_eqn).

    Returns a dict: phi (deg), volume (sites per orientation), F (GPa per rad per site),
    w (GPa per site, relative to the first orientation), D = w - <w> (GPa per site)."""
    from . import hmc as H

    e = np.ascontiguousarray(euler, np.float64)
    if np.any(e[:, 1:] != 0.0) or np.any(np.diff(e[:, 0]) <= 0):
        raise ValueError("orientations must be rotations about z on an increasing grid")
    Q = e.shape[0]
    p = H.hmc_default_params(K, 26, 2)
    p.C11, p.C12, p.C44 = C
    r = H.hmc_default_replica(p, K, Q)
    p.glob_alpha, p.glob_beta, p.glob_alphaE = r.glob_alpha, r.glob_beta, r.glob_alphaE
    lat = H.Lattice(p, Q, device=device)
    try:
        lat.set_spins(np.asarray(spins, np.int32))
        neg = H.orientation_driving_force(lat, e, [load_MPa, 0, 0, 0, 0, 0], n_steps, ckpt_every)
    finally:
        lat.close()
    vol = np.bincount(np.asarray(spins).ravel(), minlength=Q).astype(float)
    F = -neg[:, 0] / np.maximum(vol, 1.0)
    phi = np.degrees(e[:, 0])
    w = np.concatenate([[0.0], np.cumsum(0.5 * (F[1:] + F[:-1]) * np.diff(e[:, 0]))])
    D = w - (vol * w).sum() / vol.sum()
    return {"phi": phi, "volume": vol, "F": F, "w": w, "D": D}


def single_crystal_energy(euler, load_MPa, C=(250.8, 150.0, 123.5), axis=0):
    """1/2 sigma^2 S'_aa of each orientation under uniaxial stress sigma along a lab axis: the
    stored energy density of an isolated crystal (GPa per site), from the library's tables."""
    from . import hmc as H

    _, S = H.hmc_grain_tables(np.ascontiguousarray(euler, np.float64), *C)
    s = load_MPa * 1e-3
    return 0.5 * s * s * S[:, axis, axis]
