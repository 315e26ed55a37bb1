"""Zone size against the exact elastic energy change (Sec. 3, Fig. 1; Sec. 8 on larger
neighbourhoods).

The exact energy change of a trial flip under average-stress control is the change of the
Gibbs energy of the whole periodic lattice at equilibrium, Pi* = U* - K^3 Sigma.E* = -U*
(Hill-Mandel), computed here by two FP64 global solves converged to round-off (before and
after the flip).  The zone solve keeps the traction on the zone's outer boundary fixed, so
the material outside offers no resistance: each larger zone replaces part of that free
boundary by real material, which can only stiffen the response.  Hence the zone energies
rise with h towards the exact value from below, and their error falls; the tests check
both on boundary flips of a small polycrystal, without any reference to the HIP path."""
import numpy as np
import pytest

import oracle as O
from paper_1009_0457_amd.synth import voronoi_polycrystal

NI = (246.5, 147.3, 124.7)
NR = {0: 50, 1: 50, 2: 200, 3: 400}       # zone relaxation steps per half-width


@pytest.fixture(scope="module")
def study():
    K = 12
    m = voronoi_polycrystal(K, 6, 5)
    Ct, St, _ = O.tables(m.euler, *NI)
    q = m.spins.copy()
    Sig = np.array([0.2, 0.0, 0.0, 0.0, 0.0, 0.0])
    _, _, ga, gb, gE = O.solver_defaults(*NI, K, 1)
    u, E, sig, info = O.global_solve(K, q, Ct, St, Sig, 3000, True, ga, gb, gE)
    assert info["res_u"] < 1e-12
    g = q.reshape(K, K, K)
    bnd = np.nonzero((g != np.roll(g, 1, 2)).ravel())[0]
    rng = np.random.default_rng(3)
    rows = []
    for site in rng.choice(bnd, 4, replace=False):
        site = int(site)
        x, y, z = site % K, (site // K) % K, site // (K * K)
        qn = int(g[z, y, (x - 1) % K])
        q2 = q.copy()
        q2[site] = qn
        _, _, _, info2 = O.global_solve(K, q2, Ct, St, Sig, 3000, False, ga, gb, gE, u=u, E=E)
        assert info2["res_u"] < 1e-12
        exact = -(info2["U"] - info["U"])
        zones = []
        for h in range(4):
            za, zb, *_ = O.solver_defaults(*NI, K, h)
            zones.append(O.zone(K, q, Ct, St, site, qn, sig[:, site].copy(), h, NR[h], za, zb))
        scale = 0.5 * sig[:, site] @ St[q[site]] @ sig[:, site]
        rows.append((site, exact, np.array(zones), scale))
    return rows


def test_zone_energies_rise_towards_the_exact_change(study):
    for site, exact, z, scale in study:
        tol = 1e-6 * scale
        assert np.all(np.diff(z) > -tol), (site, z)
        assert z[-1] <= exact + tol, (site, z, exact)


def test_zone_error_falls_with_size(study):
    err = np.array([np.abs(z - exact) / abs(exact) for _, exact, z, _ in study])
    mean = err.mean(0)
    print("relative error of the zone energy, h = 0..3:", np.round(mean, 4))
    assert np.all(np.diff(mean) < 0)
    assert mean[3] < 0.5 * mean[1]
