"""GPU tests of the zone-kernel selector and the launch-shape autotuner."""
import sys

import numpy as np
import pytest

import oracle as O
from paper_1009_0457_amd import autotune as A
from paper_1009_0457_amd import hmc as H
from paper_1009_0457_amd.synth import voronoi_polycrystal

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():
    pytest.skip("no HIP device", allow_module_level=True)

from test_gpu_parity import compare_pass, oracle_params, zone_tol  # noqa: E402


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def lattice(K, h, tile_z=0, variant=1):
    micro = voronoi_polycrystal(K, 10, 21)
    p = H.hmc_default_params(K, 26, h)
    p.zone_variant = variant
    p.refresh_tile_z = tile_z
    p.kT = 0.8
    p.proposal = 1
    p.zone_steps = 120
    lat = H.Lattice(p, micro.Q)
    lat.set_orientations(micro.euler)
    lat.set_spins(micro.spins)
    lat.set_load([80.0, -60.0, 120.0, 20.0, 0.0, -30.0])
    return p, lat, micro


def test_zone_autotuner_selects_a_kernel_that_matches_the_oracle():
    K = 12
    p, lat, micro = lattice(K, 2)
    lat.stress_refresh(400, True)
    with pytest.raises(H.HmcError):
        lat.set_zone_variant(7)
    res = A.tune_zone_variant(lat, 2, sweeps=1)
    say(f"[autotune zone] {res}")
    assert res["best"] in A.zone_variants_for(2)
    assert all(np.isfinite(v) for v in res["ms_per_solve"].values())
    # the chosen kernel is in use: one colour pass against the oracle
    sig = lat.get_stress().cpu().numpy().astype(np.float64)
    Ct, St, _ = O.tables(micro.euler, p.C11, p.C12, p.C44)
    prm = oracle_params(p, micro.Q, True)
    snap = lat.get_spins().cpu().numpy()
    s = lat.sweep_index()
    rec = lat.colour_pass(3, records=True)
    q = snap.copy()
    ref = O.colour_pass(prm, q, Ct, St, sig, s, 3, want_records=True)
    sites = np.nonzero(O.colour_of(K, 26) == 3)[0]
    tol, _ = zone_tol(sig[:, sites], St, snap[sites], ref["dPi"][sites])
    n, k, w = compare_pass(rec, ref[sites], sites, p, tol, "autotuned kernel")
    say(f"    {n} solves, worst err/tol {w:.3f}")
    assert n > 50
    lat.close()


def test_tile_autotuner_times_every_depth():
    def build(tz):
        return lattice(20, 1, tile_z=tz)[1]

    res = A.tune_tile_depth(build, steps=10)
    say(f"[autotune tile] {res}")
    assert res["best"] in A.TILE_DEPTHS
    assert sorted(int(k) for k in res["ms_per_step"]) == list(A.TILE_DEPTHS)
