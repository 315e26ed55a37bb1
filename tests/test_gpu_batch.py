"""GPU tests of fused multi-replica batches and of graph-captured sweeps.

A batch launches every replica's colour pass, zone solves and refresh steps together;
each replica must end exactly where it ends when run alone with the same parameters
(same kernels, same per-replica arithmetic and reduction order), at zero load and with
the elastic term on.  Graph replays must reproduce eager sweeps after every replay.
"""
import sys

import numpy as np
import pytest

import oracle as O
from paper_1009_0457_amd import hmc as H
from paper_1009_0457_amd.synth import voronoi_polycrystal

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():
    pytest.skip("no HIP device", allow_module_level=True)


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def common_params(h=2, R=3, refresh_steps=60):
    p = H.hmc_default_params(16, 26, h)
    p.refresh_every = R
    p.refresh_steps = refresh_steps
    p.cold_steps = 300
    p.zone_steps = 120
    return p


def replica_set(common, n=5, seed=0):
    rng = np.random.default_rng(seed)
    reps, micros = [], []
    for r in range(n):
        K = int((8, 10, 12, 16)[rng.integers(0, 4)])
        m = voronoi_polycrystal(K, int(rng.integers(3, 20)), 100 + r)
        rep = H.hmc_default_replica(common, K, m.Q)
        rep.kT = float(rng.uniform(0.3, 1.0))
        rep.seed = r + 1
        axis = rng.normal(size=3)
        axis /= np.linalg.norm(axis)
        s = 0.0 if r == 2 else float(rng.uniform(50, 300))   # replica 2: zero load
        sig = s * np.outer(axis, axis)
        for i, v in enumerate([sig[0, 0], sig[1, 1], sig[2, 2], sig[1, 2], sig[0, 2], sig[0, 1]]):
            rep.sigma_MPa[i] = v
        reps.append(rep)
        micros.append(m)
    return reps, micros


def run_alone(common, rep, micro, sweeps):
    p = H.hmc_params.from_buffer_copy(common)
    p.K, p.kT, p.lambda_el, p.seed = rep.K, rep.kT, rep.lambda_el, rep.seed
    p.glob_alpha, p.glob_beta, p.glob_alphaE = rep.glob_alpha, rep.glob_beta, rep.glob_alphaE
    lat = H.Lattice(p, micro.Q)
    lat.set_orientations(micro.euler)
    lat.set_spins(micro.spins)
    load = list(rep.sigma_MPa)
    lat.set_load(load)
    elastic = any(v != 0 for v in load)
    if elastic:
        lat.stress_refresh(-1, True)
    lat.sweep(sweeps)
    spins = lat.get_spins().cpu().numpy()
    sig = lat.get_stress().cpu().numpy() if elastic else None
    st = lat.stats()
    lat.close()
    return spins, sig, st


@pytest.mark.parametrize("graphs", [False, True])
def test_batch_equals_replicas_run_alone(graphs):
    common = common_params()
    reps, micros = replica_set(common)
    say(f"[batch] {len(reps)} replicas K={[r.K for r in reps]} graphs={graphs}")
    b = H.Batch(common, reps)
    for r, m in enumerate(micros):
        b.set_replica(r, m.euler, m.spins)
    b.stress_refresh(-1, True)
    if graphs:
        b.set_graphs(True)
    sweeps = 7
    b.sweep(sweeps)
    b.synchronize()
    tot = b.stats()
    for r, (rep, m) in enumerate(zip(reps, micros)):
        spins, sig, st = run_alone(common, rep, m, sweeps)
        got = b.get_spins(r).cpu().numpy()
        say(f"    replica {r}: K={rep.K} changed {int(np.count_nonzero(spins != m.spins))} sites")
        assert np.array_equal(got, spins), r
        if sig is not None:
            assert np.array_equal(b.get_stress(r).cpu().numpy(), sig), r
    assert tot["site_trials"] == sweeps * sum(r.K ** 3 for r in reps)
    b.close()


@pytest.mark.parametrize("K", [112, 128])
def test_explicit_step_tile_heights_agree(K):
    """A 112^3 replica alone runs the forward explicit step on 32 x 16 node tiles (every edge a
    multiple of 16, 784 blocks at depth 4), a 128^3 one on 32 x 32 tiles (512 blocks); batched
    with a 40^3 replica either runs on 32 x 8 tiles.  A tall tile totals each of its 8-row
    groups on its own, so the stress fields and stored energies agree bit for bit, and so do
    the spins and stresses of the sweeps that follow."""
    common = H.hmc_default_params(K, 26, 2)
    common.refresh_every = 2
    common.refresh_steps = 90
    common.cold_steps = 200
    common.zone_steps = 60
    common.refresh_tile_z = 4      # the same tile depth alone and in the batch
    reps, micros = [], []
    for r, (Kr, G) in enumerate(((K, 120), (40, 30))):
        m = voronoi_polycrystal(Kr, G, 200 + r)
        rep = H.hmc_default_replica(common, Kr, m.Q)
        rep.kT, rep.seed = 0.7, 11 + r
        rep.sigma_MPa[0], rep.sigma_MPa[5] = 180.0, -60.0 * (r + 1)
        reps.append(rep)
        micros.append(m)
    say(f"[tile heights] K={[r.K for r in reps]} tile_z=4")
    b = H.Batch(common, reps)
    for r, m in enumerate(micros):
        b.set_replica(r, m.euler, m.spins)
    b.stress_refresh(-1, True)
    sig_b = b.get_stress(0).cpu().numpy()
    e_b = b.energy(0)
    b.sweep(4)
    b.synchronize()
    spins_b, sig_b4 = b.get_spins(0).cpu().numpy(), b.get_stress(0).cpu().numpy()
    b.close()

    p = H.hmc_params.from_buffer_copy(common)
    rep, m = reps[0], micros[0]
    p.K, p.kT, p.lambda_el, p.seed = rep.K, rep.kT, rep.lambda_el, rep.seed
    p.glob_alpha, p.glob_beta, p.glob_alphaE = rep.glob_alpha, rep.glob_beta, rep.glob_alphaE
    lat = H.Lattice(p, m.Q)
    lat.set_orientations(m.euler)
    lat.set_spins(m.spins)
    lat.set_load(list(rep.sigma_MPa))
    lat.stress_refresh(-1, True)
    sig_a, e_a = lat.get_stress().cpu().numpy(), lat.energy()
    lat.sweep(4)
    spins_a, sig_a4 = lat.get_spins().cpu().numpy(), lat.get_stress().cpu().numpy()
    lat.close()
    assert np.array_equal(sig_a, sig_b)
    assert e_a == e_b
    assert np.array_equal(spins_a, spins_b)
    assert np.array_equal(sig_a4, sig_b4)


def test_streamed_explicit_step_equals_cached_step():
    """Four 160^3 replicas together (16.4 M sites: 620 MB of explicit-step arrays, more than
    twice the Infinity Cache) run the explicit step with non-temporal own-node accesses; one
    alone (4.1 M sites) with ordinary ones.  The stress fields and energies agree bit for bit."""
    common = H.hmc_default_params(160, 26, 1)
    common.refresh_steps = 60
    common.cold_steps = 120
    common.refresh_tile_z = 16
    m = voronoi_polycrystal(160, 200, 300)
    reps = []
    for r in range(4):
        rep = H.hmc_default_replica(common, 160, m.Q)
        rep.sigma_MPa[2], rep.sigma_MPa[3] = 150.0, 40.0 * (r + 1)
        reps.append(rep)
    say("[streamed step] 4 x 160^3 batched against the first alone")
    b = H.Batch(common, reps)
    for r in range(4):
        b.set_replica(r, m.euler, m.spins)
    b.stress_refresh(-1, True)
    b.stress_refresh(-1, False)
    sig_b, e_b = b.get_stress(0).cpu().numpy(), b.energy(0)
    b.close()
    p = H.hmc_params.from_buffer_copy(common)
    rep = reps[0]
    p.K, p.kT, p.lambda_el, p.seed = rep.K, rep.kT, rep.lambda_el, rep.seed
    p.glob_alpha, p.glob_beta, p.glob_alphaE = rep.glob_alpha, rep.glob_beta, rep.glob_alphaE
    lat = H.Lattice(p, m.Q)
    lat.set_orientations(m.euler)
    lat.set_spins(m.spins)
    lat.set_load(list(rep.sigma_MPa))
    lat.stress_refresh(-1, True)
    lat.stress_refresh(-1, False)
    sig_a, e_a = lat.get_stress().cpu().numpy(), lat.energy()
    lat.close()
    assert np.array_equal(sig_a, sig_b)
    assert e_a == e_b


@pytest.mark.parametrize("loaded", [False, True])
def test_batch_of_large_replicas_equals_alone(loaded):
    """Four 128^3 replicas fill 1024 chunks per colour pass, so at zero load the batch runs the
    four-sites-per-thread colour pass while each replica alone (256 chunks) runs the
    one-site-per-thread pass; under load both run four per thread, and the batch's fused zone
    and refresh launches must still reproduce each replica alone.  Spins (and stress fields)
    agree bit for bit."""
    common = H.hmc_default_params(128, 26, 1)
    common.refresh_every = 2
    common.refresh_steps = 40
    common.cold_steps = 200
    common.zone_steps = 50
    common.refresh_tile_z = 8      # the same explicit-step tiles alone and in the batch
    reps, micros = [], []
    for r in range(4):
        m = voronoi_polycrystal(128, 300, 60 + r)
        rep = H.hmc_default_replica(common, 128, m.Q)
        rep.kT, rep.seed = 0.6, 30 + r
        if loaded:
            rep.sigma_MPa[r % 3] = 120.0 + 20 * r
        else:
            rep.lambda_el = 0.0
        reps.append(rep)
        micros.append(m)
    say(f"[batch] 4 replicas of 128^3, {'under load' if loaded else 'zero load'}, 3 sweeps")
    b = H.Batch(common, reps)
    for r, m in enumerate(micros):
        b.set_replica(r, m.euler, m.spins)
    if loaded:
        b.stress_refresh(-1, True)
    b.sweep(3)
    b.synchronize()
    for r, (rep, m) in enumerate(zip(reps, micros)):
        spins, sig, st = run_alone(common, rep, m, 3)
        say(f"    replica {r}: changed {int(np.count_nonzero(spins != m.spins))} sites, zone solves {st['zone_solves']}")
        assert (st["zone_solves"] > 0) == loaded
        assert np.array_equal(b.get_spins(r).cpu().numpy(), spins), r
        if loaded:
            assert np.array_equal(b.get_stress(r).cpu().numpy(), sig), r
    b.close()


def test_batch_zero_load_matches_oracle():
    """Zero-load replicas of a batch against the oracle, bit for bit."""
    common = common_params(h=1)
    common.proposal = 1
    reps, micros = [], []
    for r, K in enumerate((6, 10, 8, 12)):
        m = voronoi_polycrystal(K, 5, 40 + r)
        rep = H.hmc_default_replica(common, K, m.Q)
        rep.kT, rep.seed = 0.4 + 0.2 * r, 7 + r
        reps.append(rep)
        micros.append(m)
    b = H.Batch(common, reps)
    for r, m in enumerate(micros):
        b.set_replica(r, m.euler, m.spins)
    b.set_graphs(True)
    b.sweep(6)
    b.synchronize()
    for r, (rep, m) in enumerate(zip(reps, micros)):
        q = m.spins.copy()
        prm = O.make_params(rep.K, 26, m.Q, proposal=1, elastic=False, J=common.J, kT=rep.kT, seed=rep.seed)
        d = np.zeros(1)
        O.sweeps(prm, q, np.zeros(36 * m.Q), np.zeros(36 * m.Q), d, np.zeros(6), d, 0, 6)
        assert np.array_equal(b.get_spins(r).cpu().numpy(), q), r
    b.close()


@pytest.mark.parametrize("material_points,refresh_steps", [(1, 50), (8, 50), (1, 51), (8, 51)])
def test_graph_replays_match_eager_sweeps(material_points, refresh_steps):
    """A single lattice on its own stream: every graph replay (sweeps with and without the
    refresh, the refresh with one material point per voxel or eight per cell, an even and an
    odd number of refresh steps, which leave the displacement in either ping-pong buffer with
    one point per voxel and always in the first with eight) equals the eager sweep, with eager
    work and synchronisation in between."""
    K = 16
    m = voronoi_polycrystal(K, 10, 5)
    p = H.hmc_default_params(K, 26, 1)
    p.refresh_every = 2
    p.refresh_steps = refresh_steps
    p.kT = 0.7
    H.hmc_set_material_points(p, material_points)
    outs = {}
    for mode in ("eager", "graph"):
        s = torch.cuda.Stream()
        lat = H.Lattice(p, m.Q, stream=s)
        with torch.cuda.stream(s):
            lat.set_orientations(m.euler)
            lat.set_spins(m.spins)
            lat.set_load([0, 0, 150.0, 0, 0, 0])
            lat.stress_refresh(300, True)
            if mode == "graph":
                lat.set_graphs(True)
            seq = []
            for k in range(6):
                lat.sweep(1)
                s.synchronize()
                seq.append(lat.get_spins().cpu().numpy())
                s.synchronize()
                _ = lat.energy()        # eager work between replays
            seq.append(lat.get_stress().cpu().numpy())
        outs[mode] = seq
        lat.close()
    for k, (a, b) in enumerate(zip(outs["eager"], outs["graph"])):
        assert np.array_equal(a, b), k



def ensemble(n=None):
    """The 64-replica ensemble (K in {32, 48, 64, 96}, 8 grains per 16^3, uniaxial loads on
    random axes, kT in 0.3-1.0, 26 neighbours, 5^3 zone x 200 steps, refresh every 10)."""
    from paper_1009_0457_amd.synth import batched_configs

    cfgs = batched_configs()[:n] if n else batched_configs()
    micros = [c.microstructure() for c in cfgs]
    common = H.hmc_default_params(16, 26, 2)
    common.refresh_every = cfgs[0].refresh_every
    reps = []
    for c, m in zip(cfgs, micros):
        r = H.hmc_default_replica(common, c.K, m.Q)
        r.kT, r.seed = c.kT, c.philox_seed
        for i in range(6):
            r.sigma_MPa[i] = float(c.sigma_MPa[i])
        reps.append(r)
    return common, cfgs, micros, reps


def test_ensemble_zero_load_twin_matches_oracle():
    """Gate (1) on the whole 64-replica ensemble at zero load (about 20.6 M sites): after two
    fused, graph-replayed sweeps every replica's spins equal the oracle's, bit for bit."""
    from concurrent.futures import ThreadPoolExecutor

    common, cfgs, micros, reps = ensemble()
    for r in reps:
        for i in range(6):
            r.sigma_MPa[i] = 0.0
    b = H.Batch(common, reps)
    for i, m in enumerate(micros):
        b.set_replica(i, m.euler, m.spins)
    say(f"[ensemble zero load] {len(reps)} replicas, {sum(r.K ** 3 for r in reps)} sites, 2 sweeps")
    b.set_graphs(True)
    b.sweep(2)
    got = [b.get_spins(i).cpu().numpy() for i in range(len(reps))]
    b.close()

    def oracle_run(i):
        r, m = reps[i], micros[i]
        q = m.spins.copy()
        prm = O.make_params(r.K, 26, m.Q, proposal=0, elastic=False, J=common.J, kT=r.kT, seed=r.seed)
        d = np.zeros(1)
        O.sweeps(prm, q, np.zeros(36 * m.Q), np.zeros(36 * m.Q), d, np.zeros(6), d, 0, 2)
        return q

    with ThreadPoolExecutor(16) as ex:
        want = list(ex.map(oracle_run, range(len(reps))))
    bad = [i for i in range(len(reps)) if not np.array_equal(got[i], want[i])]
    changed = sum(int(np.count_nonzero(w != m.spins)) for w, m in zip(want, micros))
    say(f"    sites changed by the oracle: {changed}; replicas differing: {bad}")
    assert changed > 0 and not bad


def test_ensemble_under_load_matches_oracle_sampled():
    """The ensemble under load, fused: one colour pass of the first 8 replicas (after a cold
    refresh and two sweeps, the second of which follows a warm refresh) against the oracle fed
    each replica's own snapshot spins and stress field, on a 5 % site sample of each replica:
    proposals, bond counts and draws exact, zone energies within the FP32 tolerance,
    decisions identical outside the near-threshold band."""
    from test_gpu_parity import ZoneErrors, compare_pass, oracle_trials_pooled

    common, cfgs, micros, reps = ensemble(8)
    b = H.Batch(common, reps)
    for i, m in enumerate(micros):
        b.set_replica(i, m.euler, m.spins)
    b.stress_refresh(-1, True)
    b.sweep(2)
    s = b.sweep_index()
    snaps = [b.get_spins(i).cpu().numpy() for i in range(len(reps))]
    sigs = [b.get_stress(i).cpu().numpy().astype(np.float64) for i in range(len(reps))]
    col = 5
    rec = b.colour_pass(col, records=True)
    b.close()
    rng = np.random.default_rng(12)
    errs = ZoneErrors()
    off = 0
    for i, (r, m) in enumerate(zip(reps, micros)):
        K = r.K
        Ct, St, _ = O.tables(m.euler, common.C11, common.C12, common.C44)
        prm = O.make_params(K, 26, m.Q, proposal=0, h=2, nr=common.zone_steps, elastic=True, J=common.J, kT=r.kT,
                            lambda_el=r.lambda_el, zone_alpha=common.zone_alpha, zone_beta=common.zone_beta,
                            seed=r.seed)
        sites = np.nonzero(O.colour_of(K, 26) == col)[0]
        sites = np.sort(rng.choice(sites, size=max(1, sites.size // 20), replace=False))
        ref = oracle_trials_pooled(prm, snaps[i], Ct, St, sigs[i], s, sites)
        rr = rec[off:off + K ** 3]
        tol = errs.add(rr, ref, sites, sigs[i], St, snaps[i])

        class P:   # the replica's decision constants for the comparison
            kT, lambda_el = r.kT, r.lambda_el

        n, k, w = compare_pass(rr, ref, sites, P, tol, f"replica {i} (K={K})")
        errs.flagged += k
        off += K ** 3
    assert errs.report("ensemble replicas 0-7, colour 5") > 200
