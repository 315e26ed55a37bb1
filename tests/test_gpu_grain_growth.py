"""Grain-growth validation of the checkerboard update at zero load (Sec. 6): a 60^3 lattice
of 99 orientations, random spins, alpha = kT/J = 1.0, ten independent runs.

The ten runs go through the library as one fused batch, their grains counted on the GPU
(hmc_grain_labels); the same runs with the sequential (Gauss-Seidel) update come from the
oracle, counted on the host.  Checks:
* one run of the batch equals the oracle's checkerboard run bit for bit at every sample time;
* both schemes follow a power law V ~ t^m with m near the isotropic value 3/2 and with the
  same exponent and growth constant c2 (V^(2/3) = c2 t) within the stated bands.
The measured numbers are printed.
"""
import os
import sys
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest

import oracle as O
from grains import growth_constant, growth_exponent, mean_grain_volume
from paper_1009_0457_amd import hmc as H
from paper_1009_0457_amd.synth import haar_euler, random_spins

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():
    pytest.skip("no HIP device", allow_module_level=True)

K, Q, KT, RUNS = 60, 99, 1.0, 10
TIMES = [4, 8, 16, 32, 64, 128]
FIT = slice(1, None)            # t = 8 .. 128


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def initial(r):
    return random_spins(K, Q, 7000 + r), haar_euler(np.random.default_rng(8000 + r), Q)


def gs_run(M, r):
    q = initial(r)[0]
    prm = O.make_params(K, M, Q, proposal=0, elastic=False, J=1.0, kT=KT, seed=9000 + r)
    V, s = [], 0
    for t in TIMES:
        O.gs_sweeps(prm, q, s, t - s)
        s = t
        V.append(mean_grain_volume(q, K))
    return V


@pytest.mark.parametrize("M,m_band", [(26, (1.15, 1.6)), (6, (0.95, 1.6))])
def test_grain_growth_checkerboard_vs_sequential(M, m_band):
    say(f"[grain growth] K={K} Q={Q} M={M} kT/J={KT} runs={RUNS}")
    common = H.hmc_default_params(K, M, 1)
    common.proposal = 0
    common.J = 1.0
    reps = []
    for r in range(RUNS):
        rep = H.hmc_default_replica(common, K, Q)
        rep.kT, rep.lambda_el, rep.seed = KT, 0.0, 9000 + r
        reps.append(rep)
    b = H.Batch(common, reps)
    for r in range(RUNS):
        q0, eu = initial(r)
        b.set_replica(r, eu, q0)
    V_rb = np.zeros((RUNS, len(TIMES)))
    snaps0 = []
    s = 0
    for j, t in enumerate(TIMES):
        b.sweep(t - s)
        s = t
        for r in range(RUNS):
            _, n = b.grain_labels(r)             # counted on the GPU
            V_rb[r, j] = K ** 3 / n
            if r == 0:
                q = b.get_spins(r).cpu().numpy()
                snaps0.append(q)
                assert K ** 3 / n == mean_grain_volume(q, K)
    b.close()
    say("    checkerboard (library) mean V:", " ".join(f"{v:.1f}" for v in V_rb.mean(0)))

    # sampled parity: run 0 against the oracle's checkerboard sweeps at every sample time
    q = initial(0)[0]
    prm = O.make_params(K, M, Q, proposal=0, elastic=False, J=1.0, kT=KT, seed=9000)
    d = np.zeros(1)
    Ct = np.zeros(36 * Q)
    s = 0
    for t, got in zip(TIMES, snaps0):
        O.sweeps(prm, q, Ct, Ct, d, np.zeros(6), d, s, t - s)
        s = t
        assert np.array_equal(got, q), f"run 0 differs from the oracle at t={t}"
    say("    run 0 bit-exact against the oracle at every sample time")

    with ThreadPoolExecutor(max_workers=min(RUNS, os.cpu_count() or 1, 16)) as ex:
        V_gs = np.array(list(ex.map(lambda r: gs_run(M, r), range(RUNS))))
    say("    sequential (oracle) mean V:     ", " ".join(f"{v:.1f}" for v in V_gs.mean(0)))

    t = np.array(TIMES, float)[FIT]
    m_rb = np.array([growth_exponent(t, v[FIT]) for v in V_rb])
    m_gs = np.array([growth_exponent(t, v[FIT]) for v in V_gs])
    c_rb = np.array([growth_constant(t, v[FIT]) for v in V_rb])
    c_gs = np.array([growth_constant(t, v[FIT]) for v in V_gs])
    se = lambda a: a.std(ddof=1) / np.sqrt(a.size)
    say(f"    exponent m: checkerboard {m_rb.mean():.3f} +- {se(m_rb):.3f}, sequential {m_gs.mean():.3f} +- {se(m_gs):.3f}")
    say(f"    c2: checkerboard {c_rb.mean():.4f} +- {se(c_rb):.4f}, sequential {c_gs.mean():.4f} +- {se(c_gs):.4f}, "
        f"ratio {c_rb.mean() / c_gs.mean():.3f}")
    lo, hi = m_band
    assert lo < m_rb.mean() < hi and lo < m_gs.mean() < hi
    assert abs(m_rb.mean() - m_gs.mean()) < 0.12
    assert 0.85 < c_rb.mean() / c_gs.mean() < 1.18
    assert np.all(np.diff(V_rb.mean(0)) > 0) and np.all(np.diff(V_gs.mean(0)) > 0)
