"""Pins of the oracle's Monte Carlo side: Philox, neighbours, colours, grain-boundary
energy (Sec. 3, Eq. H_1), the Metropolis rule (Eq. metrop_1) and the checkerboard
schedule (Sec. 6), each checked against something other than the oracle itself."""
import itertools
import os

import numpy as np
import pytest

import oracle as O
from conftest import ROOT


def _kat():
    rows = []
    with open(os.path.join(ROOT, "tests", "golden", "philox4x32_10_kat.txt")) as f:
        for line in f:
            if line.startswith("#") or not line.strip():
                continue
            v = [int(t, 16) for t in line.split()]
            rows.append((v[0:4], v[4:6], v[6:10]))
    return rows


@pytest.mark.parametrize("ctr,key,expect", _kat())
def test_philox_known_answers(ctr, key, expect):
    assert list(O.philox4x32_10(ctr, key)) == expect


def test_draw_keying():
    # key = (seed low, seed high), counter = (site, sweep, 0, 0)
    seed = (7 << 32) | 12345
    got = O.draw(seed, 99, 3)
    assert list(got) == list(O.philox4x32_10([99, 3, 0, 0], [12345, 7]))


# --------------------------------------------------------------------------------------
# independent numpy lattice helpers (brute force)
# --------------------------------------------------------------------------------------
def offsets(M):
    if M == 6:
        return [(-1, 0, 0), (1, 0, 0), (0, -1, 0), (0, 1, 0), (0, 0, -1), (0, 0, 1)]
    return [(dx, dy, dz) for dz in (-1, 0, 1) for dy in (-1, 0, 1) for dx in (-1, 0, 1)
            if (dx, dy, dz) != (0, 0, 0)]


def unlike_slots_numpy(K, M, q):
    """Sum over sites and neighbour slots of [q_i != q_n], by array shifts."""
    g = q.reshape(K, K, K)      # [z, y, x]
    tot = 0
    for dx, dy, dz in offsets(M):
        nb = np.roll(g, shift=(-dz, -dy, -dx), axis=(0, 1, 2))
        tot += int(np.count_nonzero(nb != g))
    return tot


@pytest.mark.parametrize("M", [6, 26])
def test_slot_order(M):
    assert [tuple(r) for r in O.slot_offsets(M)] == offsets(M)


@pytest.mark.parametrize("M,K", [(6, 4), (26, 4), (6, 6), (26, 6)])
def test_colouring_no_same_colour_neighbours(M, K):
    col = O.colour_of(K, M).reshape(K, K, K)
    assert col.max() + 1 == O.num_colours(M)
    for dx, dy, dz in offsets(M):
        nb = np.roll(col, shift=(-dz, -dy, -dx), axis=(0, 1, 2))
        assert not np.any(nb == col)
    # equal class sizes
    counts = np.bincount(col.ravel())
    assert np.all(counts == K ** 3 // O.num_colours(M))


@pytest.mark.parametrize("M", [6, 26])
@pytest.mark.parametrize("K,Q", [(4, 3), (4, 5), (2, 3), (6, 4)])
def test_gb_count_equals_full_lattice_energy_difference(M, K, Q):
    """Delta E_gb of every site and every candidate state equals the change of the
    full-lattice unlike-bond energy (each bond once; wrap duplicates at K=2 counted per
    neighbour slot and halved), computed by array shifts."""
    rng = np.random.default_rng(K * 100 + Q + M)
    q = rng.integers(0, Q, size=K ** 3).astype(np.int32)
    H0 = unlike_slots_numpy(K, M, q) / 2
    assert O.unlike_bonds(K, M, q) == H0
    sites = range(K ** 3) if K ** 3 <= 64 else rng.choice(K ** 3, size=48, replace=False)
    for i in sites:
        for qn in range(Q):
            q2 = q.copy()
            q2[i] = qn
            dH = unlike_slots_numpy(K, M, q2) / 2 - H0
            assert O.gb_count(K, M, q, int(i), qn) == dH


def test_neighbour_proposal_slot_mapping():
    K, M, Q = 4, 26, 5
    q = np.arange(K ** 3, dtype=np.int32) % 7
    site = 21
    nbrs = [O.lib().ora_neighbour(K, M, site, k) for k in range(M)]
    for k in range(M):
        # the smallest r0 whose slot is k is ceil(k 2^32 / M)
        r0 = -(-(k << 32) // M)
        assert O.propose(K, M, Q, 0, q, site, r0) == q[nbrs[k]]
        r_hi = -(-((k + 1) << 32) // M) - 1
        assert O.propose(K, M, Q, 0, q, site, r_hi) == q[nbrs[k]]


def test_uniform_proposal_never_current_and_covers_all():
    K, M, Q = 2, 6, 5
    q = np.full(8, 2, np.int32)
    seen = {O.propose(K, M, Q, 1, q, 0, r0) for r0 in np.linspace(0, 2 ** 32 - 1, 4001).astype(np.uint64)}
    assert seen == {0, 1, 3, 4}


# --------------------------------------------------------------------------------------
# exact Boltzmann stationarity by enumeration (K=2, Q=2, uniform proposal, zero load)
# --------------------------------------------------------------------------------------
def _states(n):
    return np.array(list(itertools.product([0, 1], repeat=n)), dtype=np.int32)[:, ::-1].copy()


def _sweep_matrix(M, kT, J=1.0):
    K = 2
    S = _states(8)
    idx = {tuple(s): a for a, s in enumerate(S)}
    col = O.colour_of(K, M)
    P = np.eye(256)
    for c in range(O.num_colours(M)):
        sites = np.nonzero(col == c)[0]
        Pc = np.zeros((256, 256))
        for a, s in enumerate(S):
            pf = []
            for i in sites:
                dE = J * O.gb_count(K, M, s, int(i), int(1 - s[i]))
                pf.append(1.0 if dE <= 0 else np.exp(-dE / kT))
            for flips in itertools.product([0, 1], repeat=len(sites)):
                t = s.copy()
                p = 1.0
                for f, i, pi in zip(flips, sites, pf):
                    if f:
                        t[i] = 1 - t[i]
                        p *= pi
                    else:
                        p *= 1 - pi
                Pc[a, idx[tuple(t)]] += p
        P = P @ Pc
    return S, P


@pytest.mark.parametrize("M", [6, 26])
def test_boltzmann_stationary_by_enumeration(M):
    kT = 1.3
    S, P = _sweep_matrix(M, kT)
    H = np.array([unlike_slots_numpy(2, M, s) / 2 for s in S])
    pi = np.exp(-(H - H.min()) / kT)
    pi /= pi.sum()
    assert np.allclose(P.sum(axis=1), 1.0, atol=1e-14)
    assert np.abs(pi @ P - pi).max() < 1e-12


@pytest.mark.parametrize("M", [6, 26])
def test_philox_chain_matches_boltzmann(M):
    """The oracle's own sweep (Philox draws, integer-threshold Metropolis) sampled over
    many sweeps reproduces pi by a chi-square test on thinned samples.  The temperature
    keeps the chain's second eigenvalue well below one so that thinning is short."""
    from scipy import stats
    kT = 3.0 if M == 6 else 10.0
    S, P = _sweep_matrix(M, kT)
    H = np.array([unlike_slots_numpy(2, M, s) / 2 for s in S])
    pi = np.exp(-(H - H.min()) / kT)
    pi /= pi.sum()
    ev = np.sort(np.abs(np.linalg.eigvals(P)))[::-1]
    thin = max(1, int(np.ceil(np.log(0.01) / np.log(max(ev[1], 1e-9)))))
    K, Q = 2, 2
    prm = O.make_params(K, M, Q, proposal=1, elastic=False, J=1.0, kT=kT, seed=2024 + M)
    q = np.zeros(8, np.int32)
    d = np.zeros(1)
    Ct = np.zeros(36 * Q)
    n_samples = 20000
    hist = np.zeros(256, np.int64)
    weights = 1 << np.arange(8)
    s = 0
    for _ in range(n_samples):
        O.sweeps(prm, q, Ct, Ct, d, np.zeros(6), d, s, thin)
        s += thin
        hist[int(q @ weights)] += 1
    expct = pi * n_samples
    chi2 = ((hist - expct) ** 2 / expct).sum()
    p = stats.chi2.sf(chi2, df=255)
    assert p > 1e-3, (chi2, p, thin)


# --------------------------------------------------------------------------------------
# Gauss-Seidel sweeps (Sec. 6's comparison scheme): the same pins as the checkerboard
# --------------------------------------------------------------------------------------
def _gs_sweep_matrix(M, kT, J=1.0):
    """One sweep visiting sites 0..7 in turn, each a single-site Metropolis step on the
    current state: the product of eight one-site transition matrices."""
    K = 2
    S = _states(8)
    idx = {tuple(s): a for a, s in enumerate(S)}
    P = np.eye(256)
    for i in range(8):
        Pi = np.zeros((256, 256))
        for a, s in enumerate(S):
            dE = J * O.gb_count(K, M, s, i, int(1 - s[i]))
            pf = 1.0 if dE <= 0 else np.exp(-dE / kT)
            t = s.copy()
            t[i] = 1 - t[i]
            Pi[a, idx[tuple(t)]] += pf
            Pi[a, a] += 1 - pf
        P = P @ Pi
    return S, P


@pytest.mark.parametrize("M", [6, 26])
def test_gs_sweep_stationary_by_enumeration(M):
    kT = 1.3
    S, P = _gs_sweep_matrix(M, kT)
    H = np.array([unlike_slots_numpy(2, M, s) / 2 for s in S])
    pi = np.exp(-(H - H.min()) / kT)
    pi /= pi.sum()
    assert np.abs(pi @ P - pi).max() < 1e-12
    # with 2 colours the sequential sweep is a different chain from the checkerboard's; at
    # K=2 each of the 8 colours holds one site, visited in site order, so there they agree
    _, Prb = _sweep_matrix(M, kT)
    if M == 6:
        assert np.abs(P - Prb).max() > 1e-3
    else:
        assert np.abs(P - Prb).max() < 1e-12


@pytest.mark.parametrize("M", [6, 26])
def test_gs_chain_matches_gs_matrix(M):
    """The oracle's Gauss-Seidel sweep (Philox draws) started from one fixed state: the
    empirical distribution after one sweep matches that row of the enumerated one-sweep
    matrix (chi-square over many seeds), so order and immediate writes are as stated."""
    from scipy import stats
    kT = 2.0
    S, P = _gs_sweep_matrix(M, kT)
    start = np.array([0, 1, 1, 0, 1, 0, 0, 1], np.int32)
    a0 = int(start @ (1 << np.arange(8)))
    row = P[a0]
    n = 20000
    hist = np.zeros(256, np.int64)
    for seed in range(n):
        prm = O.make_params(2, M, 2, proposal=1, elastic=False, J=1.0, kT=kT, seed=seed)
        q = start.copy()
        O.gs_sweeps(prm, q, 0, 1)
        hist[int(q @ (1 << np.arange(8)))] += 1
    keep = row * n >= 5
    expct = row[keep] * n
    obs = hist[keep]
    chi2 = ((obs - expct) ** 2 / expct).sum() + (hist[~keep].sum() - row[~keep].sum() * n) ** 2 / max(row[~keep].sum() * n, 1e-9)
    p = stats.chi2.sf(chi2, df=int(keep.sum()))
    assert p > 1e-3, (chi2, p)
    if M != 6:
        return
    # the 2-colour checkerboard's one-sweep row is rejected by the same statistic
    _, Prb = _sweep_matrix(M, kT)
    rb = Prb[a0]
    chi2_rb = ((obs - rb[keep] * n) ** 2 / np.maximum(rb[keep] * n, 1e-9)).sum()
    assert stats.chi2.sf(chi2_rb, df=int(keep.sum())) < 1e-6
