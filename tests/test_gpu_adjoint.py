"""GPU tests of the hand-written adjoint of the global explicit elastic solve.

* Against FP64 central differences of the oracle's n-step stored energy (h = 1e-4 rad,
  1e-3 MPa) on a lattice small enough for the oracle, with a step count far from
  convergence (so the recurrence itself, not only its fixed point, is differentiated) and
  a checkpoint interval that does not divide it.
* At the 64^3 / 500-grain / 2000-step workload, where the relaxation has converged, the
  envelope identities dU*/dtheta_g = -sum_{v in g} 1/2 eps_v.(dC_g/dtheta) eps_v and
  dU*/dSigma = K^3 E* hold at any size and are checked on the GPU's own final state.
"""
import sys

import numpy as np
import pytest

import oracle as O
from paper_1009_0457_amd import hmc as H
from paper_1009_0457_amd.synth import adjoint_config, voronoi_polycrystal

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():
    pytest.skip("no HIP device", allow_module_level=True)


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def oracle_U(K, q, euler, sig_MPa, p, n):
    Ct, St, _ = O.tables(euler, p.C11, p.C12, p.C44)
    _, _, _, info = O.global_solve(K, q, Ct, St, np.asarray(sig_MPa) * 1e-3, n, True, p.glob_alpha, p.glob_beta,
                                   p.glob_alphaE)
    return info["U"]


@pytest.mark.parametrize("tile_z", [0, 8])
def test_adjoint_matches_oracle_central_differences(tile_z):
    """tile_z 0 (automatic: one node layer per block at this size) and 8 (two blocks in z,
    the second cut short by the lattice edge)."""
    K, n, every = 12, 100, 30
    m = voronoi_polycrystal(K, 14, 77)
    rng = np.random.default_rng(3)
    sig = rng.uniform(-200, 200, 6)
    p = H.hmc_default_params(K, 26, 1)
    p.refresh_tile_z = tile_z
    lat = H.Lattice(p, m.Q)
    lat.set_orientations(m.euler)
    lat.set_spins(m.spins)
    lat.set_load(sig)
    U_gpu = lat.elastic_forward(n, every)
    ge, gs = lat.elastic_backward(1.0)
    U_ora = oracle_U(K, m.spins, m.euler, sig, p, n)
    say(f"[adjoint FD] U gpu {U_gpu:.8e} oracle {U_ora:.8e}")
    assert U_gpu == pytest.approx(U_ora, rel=1e-5)
    h = 1e-4
    grains = rng.choice(m.Q, size=10, replace=False)
    worst = 0.0
    scale = np.abs(ge).max()
    for g in grains:
        for k in range(3):
            ep, em = m.euler.copy(), m.euler.copy()
            ep[g, k] += h
            em[g, k] -= h
            fd = (oracle_U(K, m.spins, ep, sig, p, n) - oracle_U(K, m.spins, em, sig, p, n)) / (2 * h)
            err = abs(ge[g, k] - fd)
            worst = max(worst, err / scale)
            assert err <= 2e-4 * scale + 1e-4 * abs(fd), (g, k, ge[g, k], fd)
    hs = 1e-3
    gscale = np.abs(gs).max()
    for I in range(6):
        sp, sm = sig.copy(), sig.copy()
        sp[I] += hs
        sm[I] -= hs
        fd = (oracle_U(K, m.spins, m.euler, sp, p, n) - oracle_U(K, m.spins, m.euler, sm, p, n)) / (2 * hs)
        assert abs(gs[I] - fd) <= 2e-4 * gscale + 1e-4 * abs(fd), (I, gs[I], fd)
    say(f"    worst |adjoint - FD| / max|grad| over 30 angles: {worst:.2e}")
    # the context is left at the forward's final state
    s1 = lat.get_stress().cpu().numpy()
    lat.elastic_forward(n, every)
    assert np.array_equal(lat.get_stress().cpu().numpy(), s1)
    lat.close()


def test_adjoint_envelope_identity_at_workload_size():
    micro, sig, probe = adjoint_config()
    K = micro.K
    p = H.hmc_default_params(K, 26, 2)
    lat = H.Lattice(p, micro.Q)
    lat.set_orientations(micro.euler)
    lat.set_spins(micro.spins)
    lat.set_load(sig)
    say(f"[adjoint envelope] K={K} grains={micro.Q} 2000 steps, checkpoints every 50")
    U = lat.elastic_forward(2000, 50)
    ge, gs = lat.elastic_backward(1.0)
    s = lat.get_stress().cpu().numpy().astype(np.float64)
    E = lat.macro_strain()
    Cl, Sl = H.hmc_grain_tables(micro.euler, p.C11, p.C12, p.C44)
    dC, _ = H.hmc_grain_table_derivatives(micro.euler, p.C11, p.C12, p.C44)
    q = micro.spins
    eps = np.einsum("nij,jn->in", Sl[q], s)                    # eps_v = S_q sigma_v
    # -1/2 eps . dC eps summed per grain
    contrib = -0.5 * np.einsum("in,nkij,jn->nk", eps, dC[q], eps)
    env = np.zeros((micro.Q, 3))
    np.add.at(env, q, contrib)
    scale = np.abs(env).max()
    err = np.abs(ge - env).max()
    say(f"    U = {U:.6e}; max |adjoint - envelope| / max|grad| = {err / scale:.2e}")
    assert err <= 1e-3 * scale
    # probe grains as in the workload description
    assert np.allclose(ge[probe], env[probe], rtol=2e-3, atol=1e-3 * scale)
    env_sig = K ** 3 * E * 1e-3          # dU*/dSigma = K^3 E* (per MPa)
    assert np.abs(gs - env_sig).max() <= 1e-3 * np.abs(env_sig).max()
    lat.close()


def test_autograd_function_matches_direct_adjoint():
    K, n = 10, 60
    m = voronoi_polycrystal(K, 6, 5)
    p = H.hmc_default_params(K, 26, 1)
    lat = H.Lattice(p, m.Q)
    lat.set_orientations(m.euler)
    lat.set_spins(m.spins)
    sig = np.array([100.0, -50.0, 80.0, 10.0, 0.0, 20.0])
    lat.set_load(sig)
    lat.elastic_forward(n, 25)
    ge, gs = lat.elastic_backward(2.5)
    eu = torch.tensor(m.euler, dtype=torch.float64, requires_grad=True)
    st = torch.tensor(sig, dtype=torch.float64, requires_grad=True)
    U = H.stored_elastic_energy(eu, st, lat, n_steps=n, ckpt_every=25)
    (2.5 * U).backward()
    assert np.array_equal(eu.grad.numpy(), ge)
    assert np.array_equal(st.grad.numpy(), gs)
    lat.close()


def test_checkpoint_interval_does_not_change_the_gradient():
    """The explicit steps carry (E, wE) from one step to the next inside a sequence and through
    the context's state between sequences (one per checkpoint segment, and per recomputed
    segment); both routes use the same arithmetic, so the gradient is bit-identical for any
    checkpoint interval, including one step per segment."""
    K, n = 12, 40
    m = voronoi_polycrystal(K, 10, 8)
    sig = np.array([90.0, -30.0, 60.0, 20.0, -10.0, 40.0])
    out = []
    for every in (1, 7, 40):
        p = H.hmc_default_params(K, 26, 1)
        lat = H.Lattice(p, m.Q)
        lat.set_orientations(m.euler)
        lat.set_spins(m.spins)
        lat.set_load(sig)
        U = lat.elastic_forward(n, every)
        ge, gs = lat.elastic_backward(1.0)
        out.append((U, ge, gs))
        lat.close()
    for U, ge, gs in out[1:]:
        assert U == out[0][0]
        assert np.array_equal(ge, out[0][1])
        assert np.array_equal(gs, out[0][2])



def test_forward_record_is_discarded_by_state_changes():
    """The backward pass recomputes segments from the forward's checkpoints with the context's
    current spins, stiffness tables and load; any change of those after the forward must make
    the backward refuse (HMC_ESTATE) rather than return a gradient of other inputs.  A second
    backward of the same forward is allowed.  Through autograd, two energies evaluated on one
    lattice before a backward raise instead of both using the last forward's checkpoints."""
    K, n, every = 10, 40, 10
    m = voronoi_polycrystal(K, 6, 12)
    sig = np.array([80.0, -40.0, 120.0, 15.0, -25.0, 30.0])
    p = H.hmc_default_params(K, 26, 1)
    lat = H.Lattice(p, m.Q)
    lat.set_orientations(m.euler)
    lat.set_spins(m.spins)
    lat.set_load(sig)
    for change in ("orientations", "spins", "load", "sweep", "colour pass"):
        say(f"[adjoint record] change: {change}")
        lat.elastic_forward(n, every)
        g1 = lat.elastic_backward(1.0)
        g2 = lat.elastic_backward(1.0)
        assert np.array_equal(g1[0], g2[0]) and np.array_equal(g1[1], g2[1])
        if change == "orientations":
            lat.set_orientations(m.euler)
        elif change == "spins":
            lat.set_spins(m.spins)
        elif change == "load":
            lat.set_load(sig)
        elif change == "sweep":
            lat.sweep(1)
        else:
            lat.colour_pass(3)
        with pytest.raises(H.HmcError) as e:
            lat.elastic_backward(1.0)
        assert e.value.status == H.HMC_ESTATE
    lat.set_spins(m.spins)
    st = torch.tensor(sig, dtype=torch.float64, requires_grad=True)
    e1 = torch.tensor(m.euler, dtype=torch.float64, requires_grad=True)
    e2 = torch.tensor(m.euler + 0.01, dtype=torch.float64, requires_grad=True)
    U = H.stored_elastic_energy(e1, st, lat, n_steps=n, ckpt_every=every) + \
        H.stored_elastic_energy(e2, st, lat, n_steps=n, ckpt_every=every)
    with pytest.raises(RuntimeError, match="another forward"):
        U.backward()
    # one energy per lattice per backward still works
    e3 = torch.tensor(m.euler, dtype=torch.float64, requires_grad=True)
    H.stored_elastic_energy(e3, st, lat, n_steps=n, ckpt_every=every).backward()
    assert torch.isfinite(e3.grad).all() and e3.grad.abs().max() > 0
    lat.close()


def test_adjoint_matches_oracle_central_differences_at_workload_size():
    """The adjoint workload itself (64^3, 500 grains, six stress components, a cold start and
    2000 explicit steps, checkpoints every 50) against FP64 central differences of the oracle's
    stored energy for the 10 probe grains' 30 Euler angles and the 6 stress components
    (h = 1e-4 rad, 1e-3 MPa), written by tests/golden/make_adjoint_fd.py from the oracle alone."""
    from conftest import golden

    g = golden("adjoint64_fd.txt")
    micro, sig, probe = adjoint_config()
    K = micro.K
    p = H.hmc_default_params(K, 26, 2)
    assert int(g["steps"]) == 2000
    assert p.glob_alpha == g["glob_alpha"] and p.glob_beta == g["glob_beta"]
    lat = H.Lattice(p, micro.Q)
    lat.set_orientations(micro.euler)
    lat.set_spins(micro.spins)
    lat.set_load(sig)
    say(f"[adjoint FD 64^3] K={K} grains={micro.Q} 2000 steps, checkpoints every 50")
    U = lat.elastic_forward(2000, 50)
    ge, gs = lat.elastic_backward(1.0)
    lat.close()
    assert U == pytest.approx(g["U"], rel=1e-5)
    scale = np.abs(ge).max()
    worst = 0.0
    for q in probe:
        for k in range(3):
            fd = g[f"dU_dtheta_{int(q)}_{k}"]
            err = abs(ge[q, k] - fd)
            worst = max(worst, err / scale)
            assert err <= 2e-4 * scale + 1e-4 * abs(fd), (int(q), k, ge[q, k], fd)
    gscale = np.abs(gs).max()
    worst_s = 0.0
    for i in range(6):
        fd = g[f"dU_dSigma_{i}"]
        worst_s = max(worst_s, abs(gs[i] - fd) / gscale)
        assert abs(gs[i] - fd) <= 2e-4 * gscale + 1e-4 * abs(fd), (i, gs[i], fd)
    say(f"    U gpu {U:.8e} oracle {g['U']:.8e}; worst |adjoint - FD| / max|grad|: angles {worst:.2e}, "
        f"stress {worst_s:.2e}")
