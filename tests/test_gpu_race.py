"""Race detection: the results must not depend on which work-group takes which part of a
launch, or when.  hmc_set_block_order reverses or shuffles the logical block order of the
colour-pass, zone-solve and explicit-step launches (forward and adjoint); sweeps, refreshes,
statistics and gradients must come out bit-identical under every order.  A kernel that read a
spin some other work-group of the same pass had already overwritten, or that summed floating
point across work-groups in arrival order, would fail this."""
import sys

import numpy as np
import pytest

from paper_1009_0457_amd import hmc as H
from paper_1009_0457_amd.synth import full_config, voronoi_polycrystal

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():
    pytest.skip("no HIP device", allow_module_level=True)


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def test_elastic_sweeps_do_not_depend_on_block_order():
    c = full_config()
    m = c.microstructure()
    outs = []
    for order in (0, 1, 2):
        p = H.hmc_default_params(c.K, c.neighbors, c.zone_h)
        p.kT, p.refresh_every = c.kT, c.refresh_every
        lat = H.Lattice(p, m.Q)
        lat.set_block_order(order)
        lat.set_orientations(m.euler)
        lat.set_spins(m.spins)
        lat.set_load(c.sigma_MPa)
        lat.stress_refresh(400, True)
        lat.sweep(3)
        bonds, U = lat.energy()
        outs.append((lat.get_spins().cpu().numpy(), lat.get_stress().cpu().numpy(), lat.stats(), bonds, U))
        lat.close()
    say(f"[block order] 64^3 elastic, 3 sweeps: solves {outs[0][2]['zone_solves']}, accepted {outs[0][2]['accepted']}")
    for o in outs[1:]:
        assert np.array_equal(o[0], outs[0][0]) and np.array_equal(o[1], outs[0][1])
        assert o[2] == outs[0][2] and o[3] == outs[0][3] and o[4] == outs[0][4]


@pytest.mark.parametrize("neighbors", [6, 26])
def test_batch_and_zero_load_passes_do_not_depend_on_block_order(neighbors):
    """A batch of replicas of different sizes, zero load and loaded, in one launch per pass."""
    common = H.hmc_default_params(16, neighbors, 1)
    common.refresh_every = 2
    common.refresh_steps = 60
    specs = [(16, 0.0), (24, 120.0), (12, 0.0), (32, 80.0)]
    micros = [voronoi_polycrystal(K, 9, 40 + K) for K, _ in specs]
    outs = []
    for order in (0, 1, 2):
        reps = []
        for (K, s), m in zip(specs, micros):
            r = H.hmc_default_replica(common, K, m.Q)
            r.kT, r.seed = 0.8, K
            r.sigma_MPa[2] = s
            reps.append(r)
        b = H.Batch(common, reps)
        b.set_block_order(order)
        for i, m in enumerate(micros):
            b.set_replica(i, m.euler, m.spins)
        b.stress_refresh(200, True)
        b.sweep(4)
        outs.append([b.get_spins(i).cpu().numpy() for i in range(len(reps))] + [b.stats()])
        b.close()
    for o in outs[1:]:
        for i in range(len(specs)):
            assert np.array_equal(o[i], outs[0][i]), i
        assert o[-1] == outs[0][-1]


def test_adjoint_does_not_depend_on_block_order():
    K, n = 12, 60
    m = voronoi_polycrystal(K, 8, 3)
    sig = np.array([60.0, -90.0, 120.0, 10.0, 30.0, -20.0])
    outs = []
    for order in (0, 1, 2):
        p = H.hmc_default_params(K, 26, 1)
        lat = H.Lattice(p, m.Q)
        lat.set_block_order(order)
        lat.set_orientations(m.euler)
        lat.set_spins(m.spins)
        lat.set_load(sig)
        U = lat.elastic_forward(n, 7)
        ge, gs = lat.elastic_backward(1.0)
        outs.append((U, ge, gs))
        lat.close()
    for o in outs[1:]:
        assert o[0] == outs[0][0] and np.array_equal(o[1], outs[0][1]) and np.array_equal(o[2], outs[0][2])
    with pytest.raises(H.HmcError):
        H.Lattice(H.hmc_default_params(8, 26, 1), 2).set_block_order(3)
