"""hmc_texture_histogram_noalloc (no context, no workspace: its scratch is a static device array)
against hmc_texture_histogram on a context holding the same spins and orientations, through the
C ABI: two calls in a row, the second on a smaller lattice with fewer grains, so that the
second call runs over the scratch array the first one left behind.  Integer counts: bit-exact."""
import sys

import numpy as np
import pytest

from paper_1009_0457_amd import hmc as H
from paper_1009_0457_amd.synth import voronoi_polycrystal

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

if not torch.cuda.is_available():
    pytest.skip("no HIP device", allow_module_level=True)


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def context_histogram(m, axis, width, nbins):
    p = H.hmc_default_params(m.K, 26, 1)
    p.lambda_el = 0.0
    lat = H.Lattice(p, m.Q)
    lat.set_orientations(m.euler)
    lat.set_spins(m.spins)
    out = lat.texture_histogram(axis, width, nbins)
    lat.close()
    return out


def test_noalloc_histogram_matches_context_histogram():
    stream = torch.cuda.Stream()
    cases = [(64, 500, 41, [1.0, 0.0, 0.0], 10.0, 6), (20, 37, 42, [0.3, -0.2, 0.9], 5.0, 11)]
    for K, ng, seed, axis, width, nbins in cases:
        say(f"[no-alloc texture] K={K} grains={ng} axis={axis} bins={nbins} x {width} deg")
        m = voronoi_polycrystal(K, ng, seed)
        spins = torch.from_numpy(m.spins).to("cuda")
        torch.cuda.synchronize()
        got = H.hmc_texture_histogram_noalloc(spins, K, m.euler, axis, width, nbins, stream.cuda_stream)
        want = context_histogram(m, axis, width, nbins)
        say(f"    {got.tolist()}")
        assert np.array_equal(got, want)
        assert got.sum() == K ** 3


def test_noalloc_histogram_rejects_what_does_not_fit():
    m = voronoi_polycrystal(8, 5, 3)
    bad = m.spins.copy()
    bad[7] = m.Q
    with pytest.raises(H.HmcError) as e:
        H.hmc_texture_histogram_noalloc(torch.from_numpy(bad).to("cuda"), 8, m.euler, [0, 0, 1.0], 10.0, 6, 0)
    assert e.value.status == H.HMC_EINVAL
    big = np.zeros((32768, 3))
    with pytest.raises(H.HmcError) as e:
        H.hmc_texture_histogram_noalloc(torch.from_numpy(m.spins).to("cuda"), 8, big, [0, 0, 1.0], 10.0, 6, 0)
    assert e.value.status == H.HMC_ESHAPE
    # a valid call after the rejected ones still counts from zero
    got = H.hmc_texture_histogram_noalloc(torch.from_numpy(m.spins).to("cuda"), 8, m.euler, [0, 0, 1.0], 10.0, 6, 0)
    assert np.array_equal(got, context_histogram(m, [0, 0, 1.0], 10.0, 6))
