"""Pins of the grain counter used by the grain-growth validation (Sec. 6): closed cases
and a brute-force flood fill on small random lattices."""
from collections import deque

import numpy as np
import pytest

from grains import grain_count, growth_constant, growth_exponent, mean_grain_volume


def coords(K):
    z, y, x = np.meshgrid(np.arange(K), np.arange(K), np.arange(K), indexing="ij")
    return x.ravel(), y.ravel(), z.ravel()


def flood_fill_count(q, K):
    seen = np.zeros(K ** 3, bool)
    n = 0
    for s in range(K ** 3):
        if seen[s]:
            continue
        n += 1
        seen[s] = True
        todo = deque([s])
        while todo:
            i = todo.popleft()
            x, y, z = i % K, (i // K) % K, i // (K * K)
            for dx, dy, dz in ((1, 0, 0), (-1, 0, 0), (0, 1, 0), (0, -1, 0), (0, 0, 1), (0, 0, -1)):
                j = (x + dx) % K + K * (((y + dy) % K) + K * ((z + dz) % K))
                if not seen[j] and q[j] == q[i]:
                    seen[j] = True
                    todo.append(j)
    return n


def test_closed_cases():
    K = 6
    x, y, z = coords(K)
    assert grain_count(np.zeros(K ** 3, np.int32), K) == 1
    assert grain_count((x + y + z) % 2, K) == K ** 3          # no two face neighbours alike
    assert grain_count(x // 2, K) == 3                           # slabs
    assert grain_count(((x + 1) % K) // 2, K) == 3               # a slab across the periodic seam is one grain
    assert grain_count(x // 3, K) == 2
    two = ((x < 2) & (y < 2) & (z < 2)) | ((x >= 3) & (x < 5) & (y >= 3) & (y < 5) & (z >= 3) & (z < 5))
    assert grain_count(two.astype(np.int32), K) == 3             # two separate cubes of one spin + the matrix
    diag = (x == y) & (y == z)                                   # sites touching only along body diagonals
    assert grain_count(diag.astype(np.int32), K) == K + 1
    assert mean_grain_volume(x // 2, K) == K ** 3 / 3


@pytest.mark.parametrize("K,Q,seed", [(3, 2, 0), (4, 3, 1), (5, 2, 2), (5, 4, 3), (7, 3, 4)])
def test_matches_flood_fill(K, Q, seed):
    q = np.random.default_rng(seed).integers(0, Q, K ** 3)
    assert grain_count(q, K) == flood_fill_count(q, K)


def test_growth_fits():
    t = np.array([4.0, 8, 16, 32, 64])
    V = 3.0 * t ** 1.5
    assert abs(growth_exponent(t, V) - 1.5) < 1e-12
    assert abs(growth_constant(t, V) - 3.0 ** (2 / 3)) < 1e-12
