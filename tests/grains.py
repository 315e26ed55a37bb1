"""Grain statistics for the grain-growth validation of Sec. 6 (test infrastructure).

A grain is a face-connected cluster of equal spins on the periodic lattice (site index
x + K*(y + K*z)); the mean grain volume is K^3 over the number of grains.  The growth law of
Sec. 6 (mean radius ~ t^(1/n), n = 2) makes V^(2/3) linear in t, i.e. V ~ t^(3/2)."""
import numpy as np
from scipy.sparse import coo_matrix
from scipy.sparse.csgraph import connected_components


def grain_count(spins, K):
    return int(grain_labels(spins, K).max()) + 1


def grain_labels(spins, K):
    """Component index (0..n-1, scipy's numbering) of every site."""
    g = np.asarray(spins).reshape(K, K, K)          # [z, y, x]
    idx = np.arange(K ** 3).reshape(K, K, K)
    rows, cols = [], []
    for ax in range(3):
        same = g == np.roll(g, -1, axis=ax)
        rows.append(idx[same])
        cols.append(np.roll(idx, -1, axis=ax)[same])
    r = np.concatenate(rows)
    c = np.concatenate(cols)
    A = coo_matrix((np.ones(r.size, np.int8), (r, c)), shape=(K ** 3, K ** 3))
    return connected_components(A, directed=False)[1]


def mean_grain_volume(spins, K):
    return K ** 3 / grain_count(spins, K)


def growth_exponent(t, V):
    """Least-squares slope of log V against log t."""
    return float(np.polyfit(np.log(t), np.log(V), 1)[0])


def growth_constant(t, V):
    """c2 of V^(2/3) = c2 t + const, least squares."""
    return float(np.polyfit(np.asarray(t, float), np.asarray(V, float) ** (2.0 / 3.0), 1)[0])
