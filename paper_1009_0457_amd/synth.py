"""Seeded synthetic inputs: periodic Voronoi polycrystals with random orientations.

This module only draws inputs.  It holds none of the method's arithmetic (no
stiffness, energy or acceptance math), so both the HIP library's tests/bench
and the CPU oracle take their lattices from here.

The paper's microstructures are random polycrystals (Sec. 6 grain-growth runs
and the Sec. 7 texture runs); no dataset is involved.  Inputs are drawn with
``numpy.random.default_rng(seed)`` (PCG64):

* ``n_grains`` seed points uniform in [0, K)^3 (float64), then
* ``n_grains`` x 3 uniforms mapped to Bunge Euler angles with the Haar measure
  on SO(3): phi1, phi2 ~ U[0, 2 pi), cos(Phi) ~ U[-1, 1];
* every integer site (x, y, z) takes the index of the nearest seed point under
  the periodic minimum-image distance; an exact tie goes to the lower index.

Spins are 0-based grain indices, flat index ``x + K*(y + K*z)``.
"""
from __future__ import annotations

import json
import math
import os
from dataclasses import dataclass, field

import numpy as np

__all__ = [
    "Microstructure",
    "voronoi_polycrystal",
    "haar_euler",
    "RunConfig",
    "tiny_config",
    "full_config",
    "large_config",
    "batched_configs",
    "adjoint_config",
    "random_spins",
    "z_rotation_euler",
    "texture_run_inputs",
]


@dataclass
class Microstructure:
    K: int
    spins: np.ndarray   # int32, shape (K**3,), x fastest
    euler: np.ndarray   # float64, shape (Q, 3), Bunge (phi1, Phi, phi2) in radians

    @property
    def Q(self) -> int:
        return int(self.euler.shape[0])


def haar_euler(rng: np.random.Generator, n: int) -> np.ndarray:
    """Bunge angles of ``n`` orientations drawn uniformly (Haar) on SO(3)."""
    u = rng.uniform(size=(n, 3))
    phi1 = 2.0 * math.pi * u[:, 0]
    Phi = np.arccos(2.0 * u[:, 1] - 1.0)
    phi2 = 2.0 * math.pi * u[:, 2]
    return np.stack([phi1, Phi, phi2], axis=1)


def _assign_voronoi(K: int, pts: np.ndarray) -> np.ndarray:
    from scipy.spatial import cKDTree

    g = np.arange(K, dtype=np.float64)
    z, y, x = np.meshgrid(g, g, g, indexing="ij")
    sites = np.stack([x.ravel(), y.ravel(), z.ravel()], axis=1)
    n = pts.shape[0]
    if n == 1:
        return np.zeros(K ** 3, dtype=np.int32)
    tree = cKDTree(pts, boxsize=float(K))
    _, idx = tree.query(sites, k=2)
    # exact squared minimum-image distances of the two candidates; ties -> lower index
    best = np.empty(sites.shape[0], dtype=np.int64)
    d2 = []
    for j in range(2):
        d = sites - pts[idx[:, j]]
        d -= K * np.round(d / K)
        d2.append(np.einsum("ij,ij->i", d, d))
    a, b = idx[:, 0], idx[:, 1]
    take_b = (d2[1] < d2[0]) | ((d2[1] == d2[0]) & (b < a))
    best[:] = np.where(take_b, b, a)
    return best.astype(np.int32)


def voronoi_polycrystal(K: int, n_grains: int, seed: int,
                        rng: np.random.Generator | None = None) -> Microstructure:
    """Periodic Voronoi polycrystal on a K^3 lattice with Haar-random orientations."""
    if rng is None:
        rng = np.random.default_rng(seed)
    pts = rng.uniform(0.0, float(K), size=(n_grains, 3))
    euler = haar_euler(rng, n_grains)
    spins = _assign_voronoi(K, pts)
    return Microstructure(K=K, spins=spins, euler=euler)


def refined_polycrystal(K: int, factor: int, n_grains: int, seed: int) -> Microstructure:
    """A Voronoi polycrystal built on a (K/factor)^3 lattice with each site replicated into a
    factor^3 block: the same periodic grain structure at K^3 without a K^3 nearest-seed
    search (for bandwidth measurements on lattices larger than the caches)."""
    if K % factor:
        raise ValueError("K must be a multiple of factor")
    m = voronoi_polycrystal(K // factor, n_grains, seed)
    k = K // factor
    s = m.spins.reshape(k, k, k)                       # (z, y, x), x fastest
    s = np.repeat(np.repeat(np.repeat(s, factor, axis=0), factor, axis=1), factor, axis=2)
    return Microstructure(K=K, spins=np.ascontiguousarray(s).reshape(-1).astype(np.int32), euler=m.euler)


def random_spins(K: int, Q: int, seed: int) -> np.ndarray:
    """Independent uniform spins in [0, Q): a maximally disordered test lattice."""
    rng = np.random.default_rng(seed)
    return rng.integers(0, Q, size=K ** 3, dtype=np.int64).astype(np.int32)


def z_rotation_euler(n: int = 91, step_deg: float = 1.0) -> np.ndarray:
    """Bunge angles of n rotations about z by 0, step, 2 step, ... degrees (Sec. 7's single
    Euler angle study: the other two angles zero)."""
    e = np.zeros((n, 3))
    e[:, 0] = np.radians(step_deg * np.arange(n))
    return e


def texture_run_inputs(K: int = 100, runs: int = 10, Q: int = 91, seed: int = 300, euler=None):
    """Sec. 7's texture runs: every site an independent uniform choice among Q orientations,
    by default the rotations about z by 0..90 degrees; one (euler, spins) pair per run, run r
    drawn with seed + r."""
    e = z_rotation_euler(Q, 90.0 / (Q - 1)) if euler is None else np.ascontiguousarray(euler, np.float64)
    if e.shape != (Q, 3):
        raise ValueError("euler must hold Q Bunge triples")
    return [(e, random_spins(K, Q, seed + r)) for r in range(runs)]


@dataclass
class RunConfig:
    """One workload: lattice, physics and run schedule (GPa for stresses)."""
    name: str
    K: int
    neighbors: int
    n_grains: int
    sigma_MPa: np.ndarray          # Voigt xx, yy, zz, yz, xz, xy
    kT: float
    zone_h: int
    zone_steps: int
    sweeps: int
    refresh_every: int
    seed: int = 1                  # microstructure seed
    philox_seed: int = 1
    J: float = 1.0
    C11: float = 246.5
    C12: float = 147.3
    C44: float = 124.7
    proposal: int = 0              # 0 = random neighbour's spin, 1 = uniform other spin
    refresh_steps: int = 200
    cold_steps: int = 2000
    histogram_every: int = 0
    histogram_axes: tuple = ()
    extra: dict = field(default_factory=dict)

    def microstructure(self) -> Microstructure:
        return voronoi_polycrystal(self.K, self.n_grains, self.seed)

    def zero_load(self) -> "RunConfig":
        import copy
        c = copy.deepcopy(self)
        c.name = self.name + "-zero-load"
        c.sigma_MPa = np.zeros(6)
        return c


# The workloads are described by the JSON files under configs/ at the repository root (one per
# workload; a zero-load twin is the same with the load set to zero, RunConfig.zero_load).
CONFIG_DIR = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "configs")
_RUN_KEYS = ("K", "neighbors", "n_grains", "kT", "zone_h", "zone_steps", "sweeps", "refresh_every", "seed",
             "philox_seed", "J", "C11", "C12", "C44", "proposal", "refresh_steps", "cold_steps", "histogram_every")


def load_config(name: str) -> dict:
    """The JSON description of workload `name` (configs/<name>.json)."""
    with open(os.path.join(CONFIG_DIR, name + ".json")) as f:
        return json.load(f)


def run_config(name: str) -> RunConfig:
    """A single-lattice workload from its JSON description."""
    d = load_config(name)
    kw = {k: d[k] for k in _RUN_KEYS if k in d}
    return RunConfig(name=d["name"], sigma_MPa=np.array(d["sigma_MPa"], float),
                     histogram_axes=tuple(tuple(float(v) for v in ax) for ax in d.get("histogram_axes", ())), **kw)


def tiny_config() -> RunConfig:
    """16^3, 6 neighbours (red/black), 8 grains, 100 MPa along z, 3^3 zone x 50 steps."""
    return run_config("tiny-16")


def full_config() -> RunConfig:
    """64^3, 26 neighbours (8 colours), 500 grains, 200 MPa along z, 5^3 zone x 200 steps."""
    return run_config("full-64")


def large_config() -> RunConfig:
    """128^3, 26 neighbours, 4000 grains, biaxial 150/150 MPa, 5^3 zone x 200 steps."""
    return run_config("large-128")


def batched_configs(n_replicas: int | None = None) -> list[RunConfig]:
    """Replica ensemble: K in {32,48,64,96}, 8 grains per 16^3, random uniaxial load."""
    d = load_config("batched-64")
    n_replicas = d["replicas"] if n_replicas is None else n_replicas
    rng = np.random.default_rng(d["rng_seed"])
    choices = tuple(int(k) for k in d["K_choices"])
    lo, hi = d["kT_range"]
    out = []
    for r in range(n_replicas):
        K = int(choices[rng.integers(0, len(choices))])
        s = float(rng.uniform(0.0, d["load_MPa_max"]))
        n = rng.normal(size=3)
        n /= np.linalg.norm(n)
        kT = float(rng.uniform(lo, hi))
        sig = s * np.outer(n, n)
        voigt = np.array([sig[0, 0], sig[1, 1], sig[2, 2], sig[1, 2], sig[0, 2], sig[0, 1]])
        out.append(RunConfig(name=f"replica-{r}", K=K, neighbors=d["neighbors"],
                             n_grains=d["grains_per_16_cube"] * (K // 16) ** 3, sigma_MPa=voigt, kT=kT,
                             zone_h=d["zone_h"], zone_steps=d["zone_steps"], sweeps=d["sweeps"],
                             refresh_every=d["refresh_every"], seed=r + 1, philox_seed=r + 1,
                             extra={"axis": n, "load_MPa": s}))
    return out


def adjoint_config():
    """64^3, 500 grains; six stress components U(-200, 200) MPa; 10 probe grains."""
    d = load_config("adjoint-64")
    rng = np.random.default_rng(d["rng_seed"])
    micro = voronoi_polycrystal(d["K"], d["n_grains"], d["rng_seed"], rng=rng)
    sigma = rng.uniform(-d["sigma_MPa_max"], d["sigma_MPa_max"], size=6)
    probe = rng.choice(d["n_grains"], size=d["probe_grains"], replace=False)
    return micro, sigma, probe
