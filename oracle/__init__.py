"""Python access to the serial FP64 CPU oracle (``hmc_oracle.c``).

TEST INFRASTRUCTURE ONLY: imported by the tests, by the smoke check and by the
benchmark's CPU-baseline leg, never by the library.  It shares no code with the
HIP path.  Everything here is double precision and single threaded.

Section/equation references are to Zhang, Bartel & Lusk, arXiv:1009.0457.
"""
from __future__ import annotations

import ctypes as C
import math
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "hmc_oracle.c")
_LIB = os.path.join(_HERE, "libhmc_oracle.so")

_i32p = np.ctypeslib.ndpointer(dtype=np.int32, flags="C_CONTIGUOUS")
_i64p = np.ctypeslib.ndpointer(dtype=np.int64, flags="C_CONTIGUOUS")
_f64p = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")
_u32p = np.ctypeslib.ndpointer(dtype=np.uint32, flags="C_CONTIGUOUS")


def build(force: bool = False) -> str:
    """Compile the oracle with gcc: -O2, no fast-math, no FMA contraction, one thread."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-std=c11", "-O2", "-ffp-contract=off", "-fno-fast-math",
                               "-fPIC", "-shared", "-D_GNU_SOURCE", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class Params(C.Structure):
    _fields_ = [("K", C.c_int32), ("M", C.c_int32), ("Q", C.c_int32), ("proposal", C.c_int32),
                ("h", C.c_int32), ("nr", C.c_int32), ("elastic", C.c_int32), ("R", C.c_int32),
                ("n_warm", C.c_int32), ("pad_", C.c_int32),
                ("J", C.c_double), ("kT", C.c_double), ("lambda_el", C.c_double),
                ("zone_alpha", C.c_double), ("zone_beta", C.c_double),
                ("glob_alpha", C.c_double), ("glob_beta", C.c_double), ("glob_alphaE", C.c_double),
                ("Sigma", C.c_double * 6), ("seed", C.c_uint64)]


record_dtype = np.dtype([("q_new", np.int32), ("gb", np.int32), ("dPi", np.float64),
                         ("dE", np.float64), ("r1", np.uint32), ("flags", np.int32)])
_recp = np.ctypeslib.ndpointer(dtype=record_dtype, flags="C_CONTIGUOUS")

_lib = None


def lib():
    global _lib
    if _lib is None:
        L = C.CDLL(build())
        L.ora_philox4x32_10.argtypes = [_u32p, _u32p, _u32p]
        L.ora_draw.argtypes = [C.c_uint64, C.c_uint32, C.c_uint32, _u32p]
        L.ora_slot_offset.argtypes = [C.c_int, C.c_int, C.POINTER(C.c_int)]
        L.ora_neighbour.argtypes = [C.c_int, C.c_int, C.c_int64, C.c_int]
        L.ora_neighbour.restype = C.c_int64
        L.ora_colour.argtypes = [C.c_int, C.c_int64, C.c_int64, C.c_int64]
        L.ora_colour.restype = C.c_int
        L.ora_gb_count.argtypes = [C.c_int, C.c_int, _i32p, C.c_int64, C.c_int32]
        L.ora_gb_count.restype = C.c_int
        L.ora_unlike_bonds.argtypes = [C.c_int, C.c_int, _i32p]
        L.ora_unlike_bonds.restype = C.c_int64
        L.ora_propose.argtypes = [C.c_int, C.c_int, C.c_int, C.c_int, _i32p, C.c_int64, C.c_uint32]
        L.ora_propose.restype = C.c_int32
        L.ora_rotation.argtypes = [C.c_double, C.c_double, C.c_double, _f64p]
        L.ora_rotate_stiffness.argtypes = [_f64p, _f64p, _f64p]
        L.ora_invert6.argtypes = [_f64p, _f64p]
        L.ora_invert6.restype = C.c_int
        L.ora_tables.argtypes = [C.c_int, _f64p, C.c_double, C.c_double, C.c_double, _f64p, _f64p, _f64p]
        L.ora_tables.restype = C.c_int
        L.ora_texture_angle.argtypes = [_f64p, _f64p]
        L.ora_texture_angle.restype = C.c_double
        L.ora_texture_counts.argtypes = [C.c_int, _i32p, C.c_int, _f64p, _f64p, C.c_double, C.c_int, _i64p]
        L.ora_global.argtypes = [C.c_int, _i32p, _f64p, _f64p, _f64p, C.c_int, C.c_int, C.c_double,
                                 C.c_double, C.c_double, _f64p, _f64p, C.c_void_p, _f64p]
        L.ora_elastic_energy.argtypes = [C.c_int, _i32p, _f64p, _f64p, _f64p]
        L.ora_elastic_energy.restype = C.c_double
        L.ora_zone.argtypes = [C.c_int, _i32p, _f64p, _f64p, C.c_int64, C.c_int32, _f64p, C.c_int,
                               C.c_int, C.c_double, C.c_double]
        L.ora_zone.restype = C.c_double
        L.ora_zone_literal.argtypes = [C.c_int, _i32p, _f64p, _f64p, _f64p, C.c_int64, C.c_int32,
                                       C.c_int, C.c_int, C.c_double, C.c_double]
        L.ora_zone_literal.restype = C.c_double
        L.ora_trial.argtypes = [C.POINTER(Params), _i32p, _f64p, _f64p, C.c_void_p, C.c_int64,
                                C.c_uint32, _recp]
        L.ora_pass.argtypes = [C.POINTER(Params), _i32p, _f64p, _f64p, C.c_void_p, C.c_uint32, C.c_int,
                               C.c_void_p]
        L.ora_trials.argtypes = [C.POINTER(Params), _i32p, _f64p, _f64p, C.c_void_p, C.c_uint32, _i64p,
                                 C.c_int64, C.c_void_p]
        L.ora_trials.restype = C.c_int64
        L.ora_sweeps.argtypes = [C.POINTER(Params), _i32p, _f64p, _f64p, _f64p, _f64p, _f64p,
                                 C.c_uint32, C.c_int]
        L.ora_gs_sweeps.argtypes = [C.POINTER(Params), _i32p, C.c_uint32, C.c_int]
        L.ora_global_mp8.argtypes = L.ora_global.argtypes
        L.ora_residual_mp8.argtypes = [C.c_int, _i32p, _f64p, _f64p, _f64p, _f64p, C.c_void_p,
                                       C.POINTER(C.c_double)]
        _lib = L
    return _lib


def _vp(a):
    return None if a is None else a.ctypes.data_as(C.c_void_p)


# ------------------------------------------------------------------------------------
# Random numbers
# ------------------------------------------------------------------------------------
def philox4x32_10(ctr, key) -> np.ndarray:
    out = np.zeros(4, np.uint32)
    lib().ora_philox4x32_10(np.asarray(ctr, np.uint32), np.asarray(key, np.uint32), out)
    return out


def draw(seed: int, site: int, sweep: int) -> np.ndarray:
    out = np.zeros(4, np.uint32)
    lib().ora_draw(seed, site, sweep, out)
    return out


# ------------------------------------------------------------------------------------
# Lattice
# ------------------------------------------------------------------------------------
def num_colours(M: int) -> int:
    return 2 if M == 6 else 8


def slot_offsets(M: int) -> np.ndarray:
    out = np.zeros((M, 3), np.int64)
    for k in range(M):
        o = (C.c_int * 3)()
        lib().ora_slot_offset(M, k, o)
        out[k] = list(o)
    return out


def colour_of(K: int, M: int) -> np.ndarray:
    g = np.arange(K)
    z, y, x = np.meshgrid(g, g, g, indexing="ij")
    L = lib()
    return np.array([L.ora_colour(M, int(a), int(b), int(c))
                     for a, b, c in zip(x.ravel(), y.ravel(), z.ravel())], np.int32)


def gb_count(K, M, q, site, q_new) -> int:
    return lib().ora_gb_count(K, M, np.ascontiguousarray(q, np.int32), site, q_new)


def unlike_bonds(K, M, q) -> int:
    return lib().ora_unlike_bonds(K, M, np.ascontiguousarray(q, np.int32))


def propose(K, M, Q, proposal, q, site, r0) -> int:
    return lib().ora_propose(K, M, Q, proposal, np.ascontiguousarray(q, np.int32), site, int(r0))


# ------------------------------------------------------------------------------------
# Tables (Sec. 5)
# ------------------------------------------------------------------------------------
def rotation(phi1, Phi, phi2) -> np.ndarray:
    A = np.zeros(9)
    lib().ora_rotation(phi1, Phi, phi2, A)
    return A.reshape(3, 3)


def cubic_voigt(C11, C12, C44) -> np.ndarray:
    Cc = np.zeros((6, 6))
    Cc[:3, :3] = C12
    np.fill_diagonal(Cc[:3, :3], C11)
    Cc[3, 3] = Cc[4, 4] = Cc[5, 5] = C44
    return Cc


def rotate_stiffness(A, Cvoigt) -> np.ndarray:
    out = np.zeros(36)
    lib().ora_rotate_stiffness(np.ascontiguousarray(A, np.float64).ravel(),
                               np.ascontiguousarray(Cvoigt, np.float64).ravel(), out)
    return out.reshape(6, 6)


def tables(euler, C11, C12, C44):
    """Per-grain (C, S, A): lab stiffness, its inverse and the rotation matrix."""
    euler = np.ascontiguousarray(euler, np.float64)
    Q = euler.shape[0]
    Ct = np.zeros((Q, 36))
    St = np.zeros((Q, 36))
    At = np.zeros((Q, 9))
    if lib().ora_tables(Q, euler.ravel(), C11, C12, C44, Ct.ravel(), St.ravel(), At.ravel()) != 0:
        raise ValueError("singular stiffness")
    return Ct.reshape(Q, 6, 6), St.reshape(Q, 6, 6), At.reshape(Q, 3, 3)


def texture_angle(A, axis) -> float:
    return lib().ora_texture_angle(np.ascontiguousarray(A, np.float64).ravel(),
                                   np.asarray(axis, np.float64))


def texture_counts(K, q, A_tab, axis, bin_deg=10.0, nbins=6) -> np.ndarray:
    out = np.zeros(nbins, np.int64)
    A_tab = np.ascontiguousarray(A_tab, np.float64)
    lib().ora_texture_counts(K, np.ascontiguousarray(q, np.int32), A_tab.shape[0], A_tab.ravel(),
                             np.asarray(axis, np.float64), bin_deg, nbins, out)
    return out


# ------------------------------------------------------------------------------------
# Solver parameters and units
# ------------------------------------------------------------------------------------
def polyak(L: float, mu: float):
    """Heavy-ball step and momentum for a quadratic with spectrum in [mu, L]."""
    sL, sm = math.sqrt(L), math.sqrt(mu)
    return 4.0 / (sL + sm) ** 2, ((sL - sm) / (sL + sm)) ** 2


def solver_defaults(C11, C12, C44, K, h):
    """(zone_alpha, zone_beta, glob_alpha, glob_beta, glob_alphaE).

    L = 4 * largest eigenvalue of the cubic stiffness in Mandel form (a rigorous bound on
    both Hessians).  mu: for the periodic grid the slowest shear wave,
    1/2 (C11 - C12) (2 sin(pi/K))^2; for the free-boundary zone of edge n = 2h+1 the
    softest deformation modes scale as 1/2 (C11 - C12) / n^2."""
    lam = max(C11 + 2 * C12, C11 - C12, 2 * C44)
    L = 4.0 * lam
    shear = 0.5 * (C11 - C12)
    za, zb = polyak(L, shear / (2 * h + 1) ** 2)
    ga, gb = polyak(L, shear * (2 * math.sin(math.pi / K)) ** 2)
    return za, zb, ga, gb, ga


def solver_defaults_mp8(C11, C12, C44, K):
    """(glob_alpha, glob_beta, glob_alphaE) of the 2 x 2 x 2-points-per-cell variant: L = 8 x
    the largest Mandel eigenvalue of the stiffness (the identity material's Hessian peaks at 8
    there, against 4 for one point per voxel); mu = 1/2 (C11 - C12) (2 sin(2 pi / K))^2, the
    slowest shear wave on the (K/2)^3 mesh."""
    lam = max(C11 + 2 * C12, C11 - C12, 2 * C44)
    a, b = polyak(8.0 * lam, 0.5 * (C11 - C12) * (2 * math.sin(2 * math.pi / K)) ** 2)
    return a, b, a


def calibration(K: int, l0=1.0e-3, gamma_s=0.45, gamma_mc=2.4, m_s=1.0e-13, m_star=0.27):
    """Characteristic scales of Sec. 4 (Eqs. chatime, chaeng, elamc) from Table 1 values.

    Returns (t0 [s], E0 [J], lambda_el [MC energy per GPa*voxel])."""
    delta = 1.0 / K
    t0 = l0 ** 2 * m_star * delta ** 2 / (m_s * gamma_s)
    E0 = gamma_s * l0 ** 2 * delta ** 2 / gamma_mc
    lam = 1.0e9 * (l0 * delta) ** 3 / (2.0 * E0)
    return t0, E0, lam


def make_params(K, M, Q, *, proposal=0, h=1, nr=50, elastic=False, R=1, n_warm=200, J=1.0, kT=0.5,
                lambda_el=0.0, zone_alpha=0.0, zone_beta=0.0, glob_alpha=0.0, glob_beta=0.0,
                glob_alphaE=0.0, Sigma=(0, 0, 0, 0, 0, 0), seed=1) -> Params:
    P = Params()
    P.K, P.M, P.Q, P.proposal, P.h, P.nr = K, M, Q, proposal, h, nr
    P.elastic, P.R, P.n_warm = int(bool(elastic)), R, n_warm
    P.J, P.kT, P.lambda_el = J, kT, lambda_el
    P.zone_alpha, P.zone_beta = zone_alpha, zone_beta
    P.glob_alpha, P.glob_beta, P.glob_alphaE = glob_alpha, glob_beta, glob_alphaE
    for i in range(6):
        P.Sigma[i] = float(Sigma[i])
    P.seed = seed
    return P


# ------------------------------------------------------------------------------------
# Elasticity
# ------------------------------------------------------------------------------------
def global_solve(K, q, Ct, St, Sigma_GPa, nsteps, cold, alpha, beta, alphaE, u=None, E=None):
    """Explicit damped relaxation of the periodic grid (Sec. 5).

    Returns (u (3,K^3), E (6,), sigma (6,K^3), info dict)."""
    n3 = K ** 3
    u = np.zeros(3 * n3) if u is None else np.ascontiguousarray(u, np.float64).ravel().copy()
    E = np.zeros(6) if E is None else np.ascontiguousarray(E, np.float64).copy()
    sig = np.zeros(6 * n3)
    info = np.zeros(3)
    lib().ora_global(K, np.ascontiguousarray(q, np.int32), np.ascontiguousarray(Ct).ravel(),
                     np.ascontiguousarray(St).ravel(), np.asarray(Sigma_GPa, np.float64), nsteps,
                     int(cold), alpha, beta, alphaE, u, E, _vp(sig), info)
    return u.reshape(3, n3), E, sig.reshape(6, n3), {"U": info[0], "res_u": info[1], "res_E": info[2]}


def global_solve_mp8(K, q, Ct, St, Sigma_GPa, nsteps, cold, alpha, beta, alphaE, u=None, E=None):
    """The global solve with 2 x 2 x 2 material points (sites) per background cell of 2^3
    sites (Appendix); u lives on the (K/2)^3 mesh nodes.  Returns (u (3,(K/2)^3), E, sigma
    (6,K^3) of the points, info)."""
    if K % 2:
        raise ValueError("K must be even")
    n3, nn = K ** 3, (K // 2) ** 3
    u = np.zeros(3 * nn) if u is None else np.ascontiguousarray(u, np.float64).ravel().copy()
    E = np.zeros(6) if E is None else np.ascontiguousarray(E, np.float64).copy()
    sig = np.zeros(6 * n3)
    info = np.zeros(3)
    lib().ora_global_mp8(K, np.ascontiguousarray(q, np.int32), np.ascontiguousarray(Ct).ravel(),
                         np.ascontiguousarray(St).ravel(), np.asarray(Sigma_GPa, np.float64), nsteps,
                         int(cold), alpha, beta, alphaE, u, E, _vp(sig), info)
    return u.reshape(3, nn), E, sig.reshape(6, n3), {"U": info[0], "res_u": info[1], "res_E": info[2]}


def residual_mp8(K, q, Ct, u, E):
    """(residual forces (3,(K/2)^3), point stresses (6,K^3), stored energy) of the variant."""
    nn, n3 = (K // 2) ** 3, K ** 3
    r = np.zeros(3 * nn)
    sig = np.zeros(6 * n3)
    U = C.c_double()
    lib().ora_residual_mp8(K, np.ascontiguousarray(q, np.int32), np.ascontiguousarray(Ct).ravel(),
                           np.ascontiguousarray(u, np.float64).ravel(), np.asarray(E, np.float64), r, _vp(sig),
                           C.byref(U))
    return r.reshape(3, nn), sig.reshape(6, n3), U.value


def elastic_energy(K, q, Ct, u, E) -> float:
    return lib().ora_elastic_energy(K, np.ascontiguousarray(q, np.int32), np.ascontiguousarray(Ct).ravel(),
                                    np.ascontiguousarray(u, np.float64).ravel(), np.asarray(E, np.float64))


def zone(K, q, Ct, St, site, q_new, sigma_p, h, nr, alpha, beta) -> float:
    """Elastic energy change (GPa*voxel) of one trial flip by the zone solve (Sec. 3)."""
    return lib().ora_zone(K, np.ascontiguousarray(q, np.int32), np.ascontiguousarray(Ct).ravel(),
                          np.ascontiguousarray(St).ravel(), site, q_new,
                          np.asarray(sigma_p, np.float64), h, nr, alpha, beta)


def zone_literal(K, q, Ct, u, E, site, q_new, h, nr, alpha, beta) -> float:
    return lib().ora_zone_literal(K, np.ascontiguousarray(q, np.int32), np.ascontiguousarray(Ct).ravel(),
                                  np.ascontiguousarray(u, np.float64).ravel(), np.asarray(E, np.float64),
                                  site, q_new, h, nr, alpha, beta)


# ------------------------------------------------------------------------------------
# Monte Carlo
# ------------------------------------------------------------------------------------
def _sig_ptr(sigma):
    if sigma is None:
        return None, None
    s = np.ascontiguousarray(sigma, np.float64).ravel()
    return s, s.ctypes.data_as(C.c_void_p)


def trial(P: Params, snap, Ct, St, sigma, site, sweep):
    rec = np.zeros(1, record_dtype)
    s, sp = _sig_ptr(sigma)
    lib().ora_trial(C.byref(P), np.ascontiguousarray(snap, np.int32), np.ascontiguousarray(Ct).ravel(),
                    np.ascontiguousarray(St).ravel(), sp, site, sweep, rec)
    return rec[0]


def colour_pass(P: Params, q, Ct, St, sigma, sweep, colour, want_records=False):
    """One colour pass in place on q (int32 array); returns the per-site records or None."""
    recs = np.zeros(P.K ** 3, record_dtype) if want_records else None
    s, sp = _sig_ptr(sigma)
    lib().ora_pass(C.byref(P), q, np.ascontiguousarray(Ct).ravel(), np.ascontiguousarray(St).ravel(),
                   sp, sweep, colour, _vp(recs))
    return recs


def trials(P: Params, snap, Ct, St, sigma, sweep, sites):
    sites = np.ascontiguousarray(sites, np.int64)
    recs = np.zeros(sites.shape[0], record_dtype)
    s, sp = _sig_ptr(sigma)
    lib().ora_trials(C.byref(P), np.ascontiguousarray(snap, np.int32), np.ascontiguousarray(Ct).ravel(),
                     np.ascontiguousarray(St).ravel(), sp, sweep, sites, sites.shape[0], _vp(recs))
    return recs


def gs_sweeps(P: Params, q, s0, n):
    """n Gauss-Seidel sweeps (Sec. 6's comparison scheme) in place on q, zero load only."""
    if P.elastic:
        raise ValueError("Gauss-Seidel sweeps are for zero load")
    lib().ora_gs_sweeps(C.byref(P), q, s0, n)


def sweeps(P: Params, q, Ct, St, u, E, sigma, s0, n):
    """n sweeps in place on q (and on u, E, sigma when elasticity is on)."""
    lib().ora_sweeps(C.byref(P), q, np.ascontiguousarray(Ct).ravel(), np.ascontiguousarray(St).ravel(),
                     u, E, sigma, s0, n)
