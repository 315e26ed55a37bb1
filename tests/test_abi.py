"""CPU checks of the C-ABI library: it loads, exports every entry point the header
declares, and its host-only logic (defaults, validation, per-grain tables) is right.
No call here touches a GPU."""
import ctypes as C
import math
import os
import re

import numpy as np
import pytest

import oracle as O
from conftest import ROOT

H = pytest.importorskip("paper_1009_0457_amd.hmc")


def _lib_or_skip():
    if not os.path.exists(H.LIB_PATH):
        pytest.skip("libhmc.so not built")
    return H.lib()


def header_functions():
    txt = open(os.path.join(ROOT, "include", "hmc.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(hmc_[a-z_0-9]+)\s*\(", txt)))


def test_every_declared_symbol_is_exported_and_bound():
    L = _lib_or_skip()
    names = header_functions()
    assert len(names) >= 20
    for n in names:
        assert hasattr(L, n), n
    assert sorted(H.exported_names()) == names


def test_default_params_match_the_oracle_reading():
    _lib_or_skip()
    for K, M, h in ((16, 6, 1), (64, 26, 2), (128, 26, 2), (8, 26, 0)):
        p = H.hmc_default_params(K, M, h)
        za, zb, ga, gb, gE = O.solver_defaults(p.C11, p.C12, p.C44, K, h)
        assert p.zone_alpha == pytest.approx(za, rel=1e-14)
        assert p.zone_beta == pytest.approx(zb, rel=1e-14)
        assert p.glob_alpha == pytest.approx(ga, rel=1e-14)
        assert p.glob_beta == pytest.approx(gb, rel=1e-14)
        assert p.glob_alphaE == pytest.approx(gE, rel=1e-14)
        assert p.lambda_el == pytest.approx(O.calibration(K)[2], rel=1e-12)
        assert p.zone_steps == (50 if h <= 1 else 200)


def test_grain_tables_agree_with_oracle_by_another_route():
    """Library: 6x6 transformation matrices and the closed-form cubic compliance.
    Oracle: 4-index tensor rotation and a numerical inverse."""
    _lib_or_skip()
    rng = np.random.default_rng(17)
    e = rng.uniform(0, 2 * math.pi, (64, 3))
    Cl, Sl = H.hmc_grain_tables(e, 246.5, 147.3, 124.7)
    Co, So, _ = O.tables(e, 246.5, 147.3, 124.7)
    assert np.abs(Cl - Co).max() < 1e-11
    assert np.abs(Sl - So).max() < 1e-15
    bad = e.copy()
    bad[3, 1] = np.nan
    with pytest.raises(H.HmcError) as ei:
        H.hmc_grain_tables(bad, 246.5, 147.3, 124.7)
    assert ei.value.status == H.HMC_ENUMERIC


def test_grain_table_derivatives_match_central_differences_of_the_oracle():
    _lib_or_skip()
    rng = np.random.default_rng(18)
    e = rng.uniform(0, 2 * math.pi, (6, 3))
    dC, dS = H.hmc_grain_table_derivatives(e, 246.5, 147.3, 124.7)
    h = 1e-6
    for q in range(3):
        ep, em = e.copy(), e.copy()
        ep[:, q] += h
        em[:, q] -= h
        Cp, Sp, _ = O.tables(ep, 246.5, 147.3, 124.7)
        Cm, Sm, _ = O.tables(em, 246.5, 147.3, 124.7)
        assert np.abs(dC[:, q] - (Cp - Cm) / (2 * h)).max() < 1e-6
        assert np.abs(dS[:, q] - (Sp - Sm) / (2 * h)).max() < 1e-10


@pytest.mark.parametrize("field,value,status", [
    ("K", 15, H.HMC_ESHAPE), ("K", 0, H.HMC_ESHAPE), ("K", 2048, H.HMC_ESHAPE),
    ("neighbors", 8, H.HMC_EINVAL), ("zone_h", 4, H.HMC_EINVAL), ("kT", 0.0, H.HMC_EINVAL),
    ("kT", float("nan"), H.HMC_ENUMERIC), ("proposal", 2, H.HMC_EINVAL), ("refresh_every", 0, H.HMC_EINVAL),
    ("C44", -1.0, H.HMC_ENUMERIC), ("zone_variant", 6, H.HMC_EINVAL), ("zone_variant", -1, H.HMC_EINVAL),
    ("refresh_tile_z", 3, H.HMC_EINVAL), ("refresh_tile_z", 64, H.HMC_EINVAL), ("material_points", 3, H.HMC_EINVAL),
])
def test_create_validates_before_touching_the_device(field, value, status):
    L = _lib_or_skip()
    p = H.hmc_default_params(16, 6, 1)
    setattr(p, field, value)
    assert L.hmc_workspace_bytes(C.byref(p), 8) == 0
    ctx = C.c_void_p()
    buf = (C.c_char * 512)()
    st = L.hmc_create(C.byref(p), 8, C.cast(buf, C.c_void_p), 512, None, C.byref(ctx))
    assert st == status and not ctx.value


def test_zone_variant_limits():
    L = _lib_or_skip()
    for h, variant, ok in ((0, 3, False), (3, 3, True), (3, 2, False), (1, 3, True), (2, 3, True), (3, 1, True),
                           (0, 2, True), (0, 4, False), (0, 5, False), (2, 4, True), (3, 5, True), (2, 6, False)):
        p = H.hmc_default_params(16, 26, h)
        p.zone_variant = variant
        assert (L.hmc_workspace_bytes(C.byref(p), 8) > 0) == ok, (h, variant)


def test_autotuner_candidates_are_the_variants_the_library_accepts():
    L = _lib_or_skip()
    from paper_1009_0457_amd.autotune import zone_variants_for
    for h in range(4):
        ok = []
        for v in range(1, 7):
            p = H.hmc_default_params(16, 26, h)
            p.zone_variant = v
            if L.hmc_workspace_bytes(C.byref(p), 8) > 0:
                ok.append(v)
        assert ok == zone_variants_for(h), h


def test_shape_limits():
    L = _lib_or_skip()
    p = H.hmc_default_params(4, 26, 2)          # K < 2h+2 with the elastic term on
    assert L.hmc_workspace_bytes(C.byref(p), 4) == 0
    p.lambda_el = 0.0                            # fine with elasticity off
    assert L.hmc_workspace_bytes(C.byref(p), 4) > 0
    p = H.hmc_default_params(16, 6, 1)
    assert L.hmc_workspace_bytes(C.byref(p), 32768) == 0
    assert L.hmc_workspace_bytes(C.byref(p), 32767) > 0
    ws = L.hmc_workspace_bytes(C.byref(p), 8)
    ctx = C.c_void_p()
    buf = (C.c_char * 64)()
    # too-small workspace is refused before any device call
    aligned = (C.addressof(buf) + 255) // 256 * 256
    assert ws > 64
    st = L.hmc_create(C.byref(p), 8, C.c_void_p(aligned), 16, None, C.byref(ctx))
    assert st == H.HMC_ESHAPE
    # a failed creation has no context; its message is kept per thread
    assert b"workspace smaller" in L.hmc_last_error(None)
    q = H.hmc_params.from_buffer_copy(p)
    q.neighbors = 7
    assert L.hmc_create(C.byref(q), 8, C.c_void_p(aligned), 16, None, C.byref(ctx)) == H.HMC_EINVAL
    assert L.hmc_last_error(None) == b"invalid parameters"
    with pytest.raises(H.HmcError, match="invalid parameters"):
        H._check(H.HMC_EINVAL, None, creating=True)


def test_load_range():
    """Loads beyond 5e4 MPa per component are refused: the explicit step's fixed-point stress
    sums are sized for that range."""
    L = _lib_or_skip()
    p = H.hmc_default_params(16, 26, 2)
    reps = (H.hmc_replica * 2)()
    for i in range(2):
        reps[i] = H.hmc_default_replica(p, 16, 8)
    reps[1].sigma_MPa[2] = 4.9e4
    assert L.hmc_batch_workspace_bytes(C.byref(p), 2, reps) > 0
    reps[1].sigma_MPa[2] = -5.1e4
    assert L.hmc_batch_workspace_bytes(C.byref(p), 2, reps) == 0


def test_null_context_calls_are_rejected():
    L = _lib_or_skip()
    assert L.hmc_sweep(None, 1) == H.HMC_EINVAL
    assert L.hmc_set_load(None, None) == H.HMC_EINVAL
    assert isinstance(L.hmc_last_error(None), bytes)


def test_material_points_constants_and_limits():
    """hmc_set_material_points: Polyak constants for L = 8 x the largest Mandel eigenvalue and
    the slowest shear wave of the (K/2)^3 mesh; invalid counts and lattices are refused before
    any device call."""
    L = _lib_or_skip()
    p = H.hmc_default_params(24, 26, 2)
    a1, b1 = p.glob_alpha, p.glob_beta
    H.hmc_set_material_points(p, 8)
    lam = max(p.C11 + 2 * p.C12, p.C11 - p.C12, 2 * p.C44)
    sl, sm = math.sqrt(8 * lam), math.sqrt(0.5 * (p.C11 - p.C12)) * 2 * math.sin(2 * math.pi / 24)
    assert p.material_points == 8
    assert p.glob_alpha == pytest.approx(4 / (sl + sm) ** 2, rel=1e-12)
    assert p.glob_beta == pytest.approx(((sl - sm) / (sl + sm)) ** 2, rel=1e-12)
    assert p.glob_alphaE == p.glob_alpha
    H.hmc_set_material_points(p, 1)
    assert (p.glob_alpha, p.glob_beta) == pytest.approx((a1, b1), rel=1e-14)
    assert L.hmc_set_material_points(C.byref(p), 4) == H.HMC_EINVAL
    q = H.hmc_default_params(2, 26, 0)
    q.material_points = 8
    assert L.hmc_workspace_bytes(C.byref(q), 4) == 0           # K >= 4 with 8 points per cell
    # replicas of a batch take the constants for their own K from hmc_default_replica
    p.material_points = 8
    r = H.hmc_default_replica(p, 40, 8)
    sl, sm = math.sqrt(8 * lam), math.sqrt(0.5 * (p.C11 - p.C12)) * 2 * math.sin(2 * math.pi / 40)
    assert r.glob_alpha == pytest.approx(4 / (sl + sm) ** 2, rel=1e-12)
    reps = (H.hmc_replica * 2)()
    reps[0], reps[1] = r, H.hmc_default_replica(p, 2, 8)
    assert L.hmc_batch_workspace_bytes(C.byref(p), 1, reps) > 0
    assert L.hmc_batch_workspace_bytes(C.byref(p), 2, reps) == 0     # K = 2 is too small for it


def test_per_source_build_options_name_existing_sources():
    """The build's per-source code-generation options and the sources the bench hashes for its
    counter keys must name files that exist: a renamed kernel source would otherwise lose its
    options (or its counters) without a word."""
    import sys

    sys.path.insert(0, ROOT)
    from paper_1009_0457_amd.build import SOURCE_FLAGS, sources

    import bench

    csrc = os.path.join(ROOT, "paper_1009_0457_amd", "csrc")
    built = {os.path.basename(s) for s in sources()}
    for name, flags in SOURCE_FLAGS.items():
        assert name in built, name
        assert flags and all(isinstance(f, str) for f in flags)
    for name in bench.ZONE_H2_SOURCES + ("hmc_potts.hip", "hmc_elastic.hip"):
        assert os.path.exists(os.path.join(csrc, name)), name
    # the per-size zone units instantiate their own lane-shift kernels and nothing else does
    for h, unit in ((2, "hmc_zone_h2.hip"), (3, "hmc_zone_h3.hip")):
        text = open(os.path.join(csrc, unit)).read()
        assert f"k_zone_lane<{h}, 1>" in text
        assert f"k_zone_lane<{h}," not in open(os.path.join(csrc, "hmc_zone.hip")).read()
