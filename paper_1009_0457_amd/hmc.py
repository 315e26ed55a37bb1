"""Thin Python binding of the C ABI in include/hmc.h (argument marshalling only).

Every ``hmc_*`` function here calls the function of the same name in ``libhmc.so``;
device arrays are torch tensors on the HIP device (PyTorch supplies device memory and
streams, nothing else).  ``Lattice`` is a small convenience owner of one context and its
workspace.  There is no fallback: without the built HIP library or a GPU every call
raises.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libhmc.so")

HMC_OK, HMC_EINVAL, HMC_ESHAPE, HMC_ESTATE, HMC_EDEVICE, HMC_ENUMERIC = range(6)
_STATUS = {0: "HMC_OK", 1: "HMC_EINVAL", 2: "HMC_ESHAPE", 3: "HMC_ESTATE", 4: "HMC_EDEVICE", 5: "HMC_ENUMERIC"}


class HmcError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{_STATUS.get(status, status)}: {msg}")
        self.status = status


class hmc_params(C.Structure):
    _fields_ = [("K", C.c_int32), ("neighbors", C.c_int32), ("proposal", C.c_int32), ("zone_h", C.c_int32),
                ("zone_steps", C.c_int32), ("refresh_every", C.c_int32), ("refresh_steps", C.c_int32),
                ("cold_steps", C.c_int32), ("zone_variant", C.c_int32), ("zone_screen", C.c_int32),
                ("refresh_tile_z", C.c_int32), ("material_points", C.c_int32),
                ("J", C.c_double), ("kT", C.c_double), ("C11", C.c_double), ("C12", C.c_double),
                ("C44", C.c_double), ("lambda_el", C.c_double), ("zone_alpha", C.c_double),
                ("zone_beta", C.c_double), ("glob_alpha", C.c_double), ("glob_beta", C.c_double),
                ("glob_alphaE", C.c_double), ("seed", C.c_uint64)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class hmc_kernel_time(C.Structure):
    _fields_ = [("launches", C.c_int64), ("total_ms", C.c_double)]


class hmc_kernel_times(C.Structure):
    _fields_ = [("potts", hmc_kernel_time), ("zone", hmc_kernel_time), ("apply", hmc_kernel_time),
                ("refresh_step", hmc_kernel_time), ("refresh_other", hmc_kernel_time)]


class hmc_replica(C.Structure):
    _fields_ = [("K", C.c_int32), ("Q", C.c_int32), ("kT", C.c_double), ("lambda_el", C.c_double),
                ("glob_alpha", C.c_double), ("glob_beta", C.c_double), ("glob_alphaE", C.c_double),
                ("sigma_MPa", C.c_double * 6), ("seed", C.c_uint64)]


class hmc_stats(C.Structure):
    _fields_ = [("site_trials", C.c_int64), ("real_flips", C.c_int64), ("zone_solves", C.c_int64),
                ("accepted", C.c_int64), ("screened", C.c_int64), ("refresh_steps", C.c_int64)]


# numpy view of hmc_trial_record (24 bytes)
record_dtype = np.dtype([("q_new", np.int32), ("gb", np.int32), ("dPi", np.float32), ("r1", np.uint32),
                         ("flags", np.int32), ("reserved", np.int32)])

_lib = None

# (name, restype, argtypes) of every exported entry point, in header order
_SIGS = [
    ("hmc_default_params", C.c_int, [C.POINTER(hmc_params), C.c_int32, C.c_int32, C.c_int32]),
    ("hmc_workspace_bytes", C.c_size_t, [C.POINTER(hmc_params), C.c_int32]),
    ("hmc_create", C.c_int, [C.POINTER(hmc_params), C.c_int32, C.c_void_p, C.c_size_t, C.c_void_p,
                             C.POINTER(C.c_void_p)]),
    ("hmc_destroy", None, [C.c_void_p]),
    ("hmc_last_error", C.c_char_p, [C.c_void_p]),
    ("hmc_set_orientations", C.c_int, [C.c_void_p, C.c_void_p]),
    ("hmc_set_spins", C.c_int, [C.c_void_p, C.c_void_p]),
    ("hmc_get_spins", C.c_int, [C.c_void_p, C.c_void_p]),
    ("hmc_set_load", C.c_int, [C.c_void_p, C.c_void_p]),
    ("hmc_stress_refresh", C.c_int, [C.c_void_p, C.c_int32, C.c_int32]),
    ("hmc_sweep", C.c_int, [C.c_void_p, C.c_int32]),
    ("hmc_colour_pass", C.c_int, [C.c_void_p, C.c_int32, C.c_void_p]),
    ("hmc_energy", C.c_int, [C.c_void_p, C.POINTER(C.c_int64), C.POINTER(C.c_double)]),
    ("hmc_texture_histogram", C.c_int, [C.c_void_p, C.c_void_p, C.c_double, C.c_int32, C.c_void_p]),
    ("hmc_set_block_order", C.c_int, [C.c_void_p, C.c_int32]),
    ("hmc_texture_histogram_noalloc", C.c_int, [C.c_void_p, C.c_int32, C.c_int32, C.c_void_p, C.c_void_p,
                                                C.c_double, C.c_int32, C.c_void_p, C.c_void_p]),
    ("hmc_get_stress", C.c_int, [C.c_void_p, C.c_void_p]),
    ("hmc_set_stress", C.c_int, [C.c_void_p, C.c_void_p]),
    ("hmc_get_displacement", C.c_int, [C.c_void_p, C.c_void_p]),
    ("hmc_get_macro_strain", C.c_int, [C.c_void_p, C.c_void_p]),
    ("hmc_set_elastic_state", C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p]),
    ("hmc_set_sweep_index", C.c_int, [C.c_void_p, C.c_int64]),
    ("hmc_get_sweep_index", C.c_int, [C.c_void_p, C.POINTER(C.c_int64)]),
    ("hmc_get_stats", C.c_int, [C.c_void_p, C.POINTER(hmc_stats)]),
    ("hmc_reset_stats", C.c_int, [C.c_void_p]),
    ("hmc_set_zone_screen", C.c_int, [C.c_void_p, C.c_int32]),
    ("hmc_set_zone_variant", C.c_int, [C.c_void_p, C.c_int32]),
    ("hmc_set_profiling", C.c_int, [C.c_void_p, C.c_int32]),
    ("hmc_get_kernel_times", C.c_int, [C.c_void_p, C.POINTER(hmc_kernel_times)]),
    ("hmc_set_graphs", C.c_int, [C.c_void_p, C.c_int32]),
    ("hmc_set_material_points", C.c_int, [C.POINTER(hmc_params), C.c_int32]),
    ("hmc_grain_labels", C.c_int, [C.c_void_p, C.c_int32, C.c_void_p, C.POINTER(C.c_int64)]),
    ("hmc_default_replica", C.c_int, [C.POINTER(hmc_replica), C.POINTER(hmc_params), C.c_int32, C.c_int32]),
    ("hmc_batch_workspace_bytes", C.c_size_t, [C.POINTER(hmc_params), C.c_int32, C.POINTER(hmc_replica)]),
    ("hmc_batch_create", C.c_int, [C.POINTER(hmc_params), C.c_int32, C.POINTER(hmc_replica), C.c_void_p,
                                   C.c_size_t, C.c_void_p, C.POINTER(C.c_void_p)]),
    ("hmc_batch_set_replica", C.c_int, [C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p]),
    ("hmc_batch_get_spins", C.c_int, [C.c_void_p, C.c_int32, C.c_void_p]),
    ("hmc_batch_get_stress", C.c_int, [C.c_void_p, C.c_int32, C.c_void_p]),
    ("hmc_batch_energy", C.c_int, [C.c_void_p, C.c_int32, C.POINTER(C.c_int64), C.POINTER(C.c_double)]),
    ("hmc_batch_texture_histogram", C.c_int, [C.c_void_p, C.c_int32, C.c_void_p, C.c_double, C.c_int32,
                                              C.c_void_p]),
    ("hmc_adjoint_workspace_bytes", C.c_size_t, [C.c_void_p, C.c_int32, C.c_int32]),
    ("hmc_elastic_forward", C.c_int, [C.c_void_p, C.c_int32, C.c_int32, C.c_void_p, C.c_size_t,
                                      C.POINTER(C.c_double)]),
    ("hmc_elastic_backward", C.c_int, [C.c_void_p, C.c_void_p, C.c_size_t, C.c_double, C.c_void_p, C.c_void_p]),
    ("hmc_grain_tables", C.c_int, [C.c_void_p, C.c_int32, C.c_double, C.c_double, C.c_double, C.c_void_p,
                                   C.c_void_p]),
    ("hmc_grain_table_derivatives", C.c_int, [C.c_void_p, C.c_int32, C.c_double, C.c_double, C.c_double,
                                              C.c_void_p, C.c_void_p]),
]


def lib():
    """Load libhmc.so (built by paper_1009_0457_amd.build); raises if it is missing."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"HIP library not built: {LIB_PATH} (run paper_1009_0457_amd.build)")
        # torch (which supplies device memory and streams) is loaded first: with this
        # library's HIP runtime loaded before torch's, HIP has reported no visible device.
        import torch  # noqa: F401
        L = C.CDLL(LIB_PATH)
        for name, res, args in _SIGS:
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def exported_names():
    return [n for n, _, _ in _SIGS]


def _ptr(t):
    return C.c_void_p(int(t.data_ptr()))


def _check(status, ctx=None, creating=False):
    """Raise on a failed call.  A failed context creation has no context to hold its
    message; the library keeps it per thread (hmc_last_error(NULL))."""
    if status != HMC_OK:
        if ctx:
            msg = lib().hmc_last_error(ctx).decode()
        else:
            msg = lib().hmc_last_error(None).decode() if creating else ""
        raise HmcError(status, msg)


# ---- same-name wrappers --------------------------------------------------------------
def hmc_default_params(K, neighbors, zone_h) -> hmc_params:
    p = hmc_params()
    _check(lib().hmc_default_params(C.byref(p), K, neighbors, zone_h))
    return p


def hmc_workspace_bytes(p: hmc_params, Q: int) -> int:
    return int(lib().hmc_workspace_bytes(C.byref(p), Q))


def hmc_create(p: hmc_params, Q: int, workspace, stream_handle: int):
    ctx = C.c_void_p()
    _check(lib().hmc_create(C.byref(p), Q, _ptr(workspace), workspace.numel(), C.c_void_p(stream_handle),
                            C.byref(ctx)), creating=True)
    return ctx


def hmc_destroy(ctx):
    lib().hmc_destroy(ctx)


def hmc_last_error(ctx) -> str:
    return lib().hmc_last_error(ctx).decode()


def hmc_set_orientations(ctx, euler):
    e = np.ascontiguousarray(euler, np.float64)
    _check(lib().hmc_set_orientations(ctx, e.ctypes.data_as(C.c_void_p)), ctx)


def hmc_set_spins(ctx, spins_dev):
    assert spins_dev.dtype.itemsize == 4 and spins_dev.is_contiguous() and spins_dev.is_cuda
    _check(lib().hmc_set_spins(ctx, _ptr(spins_dev)), ctx)


def hmc_get_spins(ctx, out_dev):
    assert out_dev.is_cuda and out_dev.is_contiguous()
    _check(lib().hmc_get_spins(ctx, _ptr(out_dev)), ctx)


def hmc_set_load(ctx, sigma_MPa):
    s = np.ascontiguousarray(sigma_MPa, np.float64)
    assert s.shape == (6,)
    _check(lib().hmc_set_load(ctx, s.ctypes.data_as(C.c_void_p)), ctx)


def hmc_stress_refresh(ctx, n_steps, cold_start):
    _check(lib().hmc_stress_refresh(ctx, int(n_steps), int(cold_start)), ctx)


def hmc_sweep(ctx, n):
    _check(lib().hmc_sweep(ctx, int(n)), ctx)


def hmc_colour_pass(ctx, colour, records_dev=None):
    _check(lib().hmc_colour_pass(ctx, int(colour), None if records_dev is None else _ptr(records_dev)), ctx)


def hmc_energy(ctx):
    n = C.c_int64()
    u = C.c_double()
    _check(lib().hmc_energy(ctx, C.byref(n), C.byref(u)), ctx)
    return int(n.value), float(u.value)


def hmc_texture_histogram(ctx, axis, bin_deg=10.0, nbins=6):
    a = np.ascontiguousarray(axis, np.float64)
    out = np.zeros(nbins, np.int64)
    _check(lib().hmc_texture_histogram(ctx, a.ctypes.data_as(C.c_void_p), float(bin_deg), int(nbins),
                                       out.ctypes.data_as(C.c_void_p)), ctx)
    return out


def hmc_texture_histogram_noalloc(spins_dev, K, euler, axis, bin_deg=10.0, nbins=6, stream_handle=0):
    """The texture histogram of a device spin field (K^3 int32) without a context or workspace
    (the library's static scratch array); synchronises ``stream_handle``."""
    e = np.ascontiguousarray(euler, np.float64)
    a = np.ascontiguousarray(axis, np.float64)
    if (e.ndim != 2 or e.shape[1] != 3 or spins_dev.numel() != K ** 3 or str(spins_dev.dtype) != "torch.int32"
            or not spins_dev.is_contiguous() or not spins_dev.is_cuda):
        raise HmcError(HMC_EINVAL, "euler must be (Q, 3) and spins a contiguous device tensor of K^3 int32")
    out = np.zeros(nbins, np.int64)
    st = lib().hmc_texture_histogram_noalloc(_ptr(spins_dev), int(K), int(e.shape[0]), e.ctypes.data_as(C.c_void_p),
                                             a.ctypes.data_as(C.c_void_p), float(bin_deg), int(nbins),
                                             out.ctypes.data_as(C.c_void_p), C.c_void_p(stream_handle))
    _check(st, None, creating=True)
    return out


def hmc_set_block_order(ctx, order):
    _check(lib().hmc_set_block_order(ctx, int(order)), ctx)


def hmc_get_stress(ctx, out_dev):
    _check(lib().hmc_get_stress(ctx, _ptr(out_dev)), ctx)


def hmc_set_stress(ctx, in_dev):
    _check(lib().hmc_set_stress(ctx, _ptr(in_dev)), ctx)


def hmc_get_displacement(ctx, out_dev):
    _check(lib().hmc_get_displacement(ctx, _ptr(out_dev)), ctx)


def hmc_get_macro_strain(ctx):
    E = np.zeros(6)
    _check(lib().hmc_get_macro_strain(ctx, E.ctypes.data_as(C.c_void_p)), ctx)
    return E


def hmc_set_elastic_state(ctx, u_dev, E):
    e = np.ascontiguousarray(E, np.float64)
    _check(lib().hmc_set_elastic_state(ctx, _ptr(u_dev), e.ctypes.data_as(C.c_void_p)), ctx)


def hmc_set_sweep_index(ctx, s):
    _check(lib().hmc_set_sweep_index(ctx, int(s)), ctx)


def hmc_get_sweep_index(ctx):
    s = C.c_int64()
    _check(lib().hmc_get_sweep_index(ctx, C.byref(s)), ctx)
    return int(s.value)


def hmc_get_stats(ctx) -> dict:
    st = hmc_stats()
    _check(lib().hmc_get_stats(ctx, C.byref(st)), ctx)
    return {k: int(getattr(st, k)) for k, _ in st._fields_}


def hmc_reset_stats(ctx):
    _check(lib().hmc_reset_stats(ctx), ctx)


def hmc_set_zone_screen(ctx, enable):
    _check(lib().hmc_set_zone_screen(ctx, int(bool(enable))), ctx)


def hmc_set_zone_variant(ctx, variant):
    _check(lib().hmc_set_zone_variant(ctx, int(variant)), ctx)


def hmc_set_profiling(ctx, enable):
    _check(lib().hmc_set_profiling(ctx, int(bool(enable))), ctx)


def hmc_get_kernel_times(ctx) -> dict:
    kt = hmc_kernel_times()
    _check(lib().hmc_get_kernel_times(ctx, C.byref(kt)), ctx)
    return {k: {"launches": int(getattr(kt, k).launches), "total_ms": float(getattr(kt, k).total_ms)}
            for k, _ in kt._fields_}


def hmc_set_graphs(ctx, enable):
    _check(lib().hmc_set_graphs(ctx, int(bool(enable))), ctx)


def hmc_set_material_points(p: hmc_params, n: int) -> hmc_params:
    _check(lib().hmc_set_material_points(C.byref(p), int(n)))
    return p


def hmc_default_replica(common: hmc_params, K, Q) -> hmc_replica:
    r = hmc_replica()
    _check(lib().hmc_default_replica(C.byref(r), C.byref(common), K, Q))
    return r


def _rep_array(reps):
    arr = (hmc_replica * len(reps))()
    for i, r in enumerate(reps):
        arr[i] = r
    return arr


def hmc_batch_workspace_bytes(common: hmc_params, reps) -> int:
    return int(lib().hmc_batch_workspace_bytes(C.byref(common), len(reps), _rep_array(reps)))


def hmc_batch_create(common: hmc_params, reps, workspace, stream_handle: int):
    ctx = C.c_void_p()
    _check(lib().hmc_batch_create(C.byref(common), len(reps), _rep_array(reps), _ptr(workspace), workspace.numel(),
                                  C.c_void_p(stream_handle), C.byref(ctx)), creating=True)
    return ctx


def hmc_batch_set_replica(ctx, r, euler, spins_dev):
    e = np.ascontiguousarray(euler, np.float64)
    _check(lib().hmc_batch_set_replica(ctx, int(r), e.ctypes.data_as(C.c_void_p), _ptr(spins_dev)), ctx)


def hmc_batch_get_spins(ctx, r, out_dev):
    _check(lib().hmc_batch_get_spins(ctx, int(r), _ptr(out_dev)), ctx)


def hmc_batch_get_stress(ctx, r, out_dev):
    _check(lib().hmc_batch_get_stress(ctx, int(r), _ptr(out_dev)), ctx)


def hmc_batch_energy(ctx, r):
    n = C.c_int64()
    u = C.c_double()
    _check(lib().hmc_batch_energy(ctx, int(r), C.byref(n), C.byref(u)), ctx)
    return int(n.value), float(u.value)


def hmc_batch_texture_histogram(ctx, r, axis, bin_deg=10.0, nbins=6):
    a = np.ascontiguousarray(axis, np.float64)
    out = np.zeros(nbins, np.int64)
    _check(lib().hmc_batch_texture_histogram(ctx, int(r), a.ctypes.data_as(C.c_void_p), float(bin_deg), int(nbins),
                                             out.ctypes.data_as(C.c_void_p)), ctx)
    return out


def hmc_grain_labels(ctx, r, labels_dev) -> int:
    n = C.c_int64()
    _check(lib().hmc_grain_labels(ctx, int(r), _ptr(labels_dev), C.byref(n)), ctx)
    return int(n.value)


def hmc_grain_tables(euler, C11, C12, C44):
    e = np.ascontiguousarray(euler, np.float64)
    Q = e.shape[0]
    Cl = np.zeros((Q, 6, 6))
    Sl = np.zeros((Q, 6, 6))
    _check(lib().hmc_grain_tables(e.ctypes.data_as(C.c_void_p), Q, C11, C12, C44,
                                  Cl.ctypes.data_as(C.c_void_p), Sl.ctypes.data_as(C.c_void_p)))
    return Cl, Sl


def hmc_adjoint_workspace_bytes(ctx, n_steps, ckpt_every) -> int:
    return int(lib().hmc_adjoint_workspace_bytes(ctx, int(n_steps), int(ckpt_every)))


def hmc_elastic_forward(ctx, n_steps, ckpt_every, adj_ws):
    U = C.c_double()
    _check(lib().hmc_elastic_forward(ctx, int(n_steps), int(ckpt_every), _ptr(adj_ws), adj_ws.numel(), C.byref(U)),
           ctx)
    return float(U.value)


def hmc_elastic_backward(ctx, adj_ws, dU, Q):
    ge = np.zeros((Q, 3))
    gs = np.zeros(6)
    _check(lib().hmc_elastic_backward(ctx, _ptr(adj_ws), adj_ws.numel(), float(dU), ge.ctypes.data_as(C.c_void_p),
                                      gs.ctypes.data_as(C.c_void_p)), ctx)
    return ge, gs


def hmc_grain_table_derivatives(euler, C11, C12, C44):
    e = np.ascontiguousarray(euler, np.float64)
    Q = e.shape[0]
    dC = np.zeros((Q, 3, 6, 6))
    dS = np.zeros((Q, 3, 6, 6))
    _check(lib().hmc_grain_table_derivatives(e.ctypes.data_as(C.c_void_p), Q, C11, C12, C44,
                                             dC.ctypes.data_as(C.c_void_p), dS.ctypes.data_as(C.c_void_p)))
    return dC, dS


# ---- convenience owner ------------------------------------------------------------------
class Lattice:
    """One context plus its torch-allocated workspace on ``device``.

    ``params`` may be an hmc_params or a dict of overrides on the defaults of
    (K, neighbors, zone_h)."""

    def __init__(self, params, Q, device="cuda:0", stream=None):
        import torch

        if not torch.cuda.is_available():
            raise RuntimeError("the HMC library needs a HIP device; none is visible")
        self.torch = torch
        self.device = torch.device(device)
        if isinstance(params, dict):
            d = dict(params)
            p = hmc_default_params(d.pop("K"), d.pop("neighbors"), d.pop("zone_h"))
            for k, v in d.items():
                setattr(p, k, v)
            params = p
        self.params = params
        self.Q = int(Q)
        self.K = params.K
        self.n3 = params.K ** 3
        nbytes = hmc_workspace_bytes(params, self.Q)
        if nbytes == 0:
            raise HmcError(HMC_EINVAL, "invalid parameters")
        with torch.cuda.device(self.device):
            self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
            self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
            self.ctx = hmc_create(params, self.Q, self.workspace, self.stream.cuda_stream)

    def close(self):
        if getattr(self, "ctx", None) is not None:
            hmc_destroy(self.ctx)
            self.ctx = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # thin pass-throughs
    def set_orientations(self, euler):
        hmc_set_orientations(self.ctx, euler)

    def set_spins(self, spins):
        t = self.torch.as_tensor(np.asarray(spins, np.int32) if not hasattr(spins, "is_cuda") else spins)
        t = t.to(device=self.device, dtype=self.torch.int32).contiguous()
        hmc_set_spins(self.ctx, t)

    def get_spins(self):
        out = self.torch.empty(self.n3, dtype=self.torch.int32, device=self.device)
        hmc_get_spins(self.ctx, out)
        return out

    def set_load(self, sigma_MPa):
        hmc_set_load(self.ctx, sigma_MPa)

    def stress_refresh(self, n_steps=-1, cold_start=False):
        hmc_stress_refresh(self.ctx, n_steps, cold_start)

    def sweep(self, n=1):
        hmc_sweep(self.ctx, n)

    def colour_pass(self, colour, records=False):
        rec = None
        if records:
            rec = self.torch.zeros(self.n3 * record_dtype.itemsize, dtype=self.torch.uint8, device=self.device)
        hmc_colour_pass(self.ctx, colour, rec)
        if rec is None:
            return None
        self.stream.synchronize()
        return rec.cpu().numpy().view(record_dtype)

    def energy(self):
        return hmc_energy(self.ctx)

    def texture_histogram(self, axis, bin_deg=10.0, nbins=6):
        return hmc_texture_histogram(self.ctx, axis, bin_deg, nbins)

    def grain_labels(self):
        """(per-site grain labels on the device, number of grains)."""
        out = self.torch.empty(self.n3, dtype=self.torch.int32, device=self.device)
        n = hmc_grain_labels(self.ctx, 0, out)
        return out, n

    def get_stress(self):
        out = self.torch.empty((6, self.n3), dtype=self.torch.float32, device=self.device)
        hmc_get_stress(self.ctx, out)
        return out

    def set_stress(self, sig):
        t = self.torch.as_tensor(sig).to(device=self.device, dtype=self.torch.float32).contiguous()
        assert t.numel() == 6 * self.n3
        hmc_set_stress(self.ctx, t)
        self._keep = t

    def get_displacement(self):
        out = self.torch.empty((3, self.n3), dtype=self.torch.float32, device=self.device)
        hmc_get_displacement(self.ctx, out)
        return out

    def macro_strain(self):
        return hmc_get_macro_strain(self.ctx)

    def set_elastic_state(self, u, E):
        t = self.torch.as_tensor(u).to(device=self.device, dtype=self.torch.float32).contiguous()
        hmc_set_elastic_state(self.ctx, t, E)

    def set_sweep_index(self, s):
        hmc_set_sweep_index(self.ctx, s)

    def sweep_index(self):
        return hmc_get_sweep_index(self.ctx)

    def stats(self):
        return hmc_get_stats(self.ctx)

    def reset_stats(self):
        hmc_reset_stats(self.ctx)

    def set_zone_screen(self, enable=True):
        hmc_set_zone_screen(self.ctx, enable)

    def set_zone_variant(self, variant):
        hmc_set_zone_variant(self.ctx, variant)

    def set_profiling(self, enable=True):
        hmc_set_profiling(self.ctx, enable)

    def kernel_times(self):
        return hmc_get_kernel_times(self.ctx)

    def set_graphs(self, enable=True):
        hmc_set_graphs(self.ctx, enable)

    def set_block_order(self, order):
        hmc_set_block_order(self.ctx, order)

    def synchronize(self):
        self.stream.synchronize()

    # adjoint of the global solve
    def elastic_forward(self, n_steps, ckpt_every=50):
        nbytes = hmc_adjoint_workspace_bytes(self.ctx, n_steps, ckpt_every)
        if getattr(self, "adj_ws", None) is None or self.adj_ws.numel() < nbytes:
            self.adj_ws = self.torch.empty(nbytes, dtype=self.torch.uint8, device=self.device)
        U = hmc_elastic_forward(self.ctx, n_steps, ckpt_every, self.adj_ws)
        # counts forwards: an autograd node remembers the one its backward belongs to
        self.adj_generation = getattr(self, "adj_generation", 0) + 1
        return U

    def elastic_backward(self, dU=1.0):
        return hmc_elastic_backward(self.ctx, self.adj_ws, dU, self.Q)


def _make_energy_function():
    import torch

    class StoredElasticEnergy(torch.autograd.Function):
        """U(euler, sigma_MPa): stored elastic energy (GPa*voxel) after the global explicit
        solve of ``n_steps`` from a cold start on ``lattice`` (its spins); the backward is the
        library's hand-written adjoint with checkpoints every ``ckpt_every`` steps."""

        @staticmethod
        def forward(ctx, euler, sigma_MPa, lattice, n_steps, ckpt_every):
            lattice.set_orientations(euler.detach().cpu().double().numpy())
            lattice.set_load(sigma_MPa.detach().cpu().double().numpy())
            U = lattice.elastic_forward(int(n_steps), int(ckpt_every))
            ctx.lattice = lattice
            ctx.generation = lattice.adj_generation
            ctx.shapes = (euler.shape, euler.dtype, sigma_MPa.dtype, euler.device, sigma_MPa.device)
            return torch.tensor(U, dtype=torch.float64)

        @staticmethod
        def backward(ctx, gU):
            shape, edt, sdt, edev, sdev = ctx.shapes
            if ctx.lattice.adj_generation != ctx.generation:
                # the lattice's checkpoints now belong to a later forward (another
                # stored_elastic_energy call on the same lattice): this node's gradient is gone
                raise RuntimeError("stored_elastic_energy: another forward ran on this lattice before this "
                                   "backward; evaluate one energy per lattice per backward")
            ge, gs = ctx.lattice.elastic_backward(float(gU))
            return (torch.from_numpy(ge).reshape(shape).to(dtype=edt, device=edev),
                    torch.from_numpy(gs).to(dtype=sdt, device=sdev), None, None, None)

    return StoredElasticEnergy


_energy_fn = None


def stored_elastic_energy(euler, sigma_MPa, lattice, n_steps=2000, ckpt_every=50):
    """Differentiable stored elastic energy; ``euler`` (Q, 3) and ``sigma_MPa`` (6,) tensors."""
    global _energy_fn
    if _energy_fn is None:
        _energy_fn = _make_energy_function()
    return _energy_fn.apply(euler, sigma_MPa, lattice, n_steps, ckpt_every)


def orientation_driving_force(lattice, euler, sigma_MPa, n_steps=2000, ckpt_every=50):
    """-dU/dtheta per grain (Q, 3): the elastic driving force on each grain's orientation, the
    term the texture rate equation of Sec. 7 is driven by (rotating a grain along it lowers
    the stored energy)."""
    lattice.set_orientations(np.asarray(euler, np.float64))
    lattice.set_load(np.asarray(sigma_MPa, np.float64))
    lattice.elastic_forward(n_steps, ckpt_every)
    ge, _ = lattice.elastic_backward(1.0)
    return -ge


class Batch(Lattice):
    """Many replicas fused into every launch (one context).  ``reps`` is a list of
    hmc_replica; ``common`` an hmc_params.  Runs on its own (non-null) torch stream so that
    sweeps can be captured into HIP graphs."""

    def __init__(self, common, reps, device="cuda:0", stream=None):
        import torch

        if not torch.cuda.is_available():
            raise RuntimeError("the HMC library needs a HIP device; none is visible")
        self.torch = torch
        self.device = torch.device(device)
        self.params = common
        self.reps = list(reps)
        self.n3s = [r.K ** 3 for r in self.reps]
        nbytes = hmc_batch_workspace_bytes(common, self.reps)
        if nbytes == 0:
            raise HmcError(HMC_EINVAL, "invalid batch description")
        with torch.cuda.device(self.device):
            self.stream = stream if stream is not None else torch.cuda.Stream(self.device)
            self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=self.device)
            torch.cuda.synchronize(self.device)
            self.ctx = hmc_batch_create(common, self.reps, self.workspace, self.stream.cuda_stream)

    def set_replica(self, r, euler, spins):
        t = self.torch.as_tensor(np.asarray(spins, np.int32)).to(self.device)
        self.torch.cuda.synchronize(self.device)
        hmc_batch_set_replica(self.ctx, r, euler, t)

    def get_spins(self, r=0):
        out = self.torch.empty(self.n3s[r], dtype=self.torch.int32, device=self.device)
        hmc_batch_get_spins(self.ctx, r, out)
        self.stream.synchronize()
        return out

    def get_stress(self, r=0):
        out = self.torch.empty((6, self.n3s[r]), dtype=self.torch.float32, device=self.device)
        hmc_batch_get_stress(self.ctx, r, out)
        self.stream.synchronize()
        return out

    def colour_pass(self, colour, records=False):
        """One colour pass of every replica; with records, the per-trial records of all
        replicas laid end to end (replica r's sites from the sum of the earlier replicas' K^3)."""
        rec = None
        n = sum(self.n3s)
        if records:
            rec = self.torch.zeros(n * record_dtype.itemsize, dtype=self.torch.uint8, device=self.device)
        hmc_colour_pass(self.ctx, colour, rec)
        if rec is None:
            return None
        self.stream.synchronize()
        return rec.cpu().numpy().view(record_dtype)

    def energy(self, r=0):
        return hmc_batch_energy(self.ctx, r)

    def grain_labels(self, r=0):
        out = self.torch.empty(self.n3s[r], dtype=self.torch.int32, device=self.device)
        n = hmc_grain_labels(self.ctx, r, out)
        return out, n

    def texture_histogram(self, axis, bin_deg=10.0, nbins=6, r=0):
        return hmc_batch_texture_histogram(self.ctx, r, axis, bin_deg, nbins)

    def synchronize(self):
        self.stream.synchronize()
