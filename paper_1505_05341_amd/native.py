"""Thin ctypes binding of libpk (include/pk.h): argument marshalling only.

Every step of the estimator runs in the library's HIP kernels; this module only
turns torch device tensors into pointers, passes torch's current HIP stream, and
converts the host results into numpy arrays. It fails loudly when the library is
missing: there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os
from ctypes import POINTER, c_char_p, c_double, c_int32, c_int64, c_size_t, c_void_p

import numpy as np

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libpk.so")

PK_OK = 0
STATUS_NAMES = {0: "PK_OK", -1: "PK_EINVAL", -2: "PK_ERANGE", -3: "PK_EDOM", -4: "PK_EWORKSPACE",
                -5: "PK_EDEVICE", -6: "PK_ENOTSUP"}


class PkError(RuntimeError):
    def __init__(self, status, detail):
        self.status = status
        super().__init__("%s (%d): %s" % (STATUS_NAMES.get(status, "?"), status, detail))


class PkCatalog(ctypes.Structure):
    _fields_ = [("xyz", c_void_p), ("w", c_void_p), ("nbar", c_void_p), ("n", c_int64)]


class PkConfig(ctypes.Structure):
    _fields_ = [("N", c_int32), ("assign", c_int32), ("ell_max", c_int32), ("los", c_int32),
                ("compensate", c_int32), ("dn", c_int32), ("nbins", c_int32), ("norm_from", c_int32),
                ("box_min", c_double * 3), ("L", c_double), ("observer", c_double * 3), ("x_planes", c_int32)]


class PkResult(ctypes.Structure):
    _fields_ = [("k_eff", POINTER(c_double)), ("P", POINTER(c_double)), ("noise", POINTER(c_double)),
                ("nmodes", POINTER(c_int64)), ("alpha", c_double), ("I", c_double), ("S", c_double),
                ("wedges", POINTER(c_double))]


EXPORTS = ["pk_workspace_size", "pk_multipoles", "pk_multipoles_async", "pk_result_doubles",
           "pk_stage_xgrids", "pk_xgrid_layout", "pk_num_grids", "pk_monomial", "pk_status_string",
           "pk_last_error", "pk_last_error_detail", "pk_set_stage_timing", "pk_stage_times", "pk_stage_name",
           "pk_workspace_size_batch", "pk_multipoles_batch", "pk_set_schedule", "pk_get_schedule", "pk_autotune",
           "pk_x_planes", "pk_stage_fft", "pk_stage_contract", "pk_hgrid_layout", "pk_zgroup", "pk_ygroup_terms"]

_lib = None


def load():
    """Load libpk.so (built by paper_1505_05341_amd.build) and declare its signatures."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError("libpk.so is not built (%s); run `python -m paper_1505_05341_amd.build`" % LIB_PATH)
    lib = ctypes.CDLL(LIB_PATH)
    P = POINTER
    lib.pk_workspace_size.argtypes = [P(PkConfig), c_int64, c_int64, P(c_size_t)]
    lib.pk_multipoles.argtypes = [P(PkConfig), P(PkCatalog), P(PkCatalog), c_void_p, c_size_t, P(PkResult), c_void_p]
    lib.pk_multipoles_async.argtypes = [P(PkConfig), P(PkCatalog), P(PkCatalog), c_void_p, c_size_t, c_void_p,
                                        c_void_p]
    lib.pk_result_doubles.argtypes = [P(PkConfig)]
    lib.pk_result_doubles.restype = c_int64
    lib.pk_stage_xgrids.argtypes = [P(PkConfig), P(PkCatalog), P(PkCatalog), c_void_p, c_size_t, c_void_p]
    lib.pk_xgrid_layout.argtypes = [P(PkConfig), c_int64, c_int64, c_int32, P(c_size_t), P(c_int32)]
    lib.pk_x_planes.argtypes = [P(PkConfig), c_int64, c_int64, P(c_int32)]
    lib.pk_stage_fft.argtypes = [P(PkConfig), P(PkCatalog), P(PkCatalog), c_void_p, c_size_t, c_void_p]
    lib.pk_stage_contract.argtypes = [P(PkConfig), c_int64, c_int64, c_void_p, c_size_t, P(PkResult), c_void_p]
    lib.pk_hgrid_layout.argtypes = [P(PkConfig), c_int64, c_int64, c_int32, c_int32, P(c_size_t), P(c_int32),
                                    P(c_int32)]
    lib.pk_zgroup.argtypes = [c_int32, c_int32, P(c_int32), P(c_int32)]
    lib.pk_ygroup_terms.argtypes = [c_int32, c_int32, c_int32, P(c_int32), P(c_int32), P(c_int32),
                                    P(ctypes.c_float), P(c_int32), P(c_int32)]
    lib.pk_ygroup_terms.restype = c_int32
    lib.pk_num_grids.argtypes = [c_int32]
    lib.pk_num_grids.restype = c_int32
    lib.pk_monomial.argtypes = [c_int32, P(c_int32), P(c_int32), P(c_int32)]
    lib.pk_status_string.argtypes = [c_int32]
    lib.pk_status_string.restype = c_char_p
    lib.pk_last_error.argtypes = [ctypes.c_char_p, c_size_t]
    lib.pk_last_error.restype = c_size_t
    lib.pk_last_error_detail.argtypes = [ctypes.c_char_p, c_size_t]
    lib.pk_last_error_detail.restype = c_size_t
    lib.pk_workspace_size_batch.argtypes = [P(PkConfig), P(PkCatalog), P(PkCatalog), c_int32, c_int32, P(c_size_t)]
    lib.pk_multipoles_batch.argtypes = [P(PkConfig), P(PkCatalog), P(PkCatalog), c_int32, c_int32, c_void_p, c_size_t,
                                        P(PkResult), P(c_int32), c_void_p]
    lib.pk_set_schedule.argtypes = [c_int32, c_int32, c_int32, c_int32]
    lib.pk_get_schedule.argtypes = [c_int32, c_int32, P(c_int32), P(c_int32)]
    lib.pk_autotune.argtypes = [P(PkConfig), P(PkCatalog), P(PkCatalog), c_void_p, c_size_t, c_int32, P(c_int32),
                                P(c_int32), c_void_p]
    lib.pk_set_stage_timing.argtypes = [c_int32]
    lib.pk_stage_times.argtypes = [POINTER(c_double), c_int32]
    lib.pk_stage_times.restype = c_int32
    lib.pk_stage_name.argtypes = [c_int32]
    lib.pk_stage_name.restype = c_char_p
    for name in EXPORTS:
        getattr(lib, name).restype = getattr(lib, name).restype if name in (
            "pk_result_doubles", "pk_num_grids", "pk_status_string", "pk_last_error", "pk_last_error_detail",
            "pk_ygroup_terms", "pk_stage_times",
            "pk_stage_name") else c_int32
    _lib = lib
    return lib


def ygroup_terms(ell_max, max_groups):
    """The y pass's weight table (pk_ygroup_terms) as a list of (set, group, grid, coef, a, b)."""
    lib = load()
    n = lib.pk_ygroup_terms(int(ell_max), int(max_groups), 0, None, None, None, None, None, None)
    if n < 0:
        raise PkError(-1, last_error())
    arr = {k: (c_int32 * n)() for k in ("set", "group", "grid", "a", "b")}
    coef = (ctypes.c_float * n)()
    lib.pk_ygroup_terms(int(ell_max), int(max_groups), n, arr["set"], arr["group"], arr["grid"], coef, arr["a"],
                        arr["b"])
    return [(arr["set"][i], arr["group"][i], arr["grid"][i], coef[i], arr["a"][i], arr["b"][i]) for i in range(n)]


def last_error():
    lib = load()
    buf = ctypes.create_string_buffer(1024)
    lib.pk_last_error(buf, 1024)
    return buf.value.decode()


def check(status):
    if status != PK_OK:
        raise PkError(status, last_error())


def make_config(cfg: dict) -> PkConfig:
    c = PkConfig()
    c.N = cfg["N"]
    c.assign = cfg.get("assign", 2)
    c.ell_max = cfg.get("ell_max", 4)
    c.los = cfg.get("los", 0)
    c.compensate = cfg.get("compensate", 2)
    c.dn = cfg.get("dn", 1)
    c.nbins = cfg.get("nbins", 0) or cfg["N"] // (2 * c.dn)
    c.norm_from = cfg.get("norm_from", 0)
    for i in range(3):
        c.box_min[i] = cfg["box_min"][i]
        c.observer[i] = cfg.get("observer", (0.0, 0.0, 0.0))[i]
    c.L = cfg["L"]
    c.x_planes = cfg.get("x_planes", 0)
    return c


def _ptr(t):
    return None if t is None else c_void_p(t.data_ptr())


def make_catalog(pos, w, nbar=None) -> PkCatalog:
    """pos (n, 3), w (n,), nbar (n,) float32 contiguous CUDA tensors (nbar may be None).
    Shapes and dtypes are checked here: the kernels read n positions, weights and
    densities, so a shorter array would be read past its end on the device."""
    import torch
    for t in (pos, w) + ((nbar,) if nbar is not None else ()):
        if not t.is_cuda or t.dtype != torch.float32 or not t.is_contiguous():
            raise ValueError("catalogue arrays must be contiguous float32 device tensors")
    if pos.dim() != 2 or pos.shape[1] != 3:
        raise ValueError("positions must have shape (n, 3), got %s" % (tuple(pos.shape),))
    n = int(pos.shape[0])
    if w.dim() != 1 or w.numel() != n:
        raise ValueError("weights must have shape (%d,), got %s" % (n, tuple(w.shape)))
    if nbar is not None and (nbar.dim() != 1 or nbar.numel() != n):
        raise ValueError("nbar must have shape (%d,), got %s" % (n, tuple(nbar.shape)))
    c = PkCatalog()
    c.xyz = _ptr(pos)
    c.w = _ptr(w)
    c.nbar = _ptr(nbar)
    c.n = int(pos.shape[0])
    return c


def workspace_size(cfg: dict, n_gal: int, n_ran: int) -> int:
    lib = load()
    out = c_size_t(0)
    check(lib.pk_workspace_size(ctypes.byref(make_config(cfg)), n_gal, n_ran, ctypes.byref(out)))
    return int(out.value)


def x_planes(cfg: dict, n_gal: int, n_ran: int) -> int:
    """Slab height (z planes of the x-transformed grids held at once) of this plan."""
    out = c_int32(0)
    check(load().pk_x_planes(ctypes.byref(make_config(cfg)), n_gal, n_ran, ctypes.byref(out)))
    return int(out.value)


def num_grids(ell_max: int) -> int:
    return int(load().pk_num_grids(ell_max))


def monomial(m: int):
    a, b, c = c_int32(), c_int32(), c_int32()
    check(load().pk_monomial(m, ctypes.byref(a), ctypes.byref(b), ctypes.byref(c)))
    return (a.value, b.value, c.value)


def current_stream():
    import torch
    return c_void_p(torch.cuda.current_stream().cuda_stream)


def set_stage_timing(enable: bool):
    check(load().pk_set_stage_timing(1 if enable else 0))


def stage_times():
    """{stage name: ms} of the last timed call (waits for its events)."""
    lib = load()
    buf = (c_double * 16)()
    n = lib.pk_stage_times(buf, 16)
    if n < 0:
        raise RuntimeError("no timed call recorded")
    return {lib.pk_stage_name(i).decode(): float(buf[i]) for i in range(n)}


def set_schedule(N, ell_max, y_values, z_values):
    """Values per thread (8 or 16) of the y- and z-pass column transforms for (N, ell_max)."""
    check(load().pk_set_schedule(int(N), int(ell_max), int(y_values), int(z_values)))


def get_schedule(N, ell_max):
    y, z = ctypes.c_int32(), ctypes.c_int32()
    check(load().pk_get_schedule(int(N), int(ell_max), ctypes.byref(y), ctypes.byref(z)))
    return int(y.value), int(z.value)


def zgroup(ell_max, g):
    """(degree n, power c of tz) of z-power group g."""
    n, c = c_int32(), c_int32()
    check(load().pk_zgroup(int(ell_max), int(g), ctypes.byref(n), ctypes.byref(c)))
    return int(n.value), int(c.value)
