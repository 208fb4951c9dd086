"""Least-misfit gridding and degridding on AMD MI355X (gfx950).

Thin Python binding over the C ABI of ``liblmgrid.so`` (declared in
``include/lmgrid.h``). Every step of the path runs in the library's HIP
kernels; this module only marshals torch tensors (device memory and the
current stream) into pointers. If the library is not built, importing works
but every call raises :class:`LibraryMissing` -- there is no fallback.

Method: Ye, Gull, Tan & Nikolic, "Optimal gridding and degridding in radio
interferometry imaging", MNRAS 2019.
"""
from __future__ import annotations

import ctypes
import os
from typing import Optional

import numpy as np

__all__ = [
    "F32", "F32_KAHAN", "F64", "LmgError", "LibraryMissing", "Table", "Plan", "BatchPlan", "autotune_batch",
    "library_path", "load", "grid", "degrid", "make_dirty_image", "predict_visibilities", "grid_batched",
    "degrid_batched", "fft2_centred", "sync_status", "trace_enable", "trace_only", "trace_report", "Degrid", "Grid", "PredictVisibilities",
    "MakeDirtyImage",
]

F32, F32_KAHAN, F64 = 0, 1, 2
OP_GRID, OP_DEGRID, OP_DIRTY, OP_PREDICT = 0, 1, 2, 3
NG = 32

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB = None


class LmgError(RuntimeError):
    """A non-zero lmg_status."""

    def __init__(self, status: int, what: str):
        self.status = status
        extra = ""
        if status == -3:
            extra = " [" + load().lmg_last_error().decode() + "]"
        super().__init__(f"{what}: {_status_string(status)} ({status}){extra}")


class LibraryMissing(RuntimeError):
    pass


def library_path() -> str:
    return os.path.join(_HERE, "liblmgrid.so")


def _status_string(s: int) -> str:
    lib = load()
    return lib.lmg_status_string(s).decode()


def load():
    """Load the in-tree HIP library (raises LibraryMissing if it was not built)."""
    global _LIB
    if _LIB is not None:
        return _LIB
    path = library_path()
    if not os.path.exists(path):
        raise LibraryMissing(f"{path} not found: build it with `python -m paper_1906_07102_amd.build`")
    lib = ctypes.CDLL(path)
    P, I, D, Z, I64 = ctypes.c_void_p, ctypes.c_int, ctypes.c_double, ctypes.c_size_t, ctypes.c_int64
    PD = ctypes.POINTER(ctypes.c_double)
    PI = ctypes.POINTER(ctypes.c_int)
    PZ = ctypes.POINTER(ctypes.c_size_t)
    sig = {
        "lmg_table_create": (I, [I, D, I, I, ctypes.POINTER(P)]),
        "lmg_table_create_from_h": (I, [I, D, I, I, PD, ctypes.POINTER(P)]),
        "lmg_table_create_from_nodes": (I, [I, D, I, I, PD, PD, ctypes.POINTER(P)]),
        "lmg_table_create_direct": (I, [P, ctypes.POINTER(P)]),
        "lmg_table_is_direct": (I, [P, PI]),
        "lmg_table_device_bytes": (I, [P, I, PZ]),
        "lmg_table_attach_device": (I, [P, I, P, Z, P]),
        "lmg_table_info": (I, [P, PI, PD, PI, PI, PD]),
        "lmg_table_export": (I, [P, PD, PD]),
        "lmg_table_kernel": (I, [P, I, PD, PD]),
        "lmg_correction": (I, [P, I, PD]),
        "lmg_map_error": (I, [P, I, PD, PD, PD]),
        "lmg_table_destroy": (None, [P]),
        "lmg_plan_workspace_size": (I, [I, I, I64, I, PZ]),
        "lmg_plan_create": (I, [P, I, I, I64, P, P, Z, P, ctypes.POINTER(P)]),
        "lmg_plan_check": (I, [P]),
        "lmg_plan_info": (I, [P, PI, PI, PI, ctypes.POINTER(I64)]),
        "lmg_plan_destroy": (None, [P]),
        "lmg_plan_scratch_size": (I, [P, I, PZ]),
        "lmg_grid_planned": (I, [P, P, P, P, I, P, Z, P]),
        "lmg_grid_planned_noalloc": (I, [P, P, P, P, I, P]),
        "lmg_degrid_planned": (I, [P, P, P, P, Z, P]),
        "lmg_plan_order_length": (I, [P, ctypes.POINTER(I64)]),
        "lmg_to_plan_order": (I, [P, P, P, P, P]),
        "lmg_from_plan_order": (I, [P, P, P, P]),
        "lmg_grid_planned_ordered": (I, [P, P, P, I, P, Z, P]),
        "lmg_degrid_planned_ordered": (I, [P, P, P, P, Z, P]),
        "lmg_make_dirty_image_planned": (I, [P, P, P, P, P, Z, P]),
        "lmg_predict_visibilities_planned": (I, [P, P, P, P, Z, P]),
        "lmg_workspace_size": (I, [I, I, D, I64, I, I, PZ]),
        "lmg_grid": (I, [P, I, I, I64, P, P, P, P, P, Z, P]),
        "lmg_degrid": (I, [P, I, I, I64, P, P, P, P, Z, P]),
        "lmg_make_dirty_image": (I, [P, I, I, I64, P, P, P, P, P, Z, P]),
        "lmg_predict_visibilities": (I, [P, I, I, I64, P, P, P, P, Z, P]),
        "lmg_fft2_centred": (I, [I, I, I, P, P, P]),
        "lmg_batch_workspace_size": (I, [I, I, I, I64, I, PZ]),
        "lmg_batch_plan_create": (I, [P, I, I, I, ctypes.POINTER(I64), P, I, P, Z, P, ctypes.POINTER(P)]),
        "lmg_batch_info": (I, [P, PI, PI, PI]),
        "lmg_workspace_size_batched": (I, [I, I, I, I64, I, I, PZ]),
        "lmg_grid_batched": (I, [P, I, I, I, ctypes.POINTER(I64), P, P, P, P, P, Z, P]),
        "lmg_degrid_batched": (I, [P, I, I, I, ctypes.POINTER(I64), P, P, P, P, Z, P]),
        "lmg_trace_enable": (I, [I]),
        "lmg_trace_report": (I, [ctypes.c_char_p, Z]),
        "lmg_trace_only": (I, [ctypes.c_char_p]),
        "lmg_sync_status": (I, [P]),
        "lmg_status_string": (ctypes.c_char_p, [I]),
        "lmg_last_error": (ctypes.c_char_p, []),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _LIB = lib
    return lib


def exported_symbols():
    """Names the C ABI exports (checked against the header by the library tests)."""
    load()
    return [n for n in dir(_LIB) if n.startswith("lmg_")]


def _check(status: int, what: str):
    if status != 0:
        raise LmgError(status, what)


def _dptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


# --------------------------------------------------------------------- tables
class Table:
    """A least-misfit gridding table (host object): h on 33 points, tabulated C, interpolation degree."""

    def __init__(self, handle):
        self._h = ctypes.c_void_p(handle) if not isinstance(handle, ctypes.c_void_p) else handle
        self._lib = load()
        W, x0, Ms, deg, E = ctypes.c_int(), ctypes.c_double(), ctypes.c_int(), ctypes.c_int(), ctypes.c_double()
        _check(self._lib.lmg_table_info(self._h, ctypes.byref(W), ctypes.byref(x0), ctypes.byref(Ms),
                                        ctypes.byref(deg), ctypes.byref(E)), "lmg_table_info")
        self.W, self.x0, self.Ms, self.degree, self.integrated_misfit = W.value, x0.value, Ms.value, deg.value, E.value
        self.table_size = self.W * self.Ms
        d = ctypes.c_int()
        _check(self._lib.lmg_table_is_direct(self._h, ctypes.byref(d)), "lmg_table_is_direct")
        self.direct = bool(d.value)

    @classmethod
    def create(cls, W: int, x0: float, table_size: int, degree: int = 3) -> "Table":
        out = ctypes.c_void_p()
        _check(load().lmg_table_create(W, x0, table_size, degree, ctypes.byref(out)), "lmg_table_create")
        return cls(out)

    @classmethod
    def from_h(cls, W: int, x0: float, table_size: int, degree: int, h) -> "Table":
        h = np.ascontiguousarray(h, dtype=np.float64)
        if h.shape != (NG + 1,):
            raise ValueError("h must have 33 samples")
        out = ctypes.c_void_p()
        _check(load().lmg_table_create_from_h(W, x0, table_size, degree, _dptr(h), ctypes.byref(out)),
               "lmg_table_create_from_h")
        return cls(out)

    @classmethod
    def from_nodes(cls, W: int, x0: float, table_size: int, degree: int, h, nodes) -> "Table":
        h = np.ascontiguousarray(h, dtype=np.float64)
        nodes = np.ascontiguousarray(nodes, dtype=np.float64)
        Ms = table_size // W
        if h.shape != (NG + 1,) or nodes.shape != (W, Ms + 1 + degree):
            raise ValueError("bad h or nodes shape")
        out = ctypes.c_void_p()
        _check(load().lmg_table_create_from_nodes(W, x0, table_size, degree, _dptr(h), _dptr(nodes),
                                                  ctypes.byref(out)), "lmg_table_create_from_nodes")
        return cls(out)

    def direct_calculation(self) -> "Table":
        """The same kernel evaluated exactly at each visibility's offset (no table), lmg_table_create_direct."""
        out = ctypes.c_void_p()
        _check(self._lib.lmg_table_create_direct(self._h, ctypes.byref(out)), "lmg_table_create_direct")
        return Table(out)

    def device_bytes(self, precision: int) -> int:
        """Bytes of the device copy the kernels read for a table too large for LDS (0 when staged in LDS)."""
        n = ctypes.c_size_t()
        _check(self._lib.lmg_table_device_bytes(self._h, int(precision), ctypes.byref(n)), "lmg_table_device_bytes")
        return n.value

    def attach_device(self, precision: int, device="cuda", stream=None):
        """Copy the coefficients of a table too large for LDS into a torch-owned device buffer kept by this
        object (lmg_table_attach_device); plans of that precision then read it. No-op when not needed."""
        n = self.device_bytes(precision)
        if n == 0:
            return None
        buf = _bytes(n, device)
        _check(self._lib.lmg_table_attach_device(self._h, int(precision), _ptr(buf), n, _stream_handle(stream)),
               "lmg_table_attach_device")
        if not hasattr(self, "_device_copies"):
            self._device_copies = {}
        self._device_copies[2 if precision == F64 else 0] = buf
        return buf

    def export(self):
        h = np.zeros(NG + 1)
        nodes = np.zeros((self.W, self.Ms + 1 + self.degree))
        _check(self._lib.lmg_table_export(self._h, _dptr(h), _dptr(nodes)), "lmg_table_export")
        return h, nodes

    def kernel(self, delta) -> np.ndarray:
        d = np.ascontiguousarray(np.atleast_1d(delta), dtype=np.float64)
        out = np.zeros((len(d), self.W))
        _check(self._lib.lmg_table_kernel(self._h, len(d), _dptr(d), _dptr(out)), "lmg_table_kernel")
        return out

    def correction(self, N: int) -> np.ndarray:
        out = np.zeros(N)
        _check(self._lib.lmg_correction(self._h, N, _dptr(out)), "lmg_correction")
        return out

    def map_error(self, x):
        x = np.ascontiguousarray(np.atleast_1d(x), dtype=np.float64)
        a = np.zeros(len(x))
        b = np.zeros(len(x))
        _check(self._lib.lmg_map_error(self._h, len(x), _dptr(x), _dptr(a), _dptr(b)), "lmg_map_error")
        return a, b

    @property
    def handle(self):
        return self._h

    def __del__(self):
        try:
            if self._h:
                self._lib.lmg_table_destroy(self._h)
                self._h = None
        except Exception:
            pass


# ---------------------------------------------------------------- torch glue
def _torch():
    import torch
    return torch


def _stream_handle(stream):
    torch = _torch()
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


def _prec_of(dtype, kahan: bool) -> int:
    torch = _torch()
    if dtype == torch.complex128:
        return F64
    if dtype == torch.complex64:
        return F32_KAHAN if kahan else F32
    raise TypeError(f"visibilities must be complex64 or complex128, got {dtype}")


def _cdtype(prec: int):
    torch = _torch()
    return torch.complex128 if prec == F64 else torch.complex64


def _ptr(t) -> ctypes.c_void_p:
    return ctypes.c_void_p(t.data_ptr()) if t is not None else ctypes.c_void_p(0)


def _check_tensor(t, name, dtype=None, shape=None, device=None, on_device=True):
    """Type, dtype, shape and layout first, then (unless on_device is False) that the tensor is on the device."""
    torch = _torch()
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch tensor")
    if dtype is not None and t.dtype != dtype:
        raise TypeError(f"{name} must have dtype {dtype}, got {t.dtype}")
    if shape is not None and tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} must have shape {tuple(shape)}, got {tuple(t.shape)}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if not on_device:
        return
    if not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA (HIP) tensor")
    if device is not None and t.device != device:
        raise ValueError(f"{name} is on {t.device}, expected {device}")


def _check_uv(uv):
    """uv: float64 (nvis, 2), contiguous, on a device; returns nvis."""
    torch = _torch()
    if not isinstance(uv, torch.Tensor):
        raise TypeError("uv must be a torch tensor")
    if uv.dim() != 2 or uv.shape[1] != 2:
        raise ValueError(f"uv must be (nvis, 2), got {tuple(uv.shape)}")
    _check_tensor(uv, "uv", torch.float64, on_device=False)
    return int(uv.shape[0])


def _check_vis_weights(vis, weights, nvis):
    torch = _torch()
    if not isinstance(vis, torch.Tensor) or vis.dtype not in (torch.complex64, torch.complex128):
        raise TypeError("visibilities must be a complex64 or complex128 tensor")
    _check_tensor(vis, "vis", vis.dtype, (nvis,), on_device=False)
    if weights is not None:
        _check_tensor(weights, "weights", torch.float32, (nvis,), on_device=False)


def _on_one_device(**tensors):
    """Every given tensor (None skipped) is a device tensor, all on the same device."""
    dev = None
    for name, t in tensors.items():
        if t is None:
            continue
        if not t.is_cuda:
            raise TypeError(f"{name} must be a CUDA (HIP) tensor")
        if dev is None:
            dev = t.device
        elif t.device != dev:
            raise ValueError(f"{name} is on {t.device}, expected {dev}")


def _bytes(n: int, device):
    torch = _torch()
    return torch.empty(max(int(n), 1), dtype=torch.uint8, device=device)


class Plan:
    """Per-uv-set state (tap cells, offsets, tile sort, work lists) in a torch-owned workspace."""

    def __init__(self, table: Table, N: int, uv, precision: int = F32, stream=None):
        torch = _torch()
        _check_tensor(uv, "uv", torch.float64)
        if uv.dim() != 2 or uv.shape[1] != 2:
            raise ValueError("uv must be (nvis, 2)")
        self.lib = load()
        self.table, self.N, self.precision = table, int(N), int(precision)
        self.nvis = int(uv.shape[0])
        self.device = uv.device
        self.M = int(round(2 * table.x0 * N))
        nb = ctypes.c_size_t()
        _check(self.lib.lmg_plan_workspace_size(self.N, table.W, self.nvis, self.precision, ctypes.byref(nb)),
               "lmg_plan_workspace_size")
        self.workspace = _bytes(nb.value, uv.device)
        self.uv = uv
        h = ctypes.c_void_p()
        with torch.cuda.device(uv.device):
            _check(self.lib.lmg_plan_create(table.handle, self.N, self.precision, self.nvis, _ptr(uv),
                                            _ptr(self.workspace), nb.value, _stream_handle(stream), ctypes.byref(h)),
                   "lmg_plan_create")
        self._h = h
        self._scratch = {}
        self.nchan = 1

    @property
    def grid_shape(self):
        return (self.N, self.N) if self.nchan == 1 else (self.nchan, self.N, self.N)

    @property
    def handle(self):
        return self._h

    def info(self):
        t, ni, nb, nv = ctypes.c_int(), ctypes.c_int(), ctypes.c_int(), ctypes.c_int64()
        _check(self.lib.lmg_plan_info(self._h, ctypes.byref(t), ctypes.byref(ni), ctypes.byref(nb), ctypes.byref(nv)),
               "lmg_plan_info")
        return {"tile": t.value, "items": ni.value, "busy_tiles": nb.value, "valid": nv.value}

    def check(self) -> int:
        return self.lib.lmg_plan_check(self._h)

    def scratch(self, op: int):
        if op not in self._scratch:
            n = ctypes.c_size_t()
            _check(self.lib.lmg_plan_scratch_size(self._h, op, ctypes.byref(n)), "lmg_plan_scratch_size")
            self._scratch[op] = _bytes(n.value, self.device)
        return self._scratch[op]

    def _vis_dtype(self):
        return _cdtype(self.precision)

    def grid(self, vis, weights=None, out=None, accumulate: bool = False, stream=None):
        """Gridding (lmg_grid_planned): a new grid, ``out`` overwritten, or ``out += G`` with ``accumulate``."""
        torch = _torch()
        _check_tensor(vis, "vis", self._vis_dtype(), (self.nvis,), self.device)
        if weights is not None:
            _check_tensor(weights, "weights", torch.float32, (self.nvis,), self.device)
        if out is None:
            if accumulate:
                raise ValueError("accumulate needs an output grid")
            out = torch.empty(self.grid_shape, dtype=self._vis_dtype(), device=self.device)
        _check_tensor(out, "grid", self._vis_dtype(), self.grid_shape, self.device)
        sc = self.scratch(OP_GRID)
        _check(self.lib.lmg_grid_planned(self._h, _ptr(vis), _ptr(weights), _ptr(out), 1 if accumulate else 0,
                                         _ptr(sc), sc.numel(), _stream_handle(stream)), "lmg_grid_planned")
        return out

    def grid_noalloc(self, vis, weights=None, out=None, accumulate: bool = False, stream=None):
        """Gridding with no device allocation by the library (lmg_grid_planned_noalloc): the scratch is the
        library's fixed per-device array; calls overlapping on one device race. ``out`` must be given when
        accumulating; otherwise a grid is allocated here (by torch) if it is missing."""
        torch = _torch()
        _check_tensor(vis, "vis", self._vis_dtype(), (self.nvis,), self.device)
        if weights is not None:
            _check_tensor(weights, "weights", torch.float32, (self.nvis,), self.device)
        if out is None:
            if accumulate:
                raise ValueError("accumulate needs an output grid")
            out = torch.empty(self.grid_shape, dtype=self._vis_dtype(), device=self.device)
        _check_tensor(out, "grid", self._vis_dtype(), self.grid_shape, self.device)
        _check(self.lib.lmg_grid_planned_noalloc(self._h, _ptr(vis), _ptr(weights), _ptr(out), 1 if accumulate else 0,
                                                 _stream_handle(stream)), "lmg_grid_planned_noalloc")
        return out

    def degrid(self, grid, out=None, stream=None):
        torch = _torch()
        _check_tensor(grid, "grid", self._vis_dtype(), self.grid_shape, self.device)
        if out is None:
            out = torch.empty(self.nvis, dtype=self._vis_dtype(), device=self.device)
        _check_tensor(out, "vis_out", self._vis_dtype(), (self.nvis,), self.device)
        sc = self.scratch(OP_DEGRID)
        _check(self.lib.lmg_degrid_planned(self._h, _ptr(grid), _ptr(out), _ptr(sc), sc.numel(),
                                           _stream_handle(stream)), "lmg_degrid_planned")
        return out

    # ---- plan order: keep visibility data in the plan's own order across calls (no reordering per call)
    def plan_order_length(self) -> int:
        n = ctypes.c_int64()
        _check(self.lib.lmg_plan_order_length(self._h, ctypes.byref(n)), "lmg_plan_order_length")
        return n.value

    def to_plan_order(self, vis, weights=None, out=None, stream=None):
        """w V in plan order (lmg_to_plan_order): a tensor of plan_order_length() elements."""
        torch = _torch()
        _check_tensor(vis, "vis", self._vis_dtype(), (self.nvis,), self.device)
        if weights is not None:
            _check_tensor(weights, "weights", torch.float32, (self.nvis,), self.device)
        n = self.plan_order_length()
        if out is None:
            out = torch.zeros(n, dtype=self._vis_dtype(), device=self.device)
        _check_tensor(out, "vis_plan", self._vis_dtype(), (n,), self.device)
        _check(self.lib.lmg_to_plan_order(self._h, _ptr(vis), _ptr(weights), _ptr(out), _stream_handle(stream)),
               "lmg_to_plan_order")
        return out

    def from_plan_order(self, vis_plan, out=None, stream=None):
        """Caller-order copy of plan-ordered visibilities (lmg_from_plan_order)."""
        torch = _torch()
        _check_tensor(vis_plan, "vis_plan", self._vis_dtype(), (self.plan_order_length(),), self.device)
        if out is None:
            out = torch.empty(self.nvis, dtype=self._vis_dtype(), device=self.device)
        _check_tensor(out, "vis", self._vis_dtype(), (self.nvis,), self.device)
        _check(self.lib.lmg_from_plan_order(self._h, _ptr(vis_plan), _ptr(out), _stream_handle(stream)),
               "lmg_from_plan_order")
        return out

    def grid_ordered(self, vis_plan, out=None, accumulate: bool = False, stream=None):
        """Gridding of plan-ordered visibilities (lmg_grid_planned_ordered)."""
        torch = _torch()
        _check_tensor(vis_plan, "vis_plan", self._vis_dtype(), (self.plan_order_length(),), self.device)
        if out is None:
            if accumulate:
                raise ValueError("accumulate needs an output grid")
            out = torch.empty(self.grid_shape, dtype=self._vis_dtype(), device=self.device)
        _check_tensor(out, "grid", self._vis_dtype(), self.grid_shape, self.device)
        sc = self.scratch(OP_GRID)
        _check(self.lib.lmg_grid_planned_ordered(self._h, _ptr(vis_plan), _ptr(out), 1 if accumulate else 0,
                                                 _ptr(sc), sc.numel(), _stream_handle(stream)),
               "lmg_grid_planned_ordered")
        return out

    def degrid_ordered(self, grid, out=None, stream=None):
        """Degridding into plan order (lmg_degrid_planned_ordered)."""
        torch = _torch()
        _check_tensor(grid, "grid", self._vis_dtype(), self.grid_shape, self.device)
        n = self.plan_order_length()
        if out is None:
            out = torch.zeros(n, dtype=self._vis_dtype(), device=self.device)
        _check_tensor(out, "vis_plan", self._vis_dtype(), (n,), self.device)
        sc = self.scratch(OP_DEGRID)
        _check(self.lib.lmg_degrid_planned_ordered(self._h, _ptr(grid), _ptr(out), _ptr(sc), sc.numel(),
                                                   _stream_handle(stream)), "lmg_degrid_planned_ordered")
        return out

    def make_dirty_image(self, vis, weights=None, out=None, stream=None):
        torch = _torch()
        _check_tensor(vis, "vis", self._vis_dtype(), (self.nvis,), self.device)
        if weights is not None:
            _check_tensor(weights, "weights", torch.float32, (self.nvis,), self.device)
        if out is None:
            out = torch.empty((self.M, self.M), dtype=self._vis_dtype(), device=self.device)
        _check_tensor(out, "image", self._vis_dtype(), (self.M, self.M), self.device)
        sc = self.scratch(OP_DIRTY)
        _check(self.lib.lmg_make_dirty_image_planned(self._h, _ptr(vis), _ptr(weights), _ptr(out), _ptr(sc),
                                                     sc.numel(), _stream_handle(stream)),
               "lmg_make_dirty_image_planned")
        return out

    def predict_visibilities(self, image, out=None, stream=None):
        torch = _torch()
        _check_tensor(image, "image", self._vis_dtype(), (self.M, self.M), self.device)
        if out is None:
            out = torch.empty(self.nvis, dtype=self._vis_dtype(), device=self.device)
        _check_tensor(out, "vis_out", self._vis_dtype(), (self.nvis,), self.device)
        sc = self.scratch(OP_PREDICT)
        _check(self.lib.lmg_predict_visibilities_planned(self._h, _ptr(image), _ptr(out), _ptr(sc), sc.numel(),
                                                         _stream_handle(stream)),
               "lmg_predict_visibilities_planned")
        return out

    def __del__(self):
        try:
            if self._h:
                self.lib.lmg_plan_destroy(self._h)
                self._h = None
        except Exception:
            pass


# ------------------------------------------------------------ batched channels
def _offsets_array(offsets) -> np.ndarray:
    off = np.ascontiguousarray(np.asarray(offsets, dtype=np.int64))
    if off.ndim != 1 or len(off) < 2:
        raise ValueError("offsets must be a 1-D sequence of nchan + 1 integers")
    return off


class BatchPlan(Plan):
    """Plan over nchan channels: channel c owns visibilities offsets[c]:offsets[c+1] and grid c.

    ``grid`` returns (nchan, N, N) grids and ``degrid`` takes them. ``tile`` = 0
    picks the library default; :func:`autotune_batch` measures the candidates.
    """

    def __init__(self, table: Table, N: int, uv, offsets, precision: int = F32, tile: int = 0, stream=None):
        torch = _torch()
        _check_tensor(uv, "uv", torch.float64)
        if uv.dim() != 2 or uv.shape[1] != 2:
            raise ValueError("uv must be (nvis, 2)")
        off = _offsets_array(offsets)
        if off[-1] != uv.shape[0]:
            raise ValueError(f"offsets end at {off[-1]} but uv holds {uv.shape[0]} visibilities")
        self.lib = load()
        self.table, self.N, self.precision = table, int(N), int(precision)
        self.nvis = int(uv.shape[0])
        self.device = uv.device
        self.M = int(round(2 * table.x0 * N))
        self.offsets = off
        nb = ctypes.c_size_t()
        _check(self.lib.lmg_batch_workspace_size(self.N, table.W, len(off) - 1, self.nvis, self.precision,
                                                 ctypes.byref(nb)), "lmg_batch_workspace_size")
        self.workspace = _bytes(nb.value, uv.device)
        self.uv = uv
        h = ctypes.c_void_p()
        with torch.cuda.device(uv.device):
            _check(self.lib.lmg_batch_plan_create(table.handle, self.N, self.precision, len(off) - 1,
                                                  off.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), _ptr(uv),
                                                  int(tile), _ptr(self.workspace), nb.value, _stream_handle(stream),
                                                  ctypes.byref(h)), "lmg_batch_plan_create")
        self._h = h
        self._scratch = {}
        self.nchan = len(off) - 1

    def info(self):
        d = super().info()
        nc, t, w = ctypes.c_int(), ctypes.c_int(), ctypes.c_int()
        _check(self.lib.lmg_batch_info(self._h, ctypes.byref(nc), ctypes.byref(t), ctypes.byref(w)), "lmg_batch_info")
        d.update(channels=nc.value, waves=w.value)
        return d


_TUNED = {}


def autotune_batch(table: Table, N: int, uv, offsets, vis, weights=None, precision: int = F32,
                   tiles=(16, 32, 64), reps: int = 3, stream=None):
    """Pick the uv tile edge of a batched plan by timing gridding + degridding on the caller's data.

    Each candidate tile (skipped where the library rejects it as invalid or
    unsupported; any other failure propagates) gets a plan, one
    untimed grid + degrid, then ``reps`` timed ones (HIP events on the launch
    stream). The fastest plan is returned with the timings {tile: ms}; the
    choice is remembered for the same (N, W, precision, channels, visibilities).
    """
    torch = _torch()
    off = _offsets_array(offsets)
    key = (int(N), table.W, int(precision), len(off) - 1, int(uv.shape[0]))
    if key in _TUNED:
        return BatchPlan(table, N, uv, off, precision, _TUNED[key][0], stream), _TUNED[key][1]
    s = torch.cuda.current_stream() if stream is None else stream
    best, timings = None, {}
    for T in tiles:
        if T > N or N // T > 128:
            continue
        try:
            plan = BatchPlan(table, N, uv, off, precision, T, stream)
        except LmgError as e:
            if e.status not in (-1, -5):            # only LMG_EINVAL / LMG_ENOTSUP mean "tile not usable"
                raise
            continue
        g = plan.grid(vis, weights, stream=s)
        v = plan.degrid(g, stream=s)
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(s)
        for _ in range(reps):
            plan.grid(vis, weights, out=g, stream=s)
            plan.degrid(g, out=v, stream=s)
        e1.record(s)
        e1.synchronize()
        timings[T] = e0.elapsed_time(e1) / reps
        if best is None or timings[T] < timings[best[0]]:
            best = (T, plan)
        del g, v
    if best is None:
        raise LmgError(-1, "autotune_batch: no tile edge is valid for this problem")
    _TUNED[key] = (best[0], timings)
    return best[1], timings


def _check_offsets(off, nvis):
    if off[0] != 0 or np.any(np.diff(off) < 0) or off[-1] != nvis:
        raise ValueError(f"offsets must start at 0, not decrease and end at nvis = {nvis}")


def grid_batched(table: Table, N: int, uv, offsets, vis, weights=None, kahan: bool = False, out=None,
                 stream=None):
    """One-shot batched gridding (plan built and released inside). lmg_grid_batched accumulates: into ``out``
    (nchan, N, N) if given, else into new zeroed grids, which are returned."""
    torch = _torch()
    nvis = _check_uv(uv)
    _check_vis_weights(vis, weights, nvis)
    prec = _prec_of(vis.dtype, kahan)
    off = _offsets_array(offsets)
    _check_offsets(off, nvis)
    nchan = len(off) - 1
    if out is not None:
        _check_tensor(out, "grids", vis.dtype, (nchan, N, N), on_device=False)
    _on_one_device(uv=uv, vis=vis, weights=weights, grids=out)
    lib = load()
    nb = ctypes.c_size_t()
    _check(lib.lmg_workspace_size_batched(int(N), table.W, nchan, int(off[-1]), prec, OP_GRID, ctypes.byref(nb)),
           "lmg_workspace_size_batched")
    ws = _bytes(nb.value, vis.device)
    if out is None:
        out = torch.zeros((nchan, N, N), dtype=vis.dtype, device=vis.device)
    _check(lib.lmg_grid_batched(table.handle, int(N), prec, nchan, off.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                                _ptr(uv), _ptr(vis), _ptr(weights), _ptr(out), _ptr(ws), nb.value,
                                _stream_handle(stream)), "lmg_grid_batched")
    return out


def degrid_batched(table: Table, N: int, uv, offsets, grids, stream=None):
    """One-shot batched degridding of (nchan, N, N) grids."""
    torch = _torch()
    nvis = _check_uv(uv)
    if not isinstance(grids, torch.Tensor) or grids.dtype not in (torch.complex64, torch.complex128):
        raise TypeError("grids must be a complex64 or complex128 tensor")
    off = _offsets_array(offsets)
    _check_offsets(off, nvis)
    nchan = len(off) - 1
    _check_tensor(grids, "grids", grids.dtype, (nchan, N, N), on_device=False)
    _on_one_device(uv=uv, grids=grids)
    prec = _prec_of(grids.dtype, False)
    lib = load()
    nb = ctypes.c_size_t()
    _check(lib.lmg_workspace_size_batched(int(N), table.W, nchan, int(off[-1]), prec, OP_DEGRID, ctypes.byref(nb)),
           "lmg_workspace_size_batched")
    ws = _bytes(nb.value, grids.device)
    out = torch.empty(int(off[-1]), dtype=grids.dtype, device=grids.device)
    _check(lib.lmg_degrid_batched(table.handle, int(N), prec, nchan, off.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                                  _ptr(uv), _ptr(grids), _ptr(out), _ptr(ws), nb.value, _stream_handle(stream)),
           "lmg_degrid_batched")
    return out


# ------------------------------------------------------------ autograd
# Gridding and degridding are transposes of each other (C is real), and so
# are the dirty image and the prediction (the correction is a real diagonal,
# the crop is the transpose of the zero pad, and the +i2pi transform is the
# adjoint of the -i2pi one). Each backward is therefore the other call of the
# same plan. Gradients follow torch's convention for complex tensors
# (dL/dRe + i dL/dIm). Where weights are involved, the chain rule's product
# with w, and the weight gradient Re(conj(V) * A^T g), are torch elementwise
# ops on the backward's output.


def _autograd_function():
    torch = _torch()

    class _Degrid(torch.autograd.Function):
        @staticmethod
        def forward(ctx, plan, grid_):
            ctx.plan = plan
            return plan.degrid(grid_.contiguous())

        @staticmethod
        def backward(ctx, g):
            return None, ctx.plan.grid(g.contiguous(), None)

    class _Grid(torch.autograd.Function):
        @staticmethod
        def forward(ctx, plan, vis, weights):
            ctx.plan = plan
            ctx.save_for_backward(vis, weights)
            return plan.grid(vis.contiguous(), None if weights is None else weights.contiguous())

        @staticmethod
        def backward(ctx, g):
            vis, weights = ctx.saved_tensors
            d = ctx.plan.degrid(g.contiguous())
            gv = d if weights is None else d * weights
            gw = None
            if weights is not None and ctx.needs_input_grad[2]:
                gw = (vis.conj() * d).real.to(weights.dtype)
            return None, (gv if ctx.needs_input_grad[1] else None), gw

    class _Predict(torch.autograd.Function):
        @staticmethod
        def forward(ctx, plan, image):
            ctx.plan = plan
            return plan.predict_visibilities(image.contiguous())

        @staticmethod
        def backward(ctx, g):
            return None, ctx.plan.make_dirty_image(g.contiguous(), None)

    class _Dirty(torch.autograd.Function):
        @staticmethod
        def forward(ctx, plan, vis, weights):
            ctx.plan = plan
            ctx.save_for_backward(vis, weights)
            return plan.make_dirty_image(vis.contiguous(), None if weights is None else weights.contiguous())

        @staticmethod
        def backward(ctx, g):
            vis, weights = ctx.saved_tensors
            d = ctx.plan.predict_visibilities(g.contiguous())
            gv = d if weights is None else d * weights
            gw = None
            if weights is not None and ctx.needs_input_grad[2]:
                gw = (vis.conj() * d).real.to(weights.dtype)
            return None, (gv if ctx.needs_input_grad[1] else None), gw

    return _Degrid, _Grid, _Predict, _Dirty


_AUTOGRAD = None


def _fns():
    global _AUTOGRAD
    if _AUTOGRAD is None:
        _AUTOGRAD = _autograd_function()
    return _AUTOGRAD


class Degrid:
    """Differentiable degridding: ``Degrid.apply(plan, grid) -> vis``; backward = gridding of the gradient."""

    @staticmethod
    def apply(plan: "Plan", grid_):
        return _fns()[0].apply(plan, grid_)


class Grid:
    """Differentiable gridding: ``Grid.apply(plan, vis, weights=None) -> grid``; backward = weighted degridding."""

    @staticmethod
    def apply(plan: "Plan", vis, weights=None):
        return _fns()[1].apply(plan, vis, weights)


class PredictVisibilities:
    """Differentiable prediction: ``PredictVisibilities.apply(plan, image) -> vis``; backward = dirty image."""

    @staticmethod
    def apply(plan: "Plan", image):
        return _fns()[2].apply(plan, image)


class MakeDirtyImage:
    """Differentiable dirty image: ``MakeDirtyImage.apply(plan, vis, weights=None)``; backward = prediction."""

    @staticmethod
    def apply(plan: "Plan", vis, weights=None):
        return _fns()[3].apply(plan, vis, weights)


# ------------------------------------------------------------ one-shot calls
def _oneshot_ws(table, N, nvis, prec, op, device):
    n = ctypes.c_size_t()
    _check(load().lmg_workspace_size(N, table.W, table.x0, nvis, prec, op, ctypes.byref(n)), "lmg_workspace_size")
    return _bytes(n.value, device), n.value


def grid(table: Table, N: int, uv, vis, weights=None, kahan: bool = False, out=None, stream=None):
    """One-shot gridding (builds a plan internally). lmg_grid accumulates: into ``out`` if given, else into a
    new zeroed N x N grid, which is returned."""
    torch = _torch()
    nvis = _check_uv(uv)
    _check_vis_weights(vis, weights, nvis)
    prec = _prec_of(vis.dtype, kahan)
    if out is not None:
        _check_tensor(out, "grid", vis.dtype, (N, N), on_device=False)
    _on_one_device(uv=uv, vis=vis, weights=weights, grid=out)
    if out is None:
        out = torch.zeros((N, N), dtype=vis.dtype, device=vis.device)
    ws, nb = _oneshot_ws(table, N, nvis, prec, OP_GRID, vis.device)
    _check(load().lmg_grid(table.handle, N, prec, nvis, _ptr(uv), _ptr(vis), _ptr(weights), _ptr(out),
                           _ptr(ws), nb, _stream_handle(stream)), "lmg_grid")
    return out


def degrid(table: Table, N: int, uv, grid_, stream=None):
    """One-shot degridding of an N x N grid at the uv coordinates."""
    torch = _torch()
    nvis = _check_uv(uv)
    if not isinstance(grid_, torch.Tensor) or grid_.dtype not in (torch.complex64, torch.complex128):
        raise TypeError("grid must be a complex64 or complex128 tensor")
    _check_tensor(grid_, "grid", grid_.dtype, (N, N), on_device=False)
    _on_one_device(uv=uv, grid=grid_)
    prec = _prec_of(grid_.dtype, False)
    out = torch.empty(nvis, dtype=grid_.dtype, device=grid_.device)
    ws, nb = _oneshot_ws(table, N, nvis, prec, OP_DEGRID, grid_.device)
    _check(load().lmg_degrid(table.handle, N, prec, nvis, _ptr(uv), _ptr(grid_), _ptr(out), _ptr(ws), nb,
                             _stream_handle(stream)), "lmg_degrid")
    return out


def make_dirty_image(table: Table, N: int, uv, vis, weights=None, kahan: bool = False, stream=None):
    """One-shot dirty image (grid, inverse FFT, correct, crop)."""
    torch = _torch()
    nvis = _check_uv(uv)
    _check_vis_weights(vis, weights, nvis)
    _on_one_device(uv=uv, vis=vis, weights=weights)
    prec = _prec_of(vis.dtype, kahan)
    M = int(round(2 * table.x0 * N))
    out = torch.empty((M, M), dtype=vis.dtype, device=vis.device)
    ws, nb = _oneshot_ws(table, N, nvis, prec, OP_DIRTY, vis.device)
    _check(load().lmg_make_dirty_image(table.handle, N, prec, nvis, _ptr(uv), _ptr(vis), _ptr(weights),
                                       _ptr(out), _ptr(ws), nb, _stream_handle(stream)), "lmg_make_dirty_image")
    return out


def predict_visibilities(table: Table, N: int, uv, image, stream=None):
    """One-shot prediction (correct, pad, forward FFT, degrid) of an M x M image, M = 2 x0 N."""
    torch = _torch()
    nvis = _check_uv(uv)
    M = int(round(2 * table.x0 * N))
    if not isinstance(image, torch.Tensor) or image.dtype not in (torch.complex64, torch.complex128):
        raise TypeError("image must be a complex64 or complex128 tensor")
    _check_tensor(image, "image", image.dtype, (M, M), on_device=False)
    _on_one_device(uv=uv, image=image)
    prec = _prec_of(image.dtype, False)
    out = torch.empty(nvis, dtype=image.dtype, device=image.device)
    ws, nb = _oneshot_ws(table, N, nvis, prec, OP_PREDICT, image.device)
    _check(load().lmg_predict_visibilities(table.handle, N, prec, nvis, _ptr(uv), _ptr(image), _ptr(out), _ptr(ws),
                                           nb, _stream_handle(stream)), "lmg_predict_visibilities")
    return out


def sync_status(stream=None) -> int:
    """lmg_sync_status: wait for the stream, then 0 (LMG_OK) or -4 (LMG_EDATA: non-finite coordinates were met
    by a plan on this device since the last call; the flag is cleared)."""
    s = load().lmg_sync_status(_stream_handle(stream))
    if s not in (0, -4):
        raise LmgError(s, "lmg_sync_status")
    return s


def trace_enable(on: bool = True):
    """Bracket every library kernel launch with HIP events (per-kernel timing)."""
    _check(load().lmg_trace_enable(1 if on else 0), "lmg_trace_enable")


def trace_only(name: Optional[str] = None):
    """Record only the named kernel (None: all kernels again)."""
    _check(load().lmg_trace_only(None if name is None else name.encode()), "lmg_trace_only")


def trace_report() -> dict:
    """{kernel name: (launches, total ms)} since the last report; synchronizes the recorded events."""
    buf = ctypes.create_string_buffer(1 << 16)
    _check(load().lmg_trace_report(buf, len(buf)), "lmg_trace_report")
    out = {}
    for line in buf.value.decode().splitlines():
        name, n, ms = line.split()
        out[name] = (int(n), float(ms))
    return out


def fft2_centred(data, sign: int, stream=None):
    """In-place centred 2D FFT of an N x N complex tensor (exponent sign * i 2 pi)."""
    torch = _torch()
    if not isinstance(data, torch.Tensor) or data.dim() != 2 or data.shape[0] != data.shape[1]:
        raise ValueError("data must be an N x N tensor")
    N = int(data.shape[0])
    if data.dtype not in (torch.complex64, torch.complex128):
        raise TypeError("data must be complex64 or complex128")
    _check_tensor(data, "data", data.dtype, (N, N))
    prec = _prec_of(data.dtype, False)
    cs = 16 if prec == F64 else 8
    scratch = _bytes(((N * N * cs + 255) // 256) * 256 + N * cs, data.device)
    _check(load().lmg_fft2_centred(N, prec, sign, _ptr(data), _ptr(scratch), _stream_handle(stream)),
           "lmg_fft2_centred")
    return data
