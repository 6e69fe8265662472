"""Thin ctypes binding of ``libdvl.so`` (the C ABI in ``include/dvl.h``).

Argument marshalling only: every step of the ordering and the update runs in
the HIP kernels behind the C ABI.  PyTorch provides device memory and the
current stream.  There is no CPU fallback: if the library is not built this
module raises on first use.
"""
from __future__ import annotations

import ctypes as C
import os
import re

import numpy as np
import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "_lib", "libdvl.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "dvl.h")

OK, E_INVALID, E_NOMEM, E_HIP, E_STATE, E_OVERLAP, E_RANGE = range(7)
F32, F16, BF16 = 0, 1, 2
VMAX_TF_RANGE, VMAX_TF_BOUND, VMAX_EXACT = 0, 1, 2
SCAN_FP64, SCAN_KAHAN_FP32, SCAN_NAIVE_FP32 = 0, 1, 2
ENTRY_CACHE_AUTO, ENTRY_CACHE_ALWAYS, ENTRY_CACHE_NEVER = 0, 1, 2

_DTYPE_CODE = {torch.float32: F32, torch.float16: F16, torch.bfloat16: BF16}
_CODE_DTYPE = {v: k for k, v in _DTYPE_CODE.items()}


class DvlError(RuntimeError):
    def __init__(self, status: int, where: str, message: str):
        super().__init__(f"{where}: status {status}: {message}")
        self.status = status


class dvl_params(C.Structure):
    _fields_ = [("n_bins", C.c_int32), ("exponent", C.c_float), ("min_importance", C.c_float),
                ("vmax_mode", C.c_int32), ("clamp_mode", C.c_int32), ("level_scale", C.c_int32),
                ("scan_mode", C.c_int32)]


class dvl_bins(C.Structure):
    _fields_ = [("first_cell", C.c_void_p), ("last_cell", C.c_void_p), ("mean", C.c_void_p),
                ("vmin", C.c_void_p), ("vmax", C.c_void_p), ("y", C.c_void_p),
                ("f_total", C.c_void_p), ("vmax_used", C.c_void_p)]


ALLOC_FN = C.CFUNCTYPE(C.c_void_p, C.c_void_p, C.c_size_t, C.c_void_p)
RELEASE_FN = C.CFUNCTYPE(None, C.c_void_p, C.c_void_p, C.c_void_p)


class dvl_allocator(C.Structure):
    _fields_ = [("alloc", ALLOC_FN), ("release", RELEASE_FN), ("ctx", C.c_void_p)]


class dvl_build_options(C.Structure):
    _fields_ = [("tile_steps", C.c_int32), ("run_waves", C.c_int32), ("entry_cache", C.c_int32),
                ("allocator", C.POINTER(dvl_allocator))]


class Allocator:
    """A ``dvl_allocator`` over two Python callables: ``alloc(nbytes, stream)``
    returning a device address (0 when it cannot) and ``release(ptr, stream)``.
    Keeps the ctypes callbacks alive; volumes and executors built with it hold
    a reference to it."""

    def __init__(self, alloc, release):
        def _alloc(ctx, nbytes, stream):
            try:
                return int(alloc(int(nbytes), int(stream or 0))) or None
            except Exception:
                return None

        def _release(ctx, ptr, stream):
            try:
                release(int(ptr), int(stream or 0))
            except Exception:
                pass

        self._cb = (ALLOC_FN(_alloc), RELEASE_FN(_release))
        self.struct = dvl_allocator(self._cb[0], self._cb[1], None)


def torch_allocator() -> Allocator:
    """The library's device memory from PyTorch's caching allocator (on the
    stream of the call that allocates; the current stream when it has none)."""
    def alloc(nbytes, stream):
        try:
            return torch.cuda.caching_allocator_alloc(nbytes, stream=stream or None)
        except torch.OutOfMemoryError:
            return 0

    def release(ptr, stream):
        torch.cuda.caching_allocator_delete(ptr)

    return Allocator(alloc, release)


class dvl_request(C.Structure):
    _fields_ = [("volume", C.c_void_p), ("alpha", C.c_void_p), ("n_tf", C.c_int32),
                ("lo", C.c_void_p), ("hi", C.c_void_p), ("params", dvl_params), ("out", dvl_bins)]


_lib = None


def declared_symbols(header: str = HEADER) -> list[str]:
    """Names of the functions ``include/dvl.h`` declares."""
    text = open(header).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(dvl_[a-z0-9_]+)\s*\(", text)))


def lib():
    """Load libdvl.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"HIP library missing: {LIB_PATH}; build it with "
                           "`python -m paper_2306_11612_amd.build` (there is no CPU fallback)")
    L = C.CDLL(LIB_PATH)
    vp, i32, i64, f32 = C.c_void_p, C.c_int32, C.c_int64, C.c_float
    sig = {
        "dvl_build_order": (i32, [i64, vp, vp, vp, vp, i32, i32, vp, vp, C.POINTER(vp)]),
        "dvl_build_order_ex": (i32, [i64, vp, vp, vp, vp, i32, i32, vp, C.POINTER(dvl_build_options), vp,
                                     C.POINTER(vp)]),
        "dvl_set_field": (i32, [vp, i32, vp, vp]),
        "dvl_field_range": (i32, [vp, i32, C.POINTER(f32), C.POINTER(f32)]),
        "dvl_set_tf": (i32, [vp, i32, vp, i32, f32, f32]),
        "dvl_update": (i32, [vp, C.POINTER(dvl_params), C.POINTER(dvl_bins), vp]),
        "dvl_update_noalloc": (i32, [vp, C.POINTER(dvl_params), C.POINTER(dvl_bins), vp]),
        "dvl_update_noalloc_max_bytes": (C.c_size_t, []),
        "dvl_set_carry_wait": (i32, [i32]),
        "dvl_read_bins": (i32, [vp, C.POINTER(dvl_bins), i32, vp] + [vp] * 9),
        "dvl_export_order": (i32, [vp, vp, vp, vp]),
        "dvl_export_sorted": (i32, [vp, vp, vp, vp]),
        "dvl_set_timing": (i32, [vp, i32]),
        "dvl_kernel_times": (i32, [vp, vp, C.POINTER(i32)]),
        "dvl_num_cells": (i64, [vp]),
        "dvl_num_fields": (i32, [vp]),
        "dvl_grid_bits": (i32, [vp]),
        "dvl_dtype": (i32, [vp]),
        "dvl_volume_bytes": (C.c_size_t, [vp]),
        "dvl_level_segments": (i32, [vp, vp, vp]),
        "dvl_update_workspace_bytes": (C.c_size_t, [i64, i32, i32]),
        "dvl_destroy": (None, [vp]),
        "dvl_set_entry_cache": (i32, [vp, i32]),
        "dvl_entry_cache_info": (i32, [vp, vp, vp, vp]),
        "dvl_executor_create": (i32, [C.POINTER(vp)]),
        "dvl_executor_create_ex": (i32, [C.POINTER(dvl_allocator), C.POINTER(vp)]),
        "dvl_executor_destroy": (None, [vp]),
        "dvl_executor_bytes": (C.c_size_t, [vp]),
        "dvl_request_bytes": (C.c_size_t, [vp, i32]),
        "dvl_executor_set_timing": (i32, [vp, i32]),
        "dvl_executor_kernel_times": (i32, [vp, vp, C.POINTER(i32)]),
        "dvl_update_batch": (i32, [vp, C.POINTER(dvl_request), i32, vp]),
        "dvl_graph_create": (i32, [C.POINTER(dvl_request), i32, C.POINTER(vp)]),
        "dvl_graph_set_tf": (i32, [vp, i32, vp, vp, vp]),
        "dvl_graph_launch": (i32, [vp, vp]),
        "dvl_graph_set_tf_all": (i32, [vp, vp, vp, vp]),
        "dvl_graph_destroy": (None, [vp]),
        "dvl_last_error": (C.c_char_p, []),
        "dvl_select_bins": (i32, [vp, C.POINTER(dvl_bins), i32, i32, i32, vp, vp, vp, vp, vp]),
        "dvl_select_mask": (i32, [vp, vp, i32, vp, vp]),
        "dvl_bin_histograms": (i32, [vp, C.POINTER(dvl_bins), i32, i32, i32, f32, f32, vp, vp]),
        "dvl_rasterize": (i32, [vp, i32, i32, i32, i32, vp, vp]),
        "dvl_zoom": (i32, [vp, C.c_uint32, C.c_uint32, C.POINTER(dvl_build_options), vp, C.POINTER(vp)]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(L, name)
        fn.restype = res
        fn.argtypes = args
    _lib = L
    return L


def _check(status: int, where: str):
    if status != OK:
        raise DvlError(status, where, lib().dvl_last_error().decode(errors="replace"))


def _stream_ptr(stream):
    if stream is None:
        stream = torch.cuda.current_stream()
    return C.c_void_p(stream.cuda_stream)


def _ptr(t: torch.Tensor):
    return C.c_void_p(t.data_ptr())


def _dev(t: torch.Tensor, dtype=None) -> torch.Tensor:
    if not t.is_cuda:
        raise ValueError("expected a device tensor")
    if dtype is not None and t.dtype != dtype:
        raise ValueError(f"expected {dtype}, got {t.dtype}")
    return t.contiguous()


class Bins:
    """Caller-owned device outputs of one update (``dvl_bins``)."""

    def __init__(self, n_bins: int, n_fields: int, device=None):
        device = device or torch.device("cuda", torch.cuda.current_device())
        self.n_bins, self.n_fields = int(n_bins), int(n_fields)
        W, M = self.n_bins, self.n_fields
        self.first_cell = torch.empty(W, dtype=torch.int32, device=device)
        self.last_cell = torch.empty(W, dtype=torch.int32, device=device)
        self.mean = torch.empty(M, W, dtype=torch.float32, device=device)
        self.vmin = torch.empty(M, W, dtype=torch.float32, device=device)
        self.vmax = torch.empty(M, W, dtype=torch.float32, device=device)
        self.y = torch.empty(M, W, dtype=torch.float32, device=device)
        self.f_total = torch.empty(1, dtype=torch.float64, device=device)
        self.vmax_used = torch.empty(1, dtype=torch.float32, device=device)

    def struct(self) -> dvl_bins:
        return dvl_bins(self.first_cell.data_ptr(), self.last_cell.data_ptr(), self.mean.data_ptr(),
                        self.vmin.data_ptr(), self.vmax.data_ptr(), self.y.data_ptr(),
                        self.f_total.data_ptr(), self.vmax_used.data_ptr())


def params(n_bins: int, exponent: float = 1.0, min_importance: float = 0.025,
           vmax_mode: int = VMAX_TF_RANGE, clamp_mode: int = 0, level_scale: int = 1,
           scan_mode: int = SCAN_FP64) -> dvl_params:
    return dvl_params(int(n_bins), float(exponent), float(min_importance), int(vmax_mode),
                      int(clamp_mode), int(level_scale), int(scan_mode))


# ---------------------------------------------------------------- C-ABI mirrors

def build_order(x, y, z, level, fields, stream=None, tile_steps: int = 0, run_waves: int = 0,
                entry_cache: int = ENTRY_CACHE_AUTO, allocator: Allocator | None = None) -> "Volume":
    """dvl_build_order (dvl_build_order_ex when an option is given): one-time
    Hilbert ordering of the cells.  ``allocator``: where the volume's device
    memory comes from (``torch_allocator()`` for PyTorch's caching allocator;
    None: the library's hipMalloc)."""
    x, y, z = _dev(x, torch.int32), _dev(y, torch.int32), _dev(z, torch.int32)
    level = _dev(level, torch.uint8)
    fields = [_dev(f) for f in fields]
    if not fields:
        raise ValueError("need at least one field")
    dt = fields[0].dtype
    if dt not in _DTYPE_CODE or any(f.dtype != dt for f in fields):
        raise ValueError("fields must share one of float32 / float16 / bfloat16")
    arr = (C.c_void_p * len(fields))(*[f.data_ptr() for f in fields])
    out = C.c_void_p()
    if tile_steps or run_waves or entry_cache != ENTRY_CACHE_AUTO or allocator is not None:
        opt = dvl_build_options(int(tile_steps), int(run_waves), int(entry_cache),
                                C.pointer(allocator.struct) if allocator is not None else None)
        st = lib().dvl_build_order_ex(x.numel(), _ptr(x), _ptr(y), _ptr(z), _ptr(level), len(fields),
                                      _DTYPE_CODE[dt], C.cast(arr, C.c_void_p), C.byref(opt),
                                      _stream_ptr(stream), C.byref(out))
        _check(st, "dvl_build_order_ex")
    else:
        st = lib().dvl_build_order(x.numel(), _ptr(x), _ptr(y), _ptr(z), _ptr(level), len(fields),
                                   _DTYPE_CODE[dt], C.cast(arr, C.c_void_p), _stream_ptr(stream),
                                   C.byref(out))
        _check(st, "dvl_build_order")
    return Volume(out, allocator)


def set_tf(vol: "Volume", m: int, alpha, lo: float, hi: float):
    """dvl_set_tf: alpha TF of field m with normalisation window [lo, hi]."""
    a = np.ascontiguousarray(np.asarray(alpha, dtype=np.float32))
    _check(lib().dvl_set_tf(vol.handle, int(m), a.ctypes.data_as(C.c_void_p), a.size,
                            float(lo), float(hi)), "dvl_set_tf")


def update(vol: "Volume", p: dvl_params, bins: Bins, stream=None):
    """dvl_update: enqueue one update on the stream."""
    b = bins.struct()
    _check(lib().dvl_update(vol.handle, C.byref(p), C.byref(b), _stream_ptr(stream)), "dvl_update")


def update_noalloc(vol: "Volume", p: dvl_params, bins: Bins, stream=None):
    """dvl_update_noalloc: the update through the library's fixed device
    scratch (no device allocation)."""
    b = bins.struct()
    _check(lib().dvl_update_noalloc(vol.handle, C.byref(p), C.byref(b), _stream_ptr(stream)),
           "dvl_update_noalloc")


def set_carry_wait(polls: int):
    """dvl_set_carry_wait: polls of a request's carry flag before a
    classifying workgroup computes the carry itself (test hook; 0 forces that
    path)."""
    _check(lib().dvl_set_carry_wait(int(polls)), "dvl_set_carry_wait")


CARRY_WAIT_DEFAULT = 1 << 15


def read_bins(vol: "Volume", bins: Bins, stream=None) -> dict:
    """dvl_read_bins: synchronise and copy the bins to host numpy arrays."""
    W, M = bins.n_bins, bins.n_fields
    count = np.empty(W, np.uint32); first = np.empty(W, np.uint32); last = np.empty(W, np.uint32)
    mean = np.empty((M, W), np.float32); vmin = np.empty((M, W), np.float32)
    vmax = np.empty((M, W), np.float32); y = np.empty((M, W), np.float32)
    ft = np.empty(1, np.float64); vu = np.empty(1, np.float32)
    b = bins.struct()
    P = lambda a: a.ctypes.data_as(C.c_void_p)
    _check(lib().dvl_read_bins(vol.handle, C.byref(b), W, _stream_ptr(stream), P(count), P(first),
                               P(last), P(mean), P(vmin), P(vmax), P(y), P(ft), P(vu)), "dvl_read_bins")
    return {"count": count, "first": first, "last": last, "mean": mean, "vmin": vmin, "vmax": vmax,
            "y": y, "f_total": float(ft[0]), "vmax_used": float(vu[0])}


class Volume:
    """A volume in Hilbert order, resident on the device (owns a dvl_volume*)."""

    def __init__(self, handle: C.c_void_p, allocator: Allocator | None = None):
        self.handle = handle
        self.allocator = allocator   # must outlive the handle

    # conveniences over the C-ABI mirrors
    build = staticmethod(build_order)

    @property
    def n(self) -> int:
        return int(lib().dvl_num_cells(self.handle))

    @property
    def m(self) -> int:
        return int(lib().dvl_num_fields(self.handle))

    @property
    def bits(self) -> int:
        return int(lib().dvl_grid_bits(self.handle))

    @property
    def dtype(self):
        return _CODE_DTYPE[int(lib().dvl_dtype(self.handle))]

    @property
    def nbytes(self) -> int:
        return int(lib().dvl_volume_bytes(self.handle))

    def level_segments(self):
        """(segments of 64 sorted cells, segments of mixed levels): dvl_level_segments."""
        ns, nm = C.c_int64(), C.c_int64()
        _check(lib().dvl_level_segments(self.handle, C.byref(ns), C.byref(nm)), "dvl_level_segments")
        return ns.value, nm.value

    def field_range(self, m: int):
        lo, hi = C.c_float(), C.c_float()
        _check(lib().dvl_field_range(self.handle, int(m), C.byref(lo), C.byref(hi)), "dvl_field_range")
        return lo.value, hi.value

    def set_field(self, m: int, values: torch.Tensor, stream=None):
        v = _dev(values, self.dtype)
        _check(lib().dvl_set_field(self.handle, int(m), _ptr(v), _stream_ptr(stream)), "dvl_set_field")

    def set_tf(self, m: int, alpha, lo: float | None = None, hi: float | None = None):
        if lo is None or hi is None:
            dlo, dhi = self.field_range(m)
            lo = dlo if lo is None else lo
            hi = dhi if hi is None else hi
            if not hi > lo:
                hi = np.nextafter(np.float32(lo), np.float32(np.inf))
        set_tf(self, m, alpha, lo, hi)

    def update(self, bins: Bins, stream=None, **kw):
        update(self, params(bins.n_bins, **kw), bins, stream)

    def read_bins(self, bins: Bins, stream=None) -> dict:
        return read_bins(self, bins, stream)

    def export_order(self, stream=None):
        """(keys uint64-as-int64 [n] in original order, perm int32 [n])."""
        n = self.n
        keys = torch.empty(n, dtype=torch.int64, device="cuda")
        perm = torch.empty(n, dtype=torch.int32, device="cuda")
        _check(lib().dvl_export_order(self.handle, _ptr(keys), _ptr(perm), _stream_ptr(stream)),
               "dvl_export_order")
        return keys, perm

    def export_sorted(self, stream=None):
        n, M = self.n, self.m
        level = torch.empty(n, dtype=torch.uint8, device="cuda")
        fields = [torch.empty(n, dtype=self.dtype, device="cuda") for _ in range(M)]
        arr = (C.c_void_p * M)(*[f.data_ptr() for f in fields])
        _check(lib().dvl_export_sorted(self.handle, _ptr(level), C.cast(arr, C.c_void_p),
                                       _stream_ptr(stream)), "dvl_export_sorted")
        return level, fields

    # -------------------------------------------------------- brushing, zoom, views

    def select_bins(self, bins: Bins, b0: int, b1: int, stream=None):
        """dvl_select_bins: (first, last, key_lo, key_hi) of the cells of bins b0..b1."""
        f, l = C.c_uint32(), C.c_uint32()
        klo, khi = C.c_uint64(), C.c_uint64()
        b = bins.struct()
        _check(lib().dvl_select_bins(self.handle, C.byref(b), bins.n_bins, int(b0), int(b1), _stream_ptr(stream),
                                     C.byref(f), C.byref(l), C.byref(klo), C.byref(khi)), "dvl_select_bins")
        return f.value, l.value, klo.value, khi.value

    def select_mask(self, ranges, stream=None) -> torch.Tensor:
        """dvl_select_mask: uint8 [n] (original order), 1 where the cell's key is
        in one of the closed ranges [(lo, hi), ...]."""
        r = np.ascontiguousarray(np.asarray(ranges, dtype=np.uint64).reshape(-1, 2))
        mask = torch.empty(self.n, dtype=torch.uint8, device="cuda")
        _check(lib().dvl_select_mask(self.handle, r.ctypes.data_as(C.c_void_p), r.shape[0], _ptr(mask),
                                     _stream_ptr(stream)), "dvl_select_mask")
        return mask

    def bin_histograms(self, bins: Bins, m: int, n_buckets: int, lo: float, hi: float, stream=None) -> torch.Tensor:
        """dvl_bin_histograms: int32 view of the uint32 counts [W, n_buckets]."""
        counts = torch.empty(bins.n_bins, int(n_buckets), dtype=torch.int32, device="cuda")
        b = bins.struct()
        _check(lib().dvl_bin_histograms(self.handle, C.byref(b), bins.n_bins, int(m), int(n_buckets), float(lo),
                                        float(hi), _ptr(counts), _stream_ptr(stream)), "dvl_bin_histograms")
        return counts

    def zoom(self, first: int, last: int, stream=None, tile_steps: int = 0, run_waves: int = 0,
             entry_cache: int = ENTRY_CACHE_AUTO, allocator: Allocator | None = None) -> "Volume":
        """dvl_zoom: a new volume of the sorted cells first..last."""
        opt = dvl_build_options(int(tile_steps), int(run_waves), int(entry_cache),
                                C.pointer(allocator.struct) if allocator is not None else None)
        out = C.c_void_p()
        _check(lib().dvl_zoom(self.handle, int(first), int(last), C.byref(opt), _stream_ptr(stream), C.byref(out)),
               "dvl_zoom")
        return Volume(out, allocator if allocator is not None else self.allocator)

    def set_entry_cache(self, policy: int):
        """dvl_set_entry_cache: ENTRY_CACHE_AUTO / ALWAYS / NEVER (NEVER frees it)."""
        _check(lib().dvl_set_entry_cache(self.handle, int(policy)), "dvl_set_entry_cache")

    def entry_cache_info(self):
        """None, or (lo, hi, n_tf) arrays of the windows the TF entry cache holds."""
        M = self.m
        lo, hi = np.zeros(M, np.float32), np.zeros(M, np.float32)
        nt = np.zeros(M, np.int32)
        P = lambda a: a.ctypes.data_as(C.c_void_p)
        if not lib().dvl_entry_cache_info(self.handle, P(lo), P(hi), P(nt)):
            return None
        return lo, hi, nt

    def set_timing(self, enable=True):
        """dvl_set_timing: record per-kernel HIP events on every update
        (True or 1: every kernel; 2: the importance pass only; False: off)."""
        _check(lib().dvl_set_timing(self.handle, int(enable)), "dvl_set_timing")

    def kernel_times(self):
        """dvl_kernel_times: ({phase: summed ms}, number of updates), then reset."""
        ms = np.zeros(5, np.float64)
        n = C.c_int32()
        _check(lib().dvl_kernel_times(self.handle, ms.ctypes.data_as(C.c_void_p), C.byref(n)),
               "dvl_kernel_times")
        names = ("vmax_exact", "tile_sums", "carry", "bin", "bin_stats")
        return dict(zip(names, ms.tolist())), int(n.value)

    def close(self):
        if self.handle:
            lib().dvl_destroy(self.handle)
            self.handle = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


RASTER_POLYLINE, RASTER_BARS = 0, 1


def rasterize(y: torch.Tensor, n_rows: int, mode: int = RASTER_POLYLINE, stream=None) -> torch.Tensor:
    """dvl_rasterize: uint8 images [L, n_rows, W] of the lines y [L, W] (device float32)."""
    y = _dev(y, torch.float32)
    if y.dim() == 1:
        y = y[None]
    L, W = y.shape
    img = torch.empty(L, int(n_rows), W, dtype=torch.uint8, device=y.device)
    _check(lib().dvl_rasterize(_ptr(y), L, W, int(n_rows), int(mode), _ptr(img), _stream_ptr(stream)),
           "dvl_rasterize")
    return img


def update_workspace_bytes(n_cells: int, n_fields: int, n_bins: int) -> int:
    return int(lib().dvl_update_workspace_bytes(int(n_cells), int(n_fields), int(n_bins)))


# ---------------------------------------------------------------- batches

def request_bytes(vol: "Volume", n_bins: int) -> int:
    """dvl_request_bytes: device bytes one request on `vol` needs (workspace + outputs)."""
    return int(lib().dvl_request_bytes(vol.handle, int(n_bins)))


class Request:
    """One update request (``dvl_request``): a volume, its [M][n_tf] alpha
    tables, optional windows (None: the data ranges), parameters and outputs.
    Keeps the host arrays alive for as long as the C struct points at them."""

    def __init__(self, vol: "Volume", alpha, bins: Bins | None = None, lo=None, hi=None, **kw):
        self.vol = vol
        a = np.ascontiguousarray(np.asarray(alpha, dtype=np.float32))
        if a.ndim != 2 or a.shape[0] != vol.m:
            raise ValueError(f"alpha must be [{vol.m}][n_tf], got {a.shape}")
        self.alpha = a
        self.lo = None if lo is None else np.ascontiguousarray(np.asarray(lo, np.float32))
        self.hi = None if hi is None else np.ascontiguousarray(np.asarray(hi, np.float32))
        n_bins = kw.pop("n_bins", None)
        if bins is None:
            bins = Bins(n_bins or 1920, vol.m)
        self.bins = bins
        self.params = params(bins.n_bins, **kw)

    def struct(self) -> dvl_request:
        P = lambda a: None if a is None else a.ctypes.data_as(C.c_void_p)
        return dvl_request(self.vol.handle, P(self.alpha), int(self.alpha.shape[1]), P(self.lo), P(self.hi),
                           self.params, self.bins.struct())


def _request_array(reqs) -> C.Array:
    arr = (dvl_request * len(reqs))()
    for i, r in enumerate(reqs):
        arr[i] = r.struct()
    return arr


class Executor:
    """``dvl_executor``: runs batches of requests, one launch per phase."""

    def __init__(self, allocator: Allocator | None = None):
        h = C.c_void_p()
        if allocator is None:
            _check(lib().dvl_executor_create(C.byref(h)), "dvl_executor_create")
        else:
            _check(lib().dvl_executor_create_ex(C.byref(allocator.struct), C.byref(h)), "dvl_executor_create_ex")
        self.allocator = allocator
        self.handle = h

    @property
    def nbytes(self) -> int:
        return int(lib().dvl_executor_bytes(self.handle))

    def update_batch(self, reqs, stream=None):
        """dvl_update_batch: enqueue every request of `reqs` on the stream."""
        arr = _request_array(reqs)
        _check(lib().dvl_update_batch(self.handle, arr, len(reqs), _stream_ptr(stream)), "dvl_update_batch")

    def set_timing(self, enable=True):
        _check(lib().dvl_executor_set_timing(self.handle, int(enable)), "dvl_executor_set_timing")

    def kernel_times(self):
        ms = np.zeros(5, np.float64)
        n = C.c_int32()
        _check(lib().dvl_executor_kernel_times(self.handle, ms.ctypes.data_as(C.c_void_p), C.byref(n)),
               "dvl_executor_kernel_times")
        names = ("vmax_exact", "tile_sums", "carry", "bin", "bin_stats")
        return dict(zip(names, ms.tolist())), int(n.value)

    def close(self):
        if self.handle:
            lib().dvl_executor_destroy(self.handle)
            self.handle = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Graph:
    """``dvl_graph``: a fixed batch captured once into a HIP graph and
    replayed with new TFs."""

    def __init__(self, reqs):
        self.reqs = list(reqs)
        arr = _request_array(self.reqs)
        h = C.c_void_p()
        _check(lib().dvl_graph_create(arr, len(self.reqs), C.byref(h)), "dvl_graph_create")
        self.handle = h

    def set_tf(self, i: int, alpha, lo=None, hi=None):
        """dvl_graph_set_tf: new [M][n_tf] tables (and windows) for request i."""
        r = self.reqs[i]
        a = np.ascontiguousarray(np.asarray(alpha, dtype=np.float32))
        if a.shape != r.alpha.shape:
            raise ValueError(f"alpha must keep the shape {r.alpha.shape}")
        lo = None if lo is None else np.ascontiguousarray(np.asarray(lo, np.float32))
        hi = None if hi is None else np.ascontiguousarray(np.asarray(hi, np.float32))
        P = lambda x: None if x is None else x.ctypes.data_as(C.c_void_p)
        _check(lib().dvl_graph_set_tf(self.handle, int(i), P(a), P(lo), P(hi)), "dvl_graph_set_tf")

    def set_tf_all(self, alphas):
        """dvl_graph_set_tf_all: new [M][n_tf] tables for every request (data-range windows)."""
        arrs = []
        for r, a in zip(self.reqs, alphas):
            a = np.ascontiguousarray(np.asarray(a, dtype=np.float32))
            if a.shape != r.alpha.shape:
                raise ValueError(f"alpha must keep the shape {r.alpha.shape}")
            arrs.append(a)
        if len(arrs) != len(self.reqs):
            raise ValueError("one table set per request")
        ptrs = (C.c_void_p * len(arrs))(*[a.ctypes.data for a in arrs])
        _check(lib().dvl_graph_set_tf_all(self.handle, C.cast(ptrs, C.c_void_p), None, None), "dvl_graph_set_tf_all")

    def launch(self, stream=None):
        _check(lib().dvl_graph_launch(self.handle, _stream_ptr(stream)), "dvl_graph_launch")

    def close(self):
        if self.handle:
            lib().dvl_graph_destroy(self.handle)
            self.handle = C.c_void_p()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
