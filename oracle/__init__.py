"""Python access to the FP64 CPU oracle (test infrastructure only).

Only the test suite, ``__graft_entry__.smoke`` and the benchmark's CPU
baseline leg may import this package.  The GPU library never does, and this
package never imports the GPU library.  It wraps ``dvl_oracle.c`` (plain C,
single-threaded, FP64) through ctypes, with numpy arrays in and out.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "dvl_oracle.c")
_LIB = os.path.join(_HERE, "libdvl_oracle.so")

VMAX_TF_RANGE, VMAX_TF_BOUND, VMAX_EXACT = 0, 1, 2


def build(force: bool = True) -> str:
    """Compile the oracle with gcc into ``oracle/libdvl_oracle.so``."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-ffp-contract=off", "-fPIC", "-shared",
                               "-Wall", "-Wextra", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB)
    return _LIB


class _Params(C.Structure):
    _fields_ = [("n_bins", C.c_int32), ("exponent", C.c_double), ("min_importance", C.c_double),
                ("vmax_mode", C.c_int32), ("clamp_mode", C.c_int32), ("level_scale", C.c_int32)]


class _Bins(C.Structure):
    _fields_ = [("first", C.c_void_p), ("last", C.c_void_p), ("count", C.c_void_p),
                ("sum", C.c_void_p), ("mean", C.c_void_p), ("vmin", C.c_void_p),
                ("vmax", C.c_void_p), ("y", C.c_void_p), ("f_total", C.c_double),
                ("vmax_used", C.c_double), ("degenerate", C.c_int32)]


_lib = None


def bind(path: str):
    """Load an oracle shared library and declare its C signatures."""
    L = C.CDLL(path)
    L.ora_grid_bits.restype = C.c_int32
    L.ora_grid_bits.argtypes = [C.c_int64] + [C.c_void_p] * 4
    L.ora_hilbert_index.restype = C.c_uint64
    L.ora_hilbert_index.argtypes = [C.c_uint32, C.c_uint32, C.c_uint32, C.c_int32]
    L.ora_cell_keys.restype = None
    L.ora_cell_keys.argtypes = [C.c_int64] + [C.c_void_p] * 4 + [C.c_int32, C.c_void_p]
    L.ora_sort_order.restype = C.c_int64
    L.ora_sort_order.argtypes = [C.c_int64, C.c_void_p, C.c_void_p]
    L.ora_quantiser.restype = None
    L.ora_quantiser.argtypes = [C.c_int32, C.c_float, C.c_float, C.POINTER(C.c_float), C.POINTER(C.c_float)]
    L.ora_tf_index.restype = C.c_int32
    L.ora_tf_index.argtypes = [C.c_float, C.c_float, C.c_float, C.c_int32]
    L.ora_vmax_tf.restype = C.c_double
    L.ora_vmax_tf.argtypes = [C.c_int32, C.c_int32, C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p]
    L.ora_update.restype = C.c_int32
    L.ora_update.argtypes = [C.c_int64, C.c_int32, C.c_void_p, C.c_void_p, C.c_int32, C.c_void_p,
                             C.c_void_p, C.c_void_p, C.POINTER(_Params), C.POINTER(_Bins),
                             C.c_void_p, C.c_void_p]
    L.ora_field_range.restype = None
    L.ora_field_range.argtypes = [C.c_int64, C.c_void_p, C.POINTER(C.c_float), C.POINTER(C.c_float)]
    L.ora_bin_histograms.restype = C.c_int32
    L.ora_bin_histograms.argtypes = [C.c_int64, C.c_void_p, C.c_int32, C.c_void_p, C.c_void_p, C.c_int32,
                                     C.c_float, C.c_float, C.c_void_p]
    L.ora_rasterize.restype = C.c_int32
    L.ora_rasterize.argtypes = [C.c_int32, C.c_void_p, C.c_int32, C.c_int32, C.c_void_p]
    return L


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build(force=True)
        _lib = bind(_LIB)
    return _lib


def use_library(L):
    """Swap the loaded library (the mutation tests load planted-mistake
    copies of the oracle); returns the previous one."""
    global _lib
    prev, _lib = _lib, L
    return prev


def _p(a: np.ndarray):
    return a.ctypes.data_as(C.c_void_p)


def _c(a, dtype):
    return np.ascontiguousarray(np.asarray(a), dtype=dtype)


def grid_bits(x, y, z, level) -> int:
    x, y, z, level = _c(x, np.int32), _c(y, np.int32), _c(z, np.int32), _c(level, np.uint8)
    return int(lib().ora_grid_bits(x.size, _p(x), _p(y), _p(z), _p(level)))


def hilbert_index(qx: int, qy: int, qz: int, bits: int) -> int:
    return int(lib().ora_hilbert_index(qx, qy, qz, bits))


def cell_keys(x, y, z, level, bits: int) -> np.ndarray:
    x, y, z, level = _c(x, np.int32), _c(y, np.int32), _c(z, np.int32), _c(level, np.uint8)
    out = np.empty(x.size, dtype=np.uint64)
    lib().ora_cell_keys(x.size, _p(x), _p(y), _p(z), _p(level), bits, _p(out))
    return out


def sort_order(keys):
    keys = _c(keys, np.uint64)
    perm = np.empty(keys.size, dtype=np.uint32)
    dup = int(lib().ora_sort_order(keys.size, _p(keys), _p(perm)))
    return perm, dup


@dataclass
class Order:
    bits: int
    keys: np.ndarray        # uint64 [n], original order
    perm: np.ndarray        # uint32 [n]
    duplicates: int


def build_order(x, y, z, level) -> Order:
    """Keys at finest-level resolution and the Hilbert sort permutation."""
    b = grid_bits(x, y, z, level)
    if b < 0:
        raise ValueError("invalid cells (negative corner, level > 20 or grid beyond 2^21)")
    keys = cell_keys(x, y, z, level, b)
    perm, dup = sort_order(keys)
    return Order(b, keys, perm, dup)


def quantiser(n_tf: int, lo: float, hi: float):
    s, b = C.c_float(), C.c_float()
    lib().ora_quantiser(n_tf, lo, hi, C.byref(s), C.byref(b))
    return s.value, b.value


def tf_index(x: float, s: float, b: float, n_tf: int) -> int:
    return int(lib().ora_tf_index(x, s, b, n_tf))


def vmax_tf(mode: int, alpha, i_m, j_m) -> float:
    alpha = _c(alpha, np.float32)
    M, n_tf = alpha.shape
    i_m, j_m = _c(i_m, np.int32), _c(j_m, np.int32)
    return float(lib().ora_vmax_tf(mode, M, n_tf, _p(alpha), _p(i_m), _p(j_m)))


def field_range(v):
    v = _c(v, np.float32)
    lo, hi = C.c_float(), C.c_float()
    lib().ora_field_range(v.size, _p(v), C.byref(lo), C.byref(hi))
    return lo.value, hi.value


@dataclass
class Bins:
    first: np.ndarray       # uint32 [W]
    last: np.ndarray
    count: np.ndarray
    sum: np.ndarray         # float64 [M, W]
    mean: np.ndarray        # float64 [M, W]
    vmin: np.ndarray        # float32 [M, W]
    vmax: np.ndarray
    y: np.ndarray
    f_total: float
    vmax_used: float
    degenerate: bool
    cell_f: np.ndarray | None = None   # float64 [n]
    cell_e: np.ndarray | None = None   # float64 [n + 1]


def update(level, fields, alpha, lo, hi, n_bins: int, exponent: float = 1.0,
           min_importance: float = 0.025, vmax_mode: int = VMAX_TF_RANGE,
           clamp_mode: int = 0, level_scale: int = 1, keep_cells: bool = False) -> Bins:
    """One DVL update over cells already in Hilbert order.

    level: uint8 [n]; fields: float32 [M, n]; alpha: float32 [M, n_tf];
    lo, hi: float32 [M] normalisation windows."""
    level = _c(level, np.uint8)
    fields = _c(fields, np.float32)
    if fields.ndim == 1:
        fields = fields[None, :]
    alpha = _c(alpha, np.float32)
    if alpha.ndim == 1:
        alpha = alpha[None, :]
    M, n = fields.shape
    n_tf = alpha.shape[1]
    lo, hi = _c(lo, np.float32), _c(hi, np.float32)
    W = int(n_bins)
    first = np.empty(W, np.uint32); last = np.empty(W, np.uint32); count = np.empty(W, np.uint32)
    s = np.empty((M, W), np.float64); mean = np.empty((M, W), np.float64)
    vmin = np.empty((M, W), np.float32); vmax = np.empty((M, W), np.float32); y = np.empty((M, W), np.float32)
    cf = np.empty(n, np.float64) if keep_cells else None
    ce = np.empty(n + 1, np.float64) if keep_cells else None
    par = _Params(W, float(exponent), float(min_importance), vmax_mode, clamp_mode, level_scale)
    out = _Bins(_p(first).value, _p(last).value, _p(count).value, _p(s).value, _p(mean).value,
                _p(vmin).value, _p(vmax).value, _p(y).value, 0.0, 0.0, 0)
    rc = lib().ora_update(n, M, _p(level), _p(fields), n_tf, _p(alpha), _p(lo), _p(hi),
                          C.byref(par), C.byref(out), _p(cf) if cf is not None else None,
                          _p(ce) if ce is not None else None)
    if rc != 0:
        raise ValueError("oracle update rejected its arguments")
    return Bins(first, last, count, s, mean, vmin, vmax, y, out.f_total, out.vmax_used,
                bool(out.degenerate), cf, ce)


def default_windows(fields):
    """Per-field [min, max] normalisation windows (the data range)."""
    fields = _c(fields, np.float32)
    if fields.ndim == 1:
        fields = fields[None, :]
    r = [field_range(f) for f in fields]
    return (np.array([a for a, _ in r], np.float32), np.array([b for _, b in r], np.float32))


RASTER_POLYLINE, RASTER_BARS = 0, 1


def bin_histograms(values, first, last, n_buckets: int, lo: float, hi: float) -> np.ndarray:
    """Per-bin histograms [W, H] of sorted `values` over the bins' cell ranges."""
    values = _c(values, np.float32)
    first, last = _c(first, np.uint32), _c(last, np.uint32)
    W = first.size
    out = np.empty((W, int(n_buckets)), np.uint32)
    rc = lib().ora_bin_histograms(values.size, _p(values), W, _p(first), _p(last), int(n_buckets),
                                  float(lo), float(hi), _p(out))
    if rc != 0:
        raise ValueError("oracle histograms rejected their arguments")
    return out


def rasterize(y, n_rows: int, mode: int = RASTER_POLYLINE) -> np.ndarray:
    """Image [H, W] (uint8 0/1, row 0 at the bottom) of one line of heights."""
    y = _c(y, np.float32)
    img = np.empty((int(n_rows), y.size), np.uint8)
    if lib().ora_rasterize(y.size, _p(y), int(n_rows), int(mode), _p(img)) != 0:
        raise ValueError("oracle raster rejected its arguments")
    return img
