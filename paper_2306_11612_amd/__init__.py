"""MI355X-native dynamic volume lines over multi-field AMR data.

Hot path (HIP kernels for gfx950 behind the C ABI in include/dvl.h):
one-time Hilbert ordering (``build_order``) and per-update TF lookup,
variation, importance, prefix sum and bin reduction (``update``), batched
over many volumes and TF requests (``Executor``, ``Graph``).
The ctypes binding lives in ``paper_2306_11612_amd.dvl``.
"""
from .dvl import (Bins, DvlError, Executor, Graph, Request, Volume, build_order, params,  # noqa: F401
                  read_bins, request_bytes, set_tf, update,
                  F32, F16, BF16, VMAX_TF_RANGE, VMAX_TF_BOUND, VMAX_EXACT,
                  SCAN_FP64, SCAN_KAHAN_FP32, SCAN_NAIVE_FP32)
