"""Seeded synthetic inputs (AMR volumes, fields, transfer functions).

Input generation only: this package holds none of the volume-line method's
arithmetic and is shared by the oracle tests and the GPU path's tests and
benchmark as a source of identical inputs.
"""
from .amr import Volume, make_amr, make_regular, make_tf, make_tfs, refine_amr, SEED
from .configs import cfg1, cfg2, cfg3, cfg4, cfg4_volume, cfg5, cfg5_volume, tfs_for, P_DEFAULT, FMIN_DEFAULT

__all__ = ["Volume", "make_amr", "make_regular", "make_tf", "make_tfs", "refine_amr", "SEED",
           "cfg1", "cfg2", "cfg3", "cfg4", "cfg4_volume", "cfg5", "cfg5_volume", "tfs_for", "P_DEFAULT", "FMIN_DEFAULT"]
