"""ctypes binding of ``libbddc.so`` (the C ABI declared in include/bddc.h).

Argument marshalling only.  Loading fails loudly when the library has not been
built: there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os
from ctypes import POINTER, c_char_p, c_double, c_int32, c_int64, c_void_p

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libbddc.so")

BDDC_CORNERS, BDDC_FACES, BDDC_EDGES = 1, 2, 4
ERRORS = {-1: "EINVAL", -2: "ENOMEM", -3: "EHIP", -4: "ESINGULAR", -5: "ENOTCONV", -6: "EBREAKDOWN"}


class Mesh(ctypes.Structure):
    _fields_ = [("nx", c_int32), ("ny", c_int32), ("nz", c_int32), ("h", c_double),
                ("elem_keep", c_void_p), ("node_dirichlet", c_void_p)]


class Partition(ctypes.Structure):
    _fields_ = [("n_sub", c_int32), ("elem_to_sub", c_void_p),
                ("n_subregion", c_int32), ("sub_to_subregion", c_void_p)]


class Opts(ctypes.Structure):
    _fields_ = [("constraints", c_int32), ("weights", c_int32), ("local_prec", c_int32),
                ("recycle_R", c_int32), ("recycle_strategy", c_int32), ("ritz_freeze_tol", c_double),
                ("stop_rule", c_int32), ("init_guess", c_int32), ("max_it", c_int32),
                ("save_cap", c_int32), ("use_graph", c_int32), ("autotune", c_int32),
                ("coarse_form", c_int32), ("product_cfg", c_int32 * 8),
                ("reorth", c_int32), ("adapt_max_per_face", c_int32), ("adapt_tau", c_double),
                ("local_prec_set", c_int32), ("coef_log", c_int32), ("restart_every", c_int32),
                ("adapt2_tau", c_double), ("adapt2_max_per_face", c_int32), ("adapt_lobpcg_it", c_int32)]


class BddcError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("%s (%d): %s" % (ERRORS.get(code, "?"), code, msg))
        self.code = code


SIGNATURES = {
    "bddc_default_opts": (None, [POINTER(Opts)]),
    "bddc_setup": (c_int32, [POINTER(Mesh), POINTER(Partition), c_void_p, POINTER(Opts), c_void_p, POINTER(c_void_p)]),
    "dpcg_solve": (c_int32, [c_void_p, c_void_p, c_int32, c_double, c_void_p, c_void_p, c_void_p]),
    "recycle_update": (c_int32, [c_void_p]),
    "bddc_reset_recycle": (c_int32, [c_void_p]),
    "bddc_adjoint_grad": (c_int32, [c_void_p, c_void_p, c_int32, c_void_p, c_double, c_void_p, c_void_p]),
    "bddc_adjoint_grad_block": (c_int32, [c_void_p, c_void_p, c_int32, c_void_p, c_double, c_void_p, c_void_p,
                                          POINTER(c_int32)]),
    "bddc_apply_schur": (c_int32, [c_void_p, c_void_p, c_void_p]),
    "bddc_apply_precond": (c_int32, [c_void_p, c_void_p, c_void_p]),
    "bddc_apply_schur_noalloc": (c_int32, [c_void_p, c_void_p, c_void_p]),
    "bddc_condense": (c_int32, [c_void_p, c_void_p, c_void_p]),
    "bddc_info": (c_int32, [c_void_p, POINTER(c_int64)]),
    "bddc_interface_nodes": (c_int32, [c_void_p, POINTER(c_int64)]),
    "bddc_enable_timing": (c_int32, [c_void_p, c_int32]),
    "bddc_stats": (c_int32, [c_void_p, POINTER(c_double), c_int32]),
    "bddc_ritz_values": (c_int32, [c_void_p, POINTER(c_double), c_int32, POINTER(c_int32)]),
    "bddc_tuning": (c_int32, [c_void_p, POINTER(c_double)]),
    "bddc_time_products": (c_int32, [c_void_p, c_int32, POINTER(c_double)]),
    "bddc_adaptive_stats": (c_int32, [c_void_p, POINTER(c_double)]),
    "bddc_adaptive2_stats": (c_int32, [c_void_p, POINTER(c_double)]),
    "bddc_set_local_prec": (c_int32, [c_void_p, c_int32]),
    "bddc_set_launch": (c_int32, [c_void_p, c_int32, c_void_p]),
    "bddc_time_kernels": (c_int32, [c_void_p, c_int32, POINTER(c_double), c_int32]),
    "bddc_solve_info": (c_int32, [c_void_p, POINTER(c_int64), c_int32]),
    "bddc_face_constraints": (c_int32, [c_int32, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p,
                                        c_int32, c_int32, c_int32, c_void_p, c_int32, c_void_p, c_double,
                                        c_int32, c_void_p, POINTER(c_int32), c_void_p, POINTER(c_int32)]),
    "bddc_face_constraints_lobpcg": (c_int32, [c_int32, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p,
                                               c_int32, c_int32, c_int32, c_void_p, c_int32, c_void_p, c_double,
                                               c_int32, c_int32, c_void_p, POINTER(c_int32), c_void_p,
                                               POINTER(c_int32), POINTER(c_int32)]),
    "bddc_destroy": (None, [c_void_p]),
    "bddc_last_error": (c_char_p, []),
}

_lib = None


def load(path: str = LIB_PATH):
    """Load the shared library and declare every exported signature."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError("libbddc.so not built at %s: run `python -m paper_2412_17543_amd.build`" % path)
    lib = ctypes.CDLL(path)
    for name, (res, args) in SIGNATURES.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


def check(rc: int):
    if rc != 0:
        raise BddcError(rc, load().bddc_last_error().decode())
