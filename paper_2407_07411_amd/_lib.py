"""ctypes declarations of the C ABI in include/dmrg_heff.h (marshalling only)."""
from __future__ import annotations

import ctypes
import os
from ctypes import POINTER, c_char_p, c_double, c_int, c_int32, c_int64, c_void_p

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libdmrg_heff.so")

DMRG_OK = 0
STATUS = {0: "DMRG_OK", -1: "DMRG_EINVAL", -2: "DMRG_EQN", -3: "DMRG_ENOMEM", -4: "DMRG_EHIP",
          -5: "DMRG_ENOCONV", -6: "DMRG_ENOTSUP"}
FP64, SPLIT_BF16X3, FP32 = 0, 1, 3


class Term(ctypes.Structure):
    _fields_ = [("dq", c_int32 * 2), ("odd", c_int32), ("hc", c_int32), ("one_sided", c_int32),
                ("reserved", c_int32), ("coeff", c_double), ("left_off", POINTER(c_int64)),
                ("right_off", POINTER(c_int64))]


class TermSU2(ctypes.Structure):
    _fields_ = [("two_k", c_int32), ("dn", c_int32), ("odd", c_int32), ("hc", c_int32),
                ("one_sided", c_int32), ("reserved", c_int32), ("coeff", c_double),
                ("n_left", c_int64), ("n_right", c_int64), ("left_blocks", POINTER(c_int64)),
                ("right_blocks", POINTER(c_int64))]


class DavOpts(ctypes.Structure):
    _fields_ = [("max_iter", c_int32), ("max_subspace", c_int32), ("restart_keep", c_int32),
                ("use_graph", c_int32), ("tol", c_double), ("fp64_tail", c_int32),
                ("start", c_int32)]


class DavResult(ctypes.Structure):
    _fields_ = [("energy", c_double), ("residual", c_double), ("iters", c_int32),
                ("matvecs", c_int32), ("converged", c_int32), ("tail_iters", c_int32),
                ("split_residual", c_double), ("split_iters", c_int32), ("reserved", c_int32),
                ("split_energy", c_double)]


class DmrgError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


# exported symbol -> (restype, argtypes)
SIGNATURES = {
    "dmrg_ctx_create": (c_int, [c_int, c_void_p, POINTER(c_void_p)]),
    "dmrg_ctx_set_stream": (c_int, [c_void_p, c_void_p]),
    "dmrg_ctx_destroy": (None, [c_void_p]),
    "dmrg_last_error": (c_char_p, []),
    "dmrg_build_info": (c_char_p, []),
    "dmrg_basis_create": (c_int, [c_void_p, c_int32, POINTER(c_int32), POINTER(c_int64), POINTER(c_void_p)]),
    "dmrg_basis_destroy": (None, [c_void_p]),
    "dmrg_wfn_layout": (c_int, [c_void_p, c_void_p, POINTER(c_int32), POINTER(c_int64), POINTER(c_int64),
                                POINTER(c_int64)]),
    "dmrg_heff_create": (c_int, [c_void_p, c_void_p, c_void_p, POINTER(c_int32), c_int64, POINTER(Term),
                                 c_void_p, c_int64, c_void_p, c_int64, c_int, POINTER(c_void_p)]),
    "dmrg_heff_create_streamed": (c_int, [c_void_p, c_void_p, c_void_p, POINTER(c_int32), c_int64, POINTER(Term),
                                          c_void_p, c_int64, c_void_p, c_int64, c_int, c_int64,
                                          POINTER(c_void_p)]),
    "dmrg_heff_stream_info": (c_int, [c_void_p, POINTER(c_int64), POINTER(c_int64), POINTER(c_int32),
                                      POINTER(c_int32)]),
    "dmrg_su2_weight": (c_double, [c_int32, c_int32, c_int32, c_int32, c_int32, c_int32]),
    "dmrg_wfn_layout_su2": (c_int, [c_void_p, c_void_p, POINTER(c_int32), POINTER(c_int64), c_void_p, c_void_p,
                                    c_void_p, POINTER(c_int64)]),
    "dmrg_heff_create_su2": (c_int, [c_void_p, c_void_p, c_void_p, POINTER(c_int32), c_int64, POINTER(TermSU2),
                                     c_void_p, c_int64, c_void_p, c_int64, c_int, POINTER(c_void_p)]),
    "dmrg_heff_destroy": (None, [c_void_p]),
    "dmrg_heff_set_precision": (c_int, [c_void_p, c_int]),
    "dmrg_heff_set_persistent": (c_int, [c_void_p, c_int32]),
    "dmrg_heff_check": (c_int, [c_void_p]),
    "dmrg_heff_flops": (c_int, [c_void_p, POINTER(c_double), POINTER(c_double)]),
    "dmrg_heff_size": (c_int64, [c_void_p]),
    "dmrg_heff_apply": (c_int, [c_void_p, c_void_p, c_void_p]),
    "dmrg_heff_diag": (c_int, [c_void_p, c_void_p]),
    "dmrg_heff_apply_adjoint": (c_int, [c_void_p, c_void_p, c_void_p, c_void_p, c_void_p, c_void_p]),
    "dmrg_heff_workspace_bytes": (c_int64, [c_void_p]),
    "dmrg_heff_use_graph": (c_int, [c_void_p, c_int32]),
    "dmrg_heff_autotune": (c_int, [c_void_p, c_void_p, c_void_p, c_int32]),
    "dmrg_heff_launches": (c_int, [c_void_p, POINTER(c_int64), POINTER(c_int32), POINTER(c_double)]),
    "dmrg_heff_apply_profiled": (c_int, [c_void_p, c_void_p, c_void_p, POINTER(ctypes.c_float)]),
    "dmrg_davidson_create": (c_int, [c_void_p, POINTER(DavOpts), c_void_p, POINTER(c_void_p)]),
    "dmrg_davidson_step": (c_int, [c_void_p, POINTER(DavResult)]),
    "dmrg_davidson_vector": (c_int, [c_void_p, c_void_p]),
    "dmrg_davidson_destroy": (None, [c_void_p]),
    "dmrg_davidson": (c_int, [c_void_p, c_void_p, POINTER(DavOpts), POINTER(DavResult)]),
    "dmrg_chain_create": (c_int, [c_void_p, c_int32, c_void_p, c_void_p, c_int32, c_int32, c_int64,
                                  ctypes.c_uint64, POINTER(c_void_p)]),
    "dmrg_chain_destroy": (None, [c_void_p]),
    "dmrg_chain_step": (c_int, [c_void_p, c_int32, c_int32, POINTER(DavOpts), POINTER(c_double),
                                POINTER(c_double), POINTER(DavResult)]),
    "dmrg_chain_grow_left": (c_int, [c_void_p, c_int32]),
    "dmrg_chain_export": (c_int, [c_void_p, c_int32, POINTER(c_int32), POINTER(c_int32), POINTER(c_int64),
                                  POINTER(c_int64), POINTER(c_int64), c_void_p, c_void_p, c_void_p, c_void_p,
                                  c_void_p, c_void_p, c_void_p, c_void_p, c_void_p]),
    "dmrg_svd_truncate": (c_int, [c_void_p, c_void_p, c_void_p, POINTER(c_int32), c_void_p, c_int64, c_double,
                                  POINTER(c_int64), c_void_p, c_int64, c_void_p, c_int64, c_void_p, c_int64,
                                  POINTER(c_double)]),
    "dmrg_svd_truncate_noalloc": (c_int, [c_void_p, c_void_p, c_void_p, POINTER(c_int32), c_void_p, c_int64, c_double,
                                  POINTER(c_int64), c_void_p, c_int64, c_void_p, c_int64, c_void_p, c_int64,
                                  POINTER(c_double)]),
}

_lib = None


def lib():
    """Load the built library; fails loudly when it is missing."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built; run `python -m paper_2407_07411_amd.build`")
        handle = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(handle, name)
            fn.restype = res
            fn.argtypes = args
        _lib = handle
    return _lib


def check(status):
    if status != DMRG_OK:
        raise DmrgError(status, lib().dmrg_last_error().decode())
    return status
