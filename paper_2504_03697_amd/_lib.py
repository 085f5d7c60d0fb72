"""ctypes declarations of the C ABI in include/cfdmi.h (argument marshalling only)."""
from __future__ import annotations

import ctypes
import os
import re

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libcfdmi.so")
HEADER = os.path.join(os.path.dirname(HERE), "include", "cfdmi.h")

CFD_OK, CFD_EINVAL, CFD_ENOMEM, CFD_EHIP, CFD_ENOCONV, CFD_EBREAKDOWN, CFD_ENONFINITE = 0, -1, -2, -3, -4, -5, -6
ERROR_NAMES = {0: "CFD_OK", -1: "CFD_EINVAL", -2: "CFD_ENOMEM", -3: "CFD_EHIP", -4: "CFD_ENOCONV",
               -5: "CFD_EBREAKDOWN", -6: "CFD_ENONFINITE"}


class CfdGrid(ctypes.Structure):
    _fields_ = [("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32), ("h", ctypes.c_double)]


class CfdSolveOpts(ctypes.Structure):
    _fields_ = [("precision", ctypes.c_int32), ("max_iters", ctypes.c_int32), ("ru_delta", ctypes.c_double),
                ("net", ctypes.c_void_p), ("chunk", ctypes.c_int32), ("timing", ctypes.c_int32),
                ("formulation", ctypes.c_int32), ("step_guess", ctypes.c_int32),
                ("precond", ctypes.c_int32), ("debug_breakdown_at", ctypes.c_int32),
                ("stop_margin", ctypes.c_double), ("driver", ctypes.c_int32),
                ("barrier_spins", ctypes.c_int32)]


class CfdSolveInfo(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int32), ("updates", ctypes.c_int32), ("status", ctypes.c_int32),
                ("used_fallback", ctypes.c_int32), ("rel_residual", ctypes.c_double),
                ("init_residual", ctypes.c_double), ("gamma", ctypes.c_double), ("seconds", ctypes.c_double),
                ("spmv_ms", ctypes.c_double), ("spmv_samples", ctypes.c_int32), ("pad_", ctypes.c_int32),
                ("stop_margin", ctypes.c_double)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_ if k != "pad_"}


class CfdState(ctypes.Structure):
    _fields_ = [("grid", CfdGrid), ("u", ctypes.c_void_p), ("v", ctypes.c_void_p), ("w", ctypes.c_void_p),
                ("p", ctypes.c_void_p), ("nu", ctypes.c_double), ("rho", ctypes.c_double),
                ("lid_u", ctypes.c_double), ("gx", ctypes.c_double), ("gy", ctypes.c_double),
                ("gz", ctypes.c_double), ("t", ctypes.c_double), ("step", ctypes.c_int64),
                ("A", ctypes.c_void_p), ("rhs", ctypes.c_void_p)]


_lib = None


def header_functions():
    """Names of the functions declared in include/cfdmi.h."""
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(cfd_[a-z0-9_]+)\s*\(", text)))


def load():
    """Load libcfdmi.so; raises ImportError when it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2504_03697_amd.build` "
                          "(there is no fallback implementation)")
    lib = ctypes.CDLL(LIB_PATH)
    vp, i32, i64, dbl, flt = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_double, ctypes.c_float
    P = ctypes.POINTER
    sig = {
        "cfd_assemble": (i32, [P(CfdGrid), i64, vp, P(vp)]),
        "cfd_csr_info": (i32, [vp, P(i64), P(i64)]),
        "cfd_csr_export": (i32, [vp, vp, vp, vp, vp]),
        "cfd_csr_destroy": (None, [vp]),
        "cfd_spmv": (i32, [vp, i32, vp, vp, vp]),
        "cfd_spmv_sym": (i32, [vp, i32, vp, vp, vp]),
        "cfd_rhs_prepare": (i32, [vp, vp, vp]),
        "cfd_rhs_prepare_noalloc": (i32, [vp, vp, vp]),
        "cfd_solve": (i32, [vp, vp, vp, dbl, P(CfdSolveOpts), vp, P(CfdSolveInfo), vp]),
        "cfd_step": (i32, [P(CfdState), dbl, dbl, P(CfdSolveOpts), P(CfdSolveInfo), vp]),
        "cfd_net_create": (i32, [i32, i32, vp, P(vp)]),
        "cfd_net_param_count": (i64, [i32, i32]),
        "cfd_net_destroy": (None, [vp]),
        "cfd_net_forward": (i32, [vp, P(CfdGrid), vp, vp, vp]),
        "cfd_net_train_step": (i32, [vp, P(CfdGrid), i32, vp, vp, flt, P(flt), vp]),
        "cfd_net_gradient": (i32, [vp, P(CfdGrid), i32, vp, vp, vp, P(flt), vp]),
        "cfd_net_training_pair": (i32, [vp, P(CfdGrid), vp, vp, vp, vp, vp]),
        "cfd_net_get_params": (i32, [vp, vp, i64]),
        "cfd_net_set_params": (i32, [vp, vp, i64]),
        "cfd_conv3d_forward": (i32, [P(CfdGrid), i32, i32, vp, vp, vp, i32, vp]),
        "cfd_conv3d_backward_data": (i32, [P(CfdGrid), i32, i32, vp, vp, vp, vp]),
        "cfd_conv3d_backward_weight": (i32, [P(CfdGrid), i32, i32, vp, vp, vp, vp]),
        "cfd_last_error": (ctypes.c_char_p, []),
    }
    for name, (res, args) in sig.items():
        if not hasattr(lib, name):
            continue
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    _lib = lib
    return lib


class CfdError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{ERROR_NAMES.get(code, code)}: {msg}")
        self.code = code


def check(code):
    if code != CFD_OK:
        raise CfdError(code, load().cfd_last_error().decode())
    return code
