"""ctypes view of include/sca.h (argument marshalling only).

Loads paper_2311_04435_amd/lib/libsca.so.  There is no fallback: if the
library is missing the import fails with the command that builds it.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "lib", "libsca.so")

SCA_OK, SCA_EINVAL, SCA_ENOMEM, SCA_EDEVICE, SCA_ENUMERIC, SCA_EUNSUPPORTED = \
    0, -1, -2, -3, -4, -5
STATUS_NAMES = {0: "SCA_OK", -1: "SCA_EINVAL", -2: "SCA_ENOMEM",
                -3: "SCA_EDEVICE", -4: "SCA_ENUMERIC", -5: "SCA_EUNSUPPORTED"}
SCA_FP64, SCA_FP32_REFINED = 0, 1
SCA_FACTOR_LU, SCA_FACTOR_LDLT, SCA_FACTOR_EIGH = 0, 1, 2
SCA_FLAG_NONFINITE, SCA_FLAG_PIVOT_GROWTH, SCA_FLAG_CONVERGED = 1, 2, 4
SCA_FLAG_TAIL_RANGE = 8
SCA_TAIL_NONE, SCA_TAIL_MOMENTS = 0, 1
SCA_ADAM_NO_FINAL_EVAL = 1
SCA_OPT_FP32_GROWTH_LIMIT = 1
PROFILE_SLOTS = 16
KERNEL_CLASSES = ("small", "lu", "trtri", "diagdot", "reduce", "setup",
                  "refine", "wvgemm", "ldlt", "trtri_sym", "symdiag",
                  "fallback", "tail", "tridiag", "spectrum", "expand")

# Every symbol include/sca.h declares.
EXPORTS = ("sca_create", "sca_destroy", "sca_footprint_bytes", "sca_potential",
           "sca_grad", "sca_adam_solve", "sca_hmc", "sca_dos",
           "sca_shifted_terms", "sca_tail_split", "sca_set_option",
           "sca_grad_noalloc",
           "sca_factor_bytes", "sca_factorize", "sca_grad_from_factors",
           "sca_profile", "sca_profile_read", "sca_server_create",
           "sca_server_destroy", "sca_server_clock", "sca_server_submit",
           "sca_server_progress", "sca_server_poll", "sca_last_error")


class Params(C.Structure):
    _fields_ = [("L", C.c_int32), ("n_max", C.c_int32),
                ("precision", C.c_int32), ("factor", C.c_int32),
                ("t", C.c_double), ("U", C.c_double), ("delta", C.c_double),
                ("T", C.c_double), ("onsite", C.c_void_p),
                ("tail", C.c_int32), ("reserved", C.c_int32)]


class HmcOpts(C.Structure):
    _fields_ = [("eps", C.c_double), ("n_leap", C.c_int32),
                ("n_traj", C.c_int32)]


class AdamOpts(C.Structure):
    _fields_ = [("lr", C.c_double), ("beta1", C.c_double),
                ("beta2", C.c_double), ("eps", C.c_double),
                ("grad_tol", C.c_double), ("n_steps", C.c_int32),
                ("check_every", C.c_int32), ("t0", C.c_int32),
                ("flags", C.c_int32)]


class Result(C.Structure):
    _fields_ = [("omega", C.c_double), ("omega_tilde", C.c_double),
                ("af_order", C.c_double), ("max_abs_grad", C.c_double),
                ("max_pivot_growth", C.c_double), ("steps_done", C.c_int32),
                ("flags", C.c_int32)]


class SCAError(RuntimeError):
    def __init__(self, status: int, message: str):
        self.status = status
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {message}")


def _load():
    if not os.path.exists(LIB_PATH):
        raise ImportError(
            f"{LIB_PATH} is missing; build it with "
            "`python paper_2311_04435_amd/build.py` (hipcc, gfx950)")
    lib = C.CDLL(LIB_PATH)
    vp, i32, dp = C.c_void_p, C.c_int32, C.c_void_p
    P, R, O = C.POINTER(Params), C.POINTER(Result), C.POINTER(AdamOpts)
    sig = {
        "sca_create": (i32, [C.c_int, vp, C.c_size_t, C.POINTER(vp)]),
        "sca_destroy": (None, [vp]),
        "sca_footprint_bytes": (C.c_size_t, [P]),
        "sca_potential": (i32, [vp, P, dp, dp]),
        "sca_grad": (i32, [vp, P, dp, dp, dp]),
        "sca_grad_noalloc": (i32, [vp, P, dp, dp, dp]),
        "sca_adam_solve": (i32, [vp, P, O, dp, dp, dp, R]),
        "sca_hmc": (i32, [vp, P, C.POINTER(HmcOpts), dp, dp,
                          C.POINTER(C.c_double), C.POINTER(i32),
                          C.POINTER(C.c_double), C.POINTER(C.c_double)]),
        "sca_dos": (i32, [vp, P, dp, dp, i32, C.c_double, dp]),
        "sca_shifted_terms": (i32, [vp, P, dp, dp, i32, dp, dp]),
        "sca_tail_split": (i32, [vp, P, dp, C.POINTER(i32)]),
        "sca_set_option": (i32, [vp, i32, C.c_double]),
        "sca_factor_bytes": (C.c_size_t, [P]),
        "sca_factorize": (i32, [vp, P, dp, vp, dp]),
        "sca_grad_from_factors": (i32, [vp, P, dp, vp, dp]),
        "sca_profile": (i32, [vp, C.c_int]),
        "sca_profile_read": (i32, [vp, C.POINTER(C.c_double),
                                   C.POINTER(C.c_int64)]),
        "sca_server_create": (i32, [C.c_int, C.c_size_t, i32, C.POINTER(vp)]),
        "sca_server_destroy": (None, [vp]),
        "sca_server_clock": (C.c_double, [vp]),
        "sca_server_submit": (i32, [vp, P, O, dp, dp, dp,
                                    C.POINTER(C.c_int64)]),
        "sca_server_progress": (i32, [vp, C.c_double, C.POINTER(i32),
                                      C.POINTER(i32)]),
        "sca_server_poll": (i32, [vp, C.c_int64, C.POINTER(i32), R,
                                  C.POINTER(C.c_double)]),
        "sca_last_error": (C.c_char_p, []),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    return lib


lib = _load()


def check(status: int) -> None:
    if status != SCA_OK:
        raise SCAError(status, lib.sca_last_error().decode())
