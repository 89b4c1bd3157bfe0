"""ctypes declarations of the C ABI in include/helm.h."""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(HERE, "libhelm.so")

HELM_C64 = 0
HELM_C128 = 1

STATUS = {0: "HELM_OK", 1: "HELM_EINVAL", 2: "HELM_ENOMEM", 3: "HELM_EHIP", 4: "HELM_ENOCONV",
          5: "HELM_EBREAKDOWN", 6: "HELM_ESTATE"}

# every symbol declared in include/helm.h
EXPORTS = ["helm_desc_default", "helm_setup", "helm_set_phase", "helm_set_rays", "helm_eikonal", "helm_set_weights", "helm_get_weights",
           "helm_get_lambdas", "helm_cycle", "helm_solve", "helm_residual", "helm_residual_noalloc",
           "helm_cycle_backward", "helm_cycle_record", "helm_cycle_reverse", "helm_loss",
           "helm_batch_setup", "helm_batch_get", "helm_batch_solve", "helm_batch_classes", "helm_batch_destroy",
           "helm_tune", "helm_set_tuning", "helm_get_tuning",
           "helm_debug_op", "helm_profile_begin", "helm_profile_end", "helm_destroy", "helm_status_string", "helm_last_error", "helm_version"]


class HelmDesc(ctypes.Structure):
    _fields_ = [
        ("n", ctypes.c_int32),
        ("levels", ctypes.c_int32),
        ("k", ctypes.c_double),
        ("damping_cells", ctypes.c_int32),
        ("damping_strength", ctypes.c_double),
        ("sign", ctypes.c_int32),
        ("cycle_prec", ctypes.c_int32),
        ("adr_steps", ctypes.c_int32),
        ("cheb_pre", ctypes.c_int32),
        ("cheb_post", ctypes.c_int32),
        ("cheb_coarse", ctypes.c_int32),
        ("gmres_m", ctypes.c_int32),
        ("gmres_coarse_m", ctypes.c_int32),
        ("level3_literal", ctypes.c_int32),
        ("restart", ctypes.c_int32),
        ("gmres_arnoldi", ctypes.c_int32),
        ("use_graphs", ctypes.c_int32),
        ("adr_levels", ctypes.c_int32),
        ("tail_n", ctypes.c_int32),
        ("wave_tail_n", ctypes.c_int32),
        ("shift", ctypes.c_double),
        ("cycle_shift", ctypes.c_double),
        ("ny", ctypes.c_int32),
    ]


class HelmError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{STATUS.get(status, status)}: {message}")
        self.status = status


_lib = None


def lib_path() -> str:
    return _LIB_PATH


def lib():
    """Loads libhelm.so once; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        raise ImportError(f"{_LIB_PATH} not found: build the HIP library first "
                          "(python -c 'import __graft_entry__ as g; g.build()')")
    L = ctypes.CDLL(_LIB_PATH)
    vp, i32, dbl = ctypes.c_void_p, ctypes.c_int32, ctypes.c_double
    P = ctypes.POINTER
    L.helm_desc_default.restype = None
    L.helm_desc_default.argtypes = [P(HelmDesc), i32, dbl]
    L.helm_setup.restype = i32
    L.helm_setup.argtypes = [P(HelmDesc), vp, P(vp), vp]
    L.helm_set_phase.restype = i32
    L.helm_set_phase.argtypes = [vp, vp, i32, vp]
    L.helm_set_rays.restype = i32
    L.helm_set_rays.argtypes = [vp, i32, vp]
    L.helm_eikonal.restype = i32
    L.helm_eikonal.argtypes = [vp, vp, i32, i32, ctypes.c_double, vp, vp, vp, vp, vp]
    L.helm_set_weights.restype = i32
    L.helm_set_weights.argtypes = [vp, P(dbl)]
    L.helm_get_weights.restype = i32
    L.helm_get_weights.argtypes = [vp, P(dbl)]
    L.helm_get_lambdas.restype = i32
    L.helm_get_lambdas.argtypes = [vp, P(dbl)]
    L.helm_cycle.restype = i32
    L.helm_cycle.argtypes = [vp, vp, vp, vp]
    L.helm_solve.restype = i32
    L.helm_solve.argtypes = [vp, vp, vp, dbl, i32, i32, P(i32), P(dbl), P(dbl), vp]
    L.helm_residual.restype = i32
    L.helm_residual.argtypes = [vp, vp, vp, vp, P(dbl), P(dbl), vp]
    L.helm_residual_noalloc.restype = i32
    L.helm_residual_noalloc.argtypes = [vp, vp, vp, vp, P(dbl), P(dbl), vp]
    L.helm_cycle_backward.restype = i32
    L.helm_cycle_backward.argtypes = [vp, i32, vp, vp, vp, vp, vp, vp, vp]
    L.helm_cycle_record.restype = i32
    L.helm_cycle_record.argtypes = [vp, i32, vp, vp, vp, vp, vp]
    L.helm_cycle_reverse.restype = i32
    L.helm_cycle_reverse.argtypes = [vp, i32, vp, vp, vp, vp, vp]
    L.helm_loss.restype = i32
    L.helm_batch_setup.restype = i32
    L.helm_batch_setup.argtypes = [i32, vp, P(vp), P(vp), i32, i32, P(vp), vp]
    L.helm_batch_get.restype = i32
    L.helm_batch_get.argtypes = [vp, i32, P(vp)]
    L.helm_batch_solve.restype = i32
    L.helm_batch_solve.argtypes = [vp, P(vp), P(vp), dbl, i32, i32, P(i32), P(dbl), P(i32), vp]
    L.helm_batch_classes.restype = i32
    L.helm_batch_classes.argtypes = [vp, P(i32)]
    L.helm_batch_destroy.restype = i32
    L.helm_tune.restype = i32
    L.helm_tune.argtypes = [vp, ctypes.c_char_p, ctypes.c_int64, vp]
    L.helm_set_tuning.restype = i32
    L.helm_set_tuning.argtypes = [vp, ctypes.c_char_p]
    L.helm_get_tuning.restype = i32
    L.helm_get_tuning.argtypes = [vp, ctypes.c_char_p, ctypes.c_int64]
    L.helm_batch_destroy.argtypes = [vp]
    L.helm_loss.argtypes = [vp, vp, vp, P(dbl), vp, vp]
    L.helm_debug_op.restype = i32
    L.helm_debug_op.argtypes = [vp, i32, i32, vp, vp, vp, vp]
    L.helm_profile_begin.restype = i32
    L.helm_profile_begin.argtypes = [vp]
    L.helm_profile_end.restype = i32
    L.helm_profile_end.argtypes = [vp, ctypes.c_char_p, ctypes.c_int64]
    L.helm_destroy.restype = i32
    L.helm_destroy.argtypes = [vp]
    L.helm_status_string.restype = ctypes.c_char_p
    L.helm_status_string.argtypes = [i32]
    L.helm_last_error.restype = ctypes.c_char_p
    L.helm_last_error.argtypes = []
    L.helm_version.restype = ctypes.c_char_p
    L.helm_version.argtypes = []
    _lib = L
    return L


def check(status: int):
    if status != 0:
        msg = lib().helm_last_error().decode(errors="replace")
        raise HelmError(status, msg)
