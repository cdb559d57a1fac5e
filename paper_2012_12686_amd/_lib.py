"""ctypes binding of the C ABI declared in include/adorym.h.

Argument marshalling only: every step of the computation runs in the HIP
kernels of ``libadorym.so``.  The library must have been built
(``python -m paper_2012_12686_amd.build``); loading fails loudly otherwise.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libadorym.so")

# adorym_status
OK, EINVAL, EUNSUPPORTED, ERANGE, ENOMEM, EDEVICE = 0, 1, 2, 3, 4, 5
STATUS_NAMES = {OK: "OK", EINVAL: "EINVAL", EUNSUPPORTED: "EUNSUPPORTED", ERANGE: "ERANGE",
                ENOMEM: "ENOMEM", EDEVICE: "EDEVICE"}
LOSS_GAUSSIAN, LOSS_POISSON = 0, 1
OBJ_DELTA_BETA, OBJ_REAL_IMAG = 0, 1
ACCUMULATE_GRADS = 1
DETERMINISTIC = 2
PROP_PARAXIAL = 0
PROP_SOMMERFELD = 1


class Geom(ctypes.Structure):
    """Mirror of ``adorym_geom``."""

    _fields_ = [
        ("n", ctypes.c_int32), ("n_slices", ctypes.c_int32),
        ("obj_ny", ctypes.c_int32), ("obj_nx", ctypes.c_int32),
        ("wavelength_m", ctypes.c_double), ("pixel_m", ctypes.c_double), ("slice_dz_m", ctypes.c_double),
        ("loss", ctypes.c_int32), ("obj_repr", ctypes.c_int32), ("ckpt_every", ctypes.c_int32),
        ("eps", ctypes.c_double), ("flags", ctypes.c_uint32),
    ]


class Job(ctypes.Structure):
    """Mirror of ``adorym_job``."""

    _fields_ = [
        ("g", Geom),
        ("obj_a", ctypes.c_void_p), ("obj_b", ctypes.c_void_p), ("probe", ctypes.c_void_p),
        ("corner", ctypes.c_void_p), ("shift", ctypes.c_void_p), ("batch", ctypes.c_int32),
        ("i_meas", ctypes.c_void_p),
        ("loss", ctypes.c_void_p), ("g_a", ctypes.c_void_p), ("g_b", ctypes.c_void_p),
        ("g_probe", ctypes.c_void_p), ("g_shift", ctypes.c_void_p),
        ("workspace", ctypes.c_void_p), ("ws_bytes", ctypes.c_size_t),
        ("intensity", ctypes.c_void_p),
    ]


# name -> (restype, argtypes); every function include/adorym.h declares
_P = ctypes.c_void_p
_GP = ctypes.POINTER(Geom)
SIGNATURES = {
    "adorym_create": (ctypes.c_int, [ctypes.POINTER(_P), ctypes.c_int, _P]),
    "adorym_destroy": (ctypes.c_int, [_P]),
    "adorym_set_stream": (ctypes.c_int, [_P, _P]),
    "adorym_supports_n": (ctypes.c_int, [ctypes.c_int32]),
    "adorym_workspace_size": (ctypes.c_size_t, [_GP, ctypes.c_int32]),
    "adorym_forward_workspace_size": (ctypes.c_size_t, [_GP, ctypes.c_int32]),
    "adorym_forward": (ctypes.c_int, [_P, _GP, _P, _P, _P, _P, _P, ctypes.c_int32, _P, _P, ctypes.c_size_t]),
    "adorym_forward_static": (ctypes.c_int, [_P, _GP, _P, _P, _P, _P, _P, ctypes.c_int32, _P]),
    "adorym_loss_grad": (ctypes.c_int, [_P, _GP, _P, _P, _P, _P, _P, ctypes.c_int32, _P, _P, ctypes.c_size_t,
                                        _P, _P, _P, _P, _P, _P]),
    "adorym_forward_defocus": (ctypes.c_int, [_P, _GP, _P, _P, _P, _P, _P, ctypes.c_int32, ctypes.c_double, _P, _P,
                                              ctypes.c_size_t]),
    "adorym_loss_grad_defocus": (ctypes.c_int, [_P, _GP, _P, _P, _P, _P, _P, ctypes.c_int32, ctypes.c_double, _P,
                                                _P, ctypes.c_size_t, _P, _P, _P, _P, _P, _P, _P]),
    "adorym_nearfield_workspace_size": (ctypes.c_size_t, [_GP, ctypes.c_int32, ctypes.c_int32]),
    "adorym_forward_nearfield": (ctypes.c_int, [_P, _GP, _P, _P, _P, _P, _P, ctypes.c_int32, ctypes.c_int32, _P,
                                                ctypes.c_int32, _P, _P, _P, ctypes.c_size_t]),
    "adorym_loss_grad_nearfield": (ctypes.c_int, [_P, _GP, _P, _P, _P, _P, _P, ctypes.c_int32, ctypes.c_int32, _P,
                                                  ctypes.c_int32, _P, _P, _P, ctypes.c_size_t, _P, _P, _P, _P, _P,
                                                  _P, _P]),
    "adorym_loss_fwd_workspace_size": (ctypes.c_size_t, [_GP, ctypes.c_int32]),
    "adorym_loss_fwd": (ctypes.c_int, [_P, _GP, _P, _P, _P, _P, _P, ctypes.c_int32, _P, _P, ctypes.c_size_t, _P,
                                       _P]),
    "adorym_loss_bwd": (ctypes.c_int, [_P, _GP, _P, _P, _P, _P, _P, ctypes.c_int32, _P, _P, ctypes.c_size_t,
                                       ctypes.c_double, _P, _P, _P, _P]),
    "adorym_loss_grad_batched": (ctypes.c_int, [_P, _P, ctypes.c_int32]),
    "adorym_autotune": (ctypes.c_int, [_P, _P, ctypes.c_int32, ctypes.c_int32, _P]),
    "adorym_gaps_workspace_size": (ctypes.c_size_t, [_GP, ctypes.c_int32]),
    "adorym_forward_gaps": (ctypes.c_int, [_P, _GP, _P, _P, _P, _P, _P, ctypes.c_int32, _P, _P, _P,
                                           ctypes.c_size_t]),
    "adorym_loss_grad_gaps": (ctypes.c_int, [_P, _GP, _P, _P, _P, _P, _P, ctypes.c_int32, _P, _P, _P,
                                             ctypes.c_size_t, _P, _P, _P, _P, _P, _P, _P]),
    "adorym_prior_workspace_size": (ctypes.c_size_t, [ctypes.c_int32, ctypes.c_int32, ctypes.c_int32]),
    "adorym_prior_grad": (ctypes.c_int, [_P, ctypes.c_int32, _P, _P, ctypes.c_int32, ctypes.c_int32,
                                         ctypes.c_int32, ctypes.c_double, ctypes.c_double, ctypes.c_double, _P, _P,
                                         _P, ctypes.c_size_t, _P, _P, _P, ctypes.c_int32]),
    "adorym_prior_weights": (ctypes.c_int, [_P, ctypes.c_int32, _P, _P, ctypes.c_int32, ctypes.c_int32,
                                            ctypes.c_int32, ctypes.c_double, _P, ctypes.c_size_t, _P, _P]),
    "adorym_support_project": (ctypes.c_int, [_P, ctypes.c_int32, _P, _P, _P, ctypes.c_size_t]),
    "adorym_modes_workspace_size": (ctypes.c_size_t, [_GP, ctypes.c_int32, ctypes.c_int32]),
    "adorym_loss_grad_modes": (ctypes.c_int, [_P, _GP, _P, _P, _P, ctypes.c_int32, _P, _P, ctypes.c_int32, _P, _P,
                                              ctypes.c_size_t, _P, _P, _P, _P, _P, _P]),
    "adorym_rotate": (ctypes.c_int, [_P, _P, _P, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, ctypes.c_double,
                                     ctypes.c_int]),
    "adorym_adam": (ctypes.c_int, [_P, _P, _P, _P, _P, ctypes.c_size_t, ctypes.c_double, ctypes.c_double,
                                   ctypes.c_double, ctypes.c_double, ctypes.c_int32]),
    "adorym_adam_dev": (ctypes.c_int, [_P, _P, _P, _P, _P, ctypes.c_size_t, ctypes.c_double, ctypes.c_double,
                                       ctypes.c_double, ctypes.c_double, _P]),
    "adorym_sync_error": (ctypes.c_int, [_P]),
    "adorym_last_error_message": (ctypes.c_char_p, [_P]),
    "adorym_set_split": (ctypes.c_int, [_P, ctypes.c_int32, ctypes.c_int32]),
    "adorym_plan_create": (ctypes.c_int, [_P, ctypes.POINTER(Job), ctypes.c_int32, ctypes.POINTER(_P)]),
    "adorym_plan_run": (ctypes.c_int, [_P, _P]),
    "adorym_plan_destroy": (ctypes.c_int, [_P]),
    "adorym_profile_start": (ctypes.c_int, [_P, ctypes.c_int32]),
    "adorym_profile_stop": (ctypes.c_int, [_P, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(ctypes.c_int32)]),
}

_lib = None


def load():
    """Load libadorym.so (once).  Raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_2012_12686_amd.build`")
        lib = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
    return _lib


class AdorymError(RuntimeError):
    def __init__(self, status, message=""):
        super().__init__(f"adorym: {STATUS_NAMES.get(status, status)}: {message}")
        self.status = status


def check(status, ctx=None):
    if status != OK:
        msg = ""
        if ctx is not None:
            raw = load().adorym_last_error_message(ctx)
            msg = raw.decode() if raw else ""
        raise AdorymError(status, msg)
