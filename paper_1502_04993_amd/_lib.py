"""ctypes declarations of the glmrec C ABI (include/glmrec.h).

Argument marshalling only: every step of the likelihood runs in libglmrec.so.
Importing this module raises if the library has not been built; there is no
other implementation to fall back to.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libglmrec.so")

GLMR_OK = 0
GLMR_NOT_CONVERGED = 1
GLMR_EINVAL = -1
GLMR_ENOMEM = -2
GLMR_EDEVICE = -3
GLMR_ENOSPIKES = -4
GLMR_ENONFINITE = -5
GLMR_ESTATE = -6

GLMR_FP64, GLMR_FP32, GLMR_BF16, GLMR_FP8, GLMR_BF16_J2 = 0, 1, 2, 3, 4
GLMR_HOST, GLMR_DEVICE = 0, 1
GLMR_TRACE_AUTO, GLMR_TRACE_RESIDENT, GLMR_TRACE_RECOMPUTE = 0, 1, 2
TRACE_MODES = {"auto": GLMR_TRACE_AUTO, "resident": GLMR_TRACE_RESIDENT, "recompute": GLMR_TRACE_RECOMPUTE}

PRECISIONS = {"fp64": GLMR_FP64, "fp32": GLMR_FP32, "bf16": GLMR_BF16, "fp8": GLMR_FP8,
              "bf16j2": GLMR_BF16_J2}
GLMR_TIME_GRID, GLMR_TIME_EVENTS = 0, 1
TIME_MODES = {"grid": GLMR_TIME_GRID, "events": GLMR_TIME_EVENTS}


class glmr_config(ctypes.Structure):
    _fields_ = [("n_neurons", ctypes.c_int32), ("n_bins", ctypes.c_int64), ("dt", ctypes.c_double),
                ("chunk_bins", ctypes.c_int64), ("precision", ctypes.c_int32),
                ("device", ctypes.c_int32), ("stream", ctypes.c_void_p), ("tile_n", ctypes.c_int32),
                ("trace", ctypes.c_int32), ("time_mode", ctypes.c_int32)]


class glmr_fit_opts(ctypes.Structure):
    _fields_ = [("max_iter", ctypes.c_int32), ("ftol", ctypes.c_double), ("lbfgs_m", ctypes.c_int32),
                ("max_backtracks", ctypes.c_int32), ("warm_start_mu", ctypes.c_int32),
                ("from_zero", ctypes.c_int32), ("l1_alpha", ctypes.c_double),
                ("l1_eps", ctypes.c_double), ("j_max", ctypes.c_double), ("rate_min", ctypes.c_double),
                ("rate_max", ctypes.c_double), ("resume", ctypes.c_int32), ("keep_history", ctypes.c_int32)]


class glmr_fit_report(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int32), ("evals", ctypes.c_int32), ("ll", ctypes.c_double),
                ("max_eta", ctypes.c_double), ("rows_converged", ctypes.c_int32),
                ("seconds", ctypes.c_double)]


# every symbol the header declares, with (restype, argtypes)
_vp = ctypes.c_void_p
_dp = ctypes.POINTER(ctypes.c_double)
SIGNATURES = {
    "glmr_create": (ctypes.c_int, [ctypes.POINTER(glmr_config), ctypes.POINTER(_vp)]),
    "glmr_destroy": (None, [_vp]),
    "glmr_set_spikes": (ctypes.c_int, [_vp, _vp, _vp, ctypes.c_int64, ctypes.c_int32]),
    "glmr_event_slots": (ctypes.c_int, [_vp, ctypes.c_int64, ctypes.c_double, ctypes.c_double,
                                        ctypes.c_double, ctypes.POINTER(ctypes.c_int64)]),
    "glmr_set_spike_times": (ctypes.c_int, [_vp, _vp, _vp, ctypes.c_int64, ctypes.c_double, ctypes.c_double,
                                            ctypes.c_double, ctypes.c_int32]),
    "glmr_ei_interval": (None, [ctypes.c_double, ctypes.c_double, _dp, _dp]),
    "glmr_ei_interval_f32": (None, [ctypes.c_float, ctypes.c_double, ctypes.POINTER(ctypes.c_float),
                                    ctypes.POINTER(ctypes.c_float)]),
    "glmr_set_kernel": (ctypes.c_int, [_vp, ctypes.c_double]),
    "glmr_set_kernel_noalloc": (ctypes.c_int, [_vp, ctypes.c_double]),
    "glmr_get_state": (ctypes.c_int, [_vp, _vp, ctypes.POINTER(ctypes.c_size_t)]),
    "glmr_set_state": (ctypes.c_int, [_vp, ctypes.c_char_p, ctypes.c_size_t]),
    "glmr_set_delays": (ctypes.c_int, [_vp, ctypes.c_int64, ctypes.c_int64]),
    "glmr_set_precision": (ctypes.c_int, [_vp, ctypes.c_int32]),
    "glmr_set_params": (ctypes.c_int, [_vp, _vp, _vp, ctypes.c_int32]),
    "glmr_get_params": (ctypes.c_int, [_vp, _vp, _vp, _dp, ctypes.c_int32]),
    "glmr_eval": (ctypes.c_int, [_vp, _dp, _vp, _vp, _vp, _dp, ctypes.c_int32]),
    "glmr_fit_defaults": (None, [ctypes.POINTER(glmr_fit_opts)]),
    "glmr_fit": (ctypes.c_int, [_vp, ctypes.POINTER(glmr_fit_opts), ctypes.POINTER(glmr_fit_report)]),
    "glmr_batch_create": (ctypes.c_int, [ctypes.POINTER(_vp), ctypes.c_int32, ctypes.POINTER(_vp)]),
    "glmr_batch_destroy": (None, [_vp]),
    "glmr_batch_eval": (ctypes.c_int, [_vp, _dp]),
    "glmr_batch_get_grad": (ctypes.c_int, [_vp, ctypes.c_int32, _vp, _vp, ctypes.c_int32]),
    "glmr_batch_autotune": (ctypes.c_int, [_vp, ctypes.c_char_p, ctypes.POINTER(ctypes.c_int32),
                                           ctypes.POINTER(ctypes.c_int32)]),
    "glmr_batch_fit": (ctypes.c_int, [_vp, ctypes.POINTER(glmr_fit_opts), ctypes.POINTER(glmr_fit_report)]),
    "glmr_status_string": (ctypes.c_char_p, [ctypes.c_int]),
    "glmr_last_error": (ctypes.c_char_p, [_vp]),
    "glmr_prof_enable": (ctypes.c_int, [_vp, ctypes.c_int32]),
    "glmr_prof_get": (ctypes.c_int32, [_vp, ctypes.POINTER(ctypes.c_char_p), _dp,
                                        ctypes.POINTER(ctypes.c_int64), ctypes.c_int32]),
    "glmr_prof_reset": (None, [_vp]),
    "glmr_autotune": (ctypes.c_int, [_vp, ctypes.c_char_p, ctypes.POINTER(ctypes.c_int32),
                                     ctypes.POINTER(ctypes.c_int32)]),
    "glmr_query": (ctypes.c_int, [_vp, ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int64),
                                  ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int32),
                                  ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32)]),
}

_lib = None


def load():
    """Load libglmrec.so (built by paper_1502_04993_amd/build.py)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_1502_04993_amd.build` "
                          "(there is no fallback implementation)")
    lib = ctypes.CDLL(LIB_PATH)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


class GlmrError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"glmrec status {status}: {msg}")
        self.status = status
