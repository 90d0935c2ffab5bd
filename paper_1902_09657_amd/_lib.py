"""ctypes binding of libkpdhg (the C ABI in include/kpdhg.h).

Argument marshalling only: torch tensors supply device memory and the
current HIP stream; every step of the computation runs in the library's HIP
kernels.  There is no fallback: if the shared library is missing or cannot
be loaded, every call raises.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libkpdhg.so")

KP_OK = 0
KP_ERR_INVALID_ARG = -1
KP_ERR_UNSUPPORTED = -2
KP_ERR_OOM = -3
KP_ERR_HIP = -4
KP_PRECOND_NONE, KP_PRECOND_SC, KP_PRECOND_MC, KP_PRECOND_DCF = 0, 1, 2, 3
KP_REG_L2, KP_REG_L1_WAVELET, KP_REG_TV = 0, 1, 2

# every symbol the header declares
EXPORTS = [
    "nufft_plan", "nufft_forward", "nufft_forward_noalloc", "nufft_adjoint", "precond_build", "pdhg_lambda_max",
    "pdhg_solve", "pdhg_unrolled_ckpt_bytes", "pdhg_unrolled_forward", "pdhg_unrolled_backward",
    "nufft_destroy", "nufft_plan_info", "nufft_plan_sort", "nufft_plan_grid_coords",
    "kp_db4_filter", "nufft_plan_validate", "kp_last_error", "nufft_stage",
    "pdhg_schedule_params", "l2_dual_cg", "nufft_autotune", "nufft_plan_batch", "nufft_batch_info", "pdhg_solve_batch", "nufft_batch_destroy",
]
KP_STAGE_FWD_FFT, KP_STAGE_INTERP, KP_STAGE_SPREAD, KP_STAGE_ADJ_FFT, KP_STAGE_SPREAD_TILES, KP_STAGE_PROX = 0, 1, 2, 3, 4, 5


class KpError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__("kpdhg error %d: %s" % (code, msg))
        self.code = code


class Tuning(ctypes.Structure):
    _fields_ = [("bin_size", ctypes.c_int * 3), ("max_chunk", ctypes.c_int), ("spread_bin_size", ctypes.c_int * 3)]


class PlanInfo(ctypes.Structure):
    _fields_ = [
        ("ndim", ctypes.c_int),
        ("shape", ctypes.c_int64 * 3),
        ("grid", ctypes.c_int64 * 3),
        ("ncoils", ctypes.c_int64),
        ("nsamples", ctypes.c_int64),
        ("kb_width", ctypes.c_int),
        ("oversamp", ctypes.c_float),
        ("kb_beta", ctypes.c_double),
        ("bin_size", ctypes.c_int * 3),
        ("nbins", ctypes.c_int64),
        ("ntouch", ctypes.c_int64),
        ("nwork", ctypes.c_int64),
        ("heavy_tiles", ctypes.c_int64),
        ("workspace_bytes", ctypes.c_int64),
        ("spread_bin_size", ctypes.c_int * 3),
        ("nspread_tiles", ctypes.c_int64),
        ("max_chunk", ctypes.c_int),
    ]


class PdhgOpts(ctypes.Structure):
    _fields_ = [
        ("reg", ctypes.c_int),
        ("lam", ctypes.c_float),
        ("iters", ctypes.c_int),
        ("wavelet_levels", ctypes.c_int),
        ("lambda_max", ctypes.c_float),
        ("power_iters", ctypes.c_int),
        ("sigma0", ctypes.c_float),
        ("accel", ctypes.c_int),
        ("x0", ctypes.c_void_p),
        ("u0", ctypes.c_void_p),
        ("objective_host", ctypes.POINTER(ctypes.c_double)),
        ("lambda_max_out", ctypes.c_void_p),
    ]


_lib = None


def load(path: str = LIB_PATH):
    """Load the shared library (raises if it is not built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError("libkpdhg.so is not built (run __graft_entry__.build())")
    L = ctypes.CDLL(path)
    vp, i32, i64, f32 = ctypes.c_void_p, ctypes.c_int, ctypes.c_int64, ctypes.c_float
    P = ctypes.POINTER
    sig = {
        "nufft_plan": (i32, [P(vp), i32, P(i64), i64, i64, vp, vp, f32, i32, P(Tuning), vp]),
        "nufft_forward": (i32, [vp, vp, vp, vp]),
        "nufft_forward_noalloc": (i32, [vp, vp, vp, vp]),
        "nufft_adjoint": (i32, [vp, vp, vp, vp]),
        "precond_build": (i32, [vp, i32, vp, vp]),
        "pdhg_lambda_max": (i32, [vp, vp, i32, i32, vp, vp]),
        "pdhg_solve": (i32, [vp, vp, vp, i32, P(PdhgOpts), vp, vp, vp]),
        "pdhg_unrolled_ckpt_bytes": (i64, [vp, i32, i32]),
        "pdhg_unrolled_forward": (i32, [vp, vp, vp, i32, vp, i32, i32, vp, vp, vp, vp]),
        "pdhg_unrolled_backward": (i32, [vp, vp, vp, i32, vp, i32, i32, vp, vp, vp, vp, vp, vp, vp]),
        "nufft_destroy": (None, [vp]),
        "nufft_plan_info": (i32, [vp, P(PlanInfo)]),
        "nufft_plan_sort": (i32, [vp, vp, vp, vp, vp, vp]),
        "nufft_plan_grid_coords": (i32, [vp, vp, vp]),
        "kp_db4_filter": (i32, [P(ctypes.c_double)]),
        "nufft_plan_validate": (i32, [i32, P(i64), i64, i64, vp, vp, f32, i32, P(Tuning)]),
        "kp_last_error": (ctypes.c_char_p, []),
        "nufft_stage": (i32, [vp, i32, i32, vp]),
        "pdhg_schedule_params": (i32, [vp, vp, i32, P(PdhgOpts), vp, vp]),
        "l2_dual_cg": (i32, [vp, vp, vp, i32, f32, i32, vp, vp, P(ctypes.c_double), vp]),
        "nufft_autotune": (i32, [i32, P(i64), i64, i64, vp, vp, f32, i32, P(Tuning), vp]),
        "nufft_plan_batch": (i32, [P(vp), i32, P(i64), P(i64), i64, P(vp), P(vp), f32, i32, i32, vp]),
        "nufft_batch_info": (i32, [vp, i32, P(PlanInfo), P(i32)]),
        "pdhg_solve_batch": (i32, [vp, P(vp), P(vp), i32, P(PdhgOpts), P(f32), P(vp), vp]),
        "nufft_batch_destroy": (None, [vp]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(L, name)
        fn.restype = res
        fn.argtypes = args
    _lib = L
    return L


def check(code: int):
    if code != KP_OK:
        msg = load().kp_last_error()
        raise KpError(code, msg.decode() if msg else "")
    return code
