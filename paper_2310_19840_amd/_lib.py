"""ctypes declarations of the C interface in include/sbi.h, sbi_net.h and sbi_batch.h (libsbi.so)."""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libsbi.so")

SBI_OK = 0
SBI_WARN_NOT_CONVERGED = 1
SBI_WARN_DEPTH_CRITERION = 2
SBI_WARN_FALLBACK_USED = 3
SBI_WARN_STEP_LIMIT = 4
SBI_ERR_INVALID_ARG = -1
SBI_ERR_UNSUPPORTED = -2
SBI_ERR_WORKSPACE = -3
SBI_ERR_HIP = -4
SBI_ERR_NONFINITE = -5
SBI_ERR_DIVERGED = -6

SBI_PROFILE_OFF, SBI_PROFILE_ALL, SBI_PROFILE_SWEEPS = 0, 1, 2

SBI_FP64, SBI_FP32, SBI_MIXED = 0, 1, 2
SBI_MODE_ITER, SBI_MODE_SA, SBI_MODE_FULL = 0, 1, 2
SBI_SEED_LINEAR, SBI_SEED_PREV, SBI_SEED_NET, SBI_SEED_USER = 0, 1, 2, 3
SBI_ACCEL_NONE, SBI_ACCEL_ANDERSON = 0, 1


class sbi_grid(C.Structure):
    _fields_ = [
        ("nx", C.c_int32), ("ny", C.c_int32),
        ("lx", C.c_double), ("ly", C.c_double),
        ("order", C.c_int32),
        ("dealias", C.c_double),
        ("precision", C.c_int32), ("mode", C.c_int32), ("seed", C.c_int32),
        ("max_sweeps", C.c_int32), ("relax", C.c_int32),
        ("filter_beta1", C.c_double), ("filter_beta2", C.c_double),
        ("accel", C.c_int32),
    ]


class sbi_state(C.Structure):
    _fields_ = [("eta", C.c_void_p), ("phi_s", C.c_void_p), ("t", C.c_double)]


class sbi_solve_info(C.Structure):
    _fields_ = [("sweeps", C.c_int32), ("status", C.c_int32), ("residual", C.c_double), ("omega", C.c_double),
                ("sweeps_fp32", C.c_int32)]


class sbi_step_info(C.Structure):
    _fields_ = [("solves", C.c_int64), ("sweeps_total", C.c_int64), ("sweeps_max", C.c_int32),
                ("fallbacks", C.c_int32), ("max_residual", C.c_double), ("sweeps_fp32_total", C.c_int64)]


class sbi_adapt_info(C.Structure):
    _fields_ = [("accepted", C.c_int32), ("rejected", C.c_int32), ("dt_next", C.c_double),
                ("err_last", C.c_double), ("err_max", C.c_double), ("solve", sbi_step_info)]


class sbi_plan(C.Structure):
    _fields_ = [("row_variant", C.c_int32), ("row_rows", C.c_int32), ("col_split", C.c_int32), ("us", C.c_float),
                ("cached", C.c_int32)]


SBI_TUNE_FORCE = 1

# exported symbols and their signatures: (restype, argtypes)
SIGNATURES = {
    "sbi_grid_defaults": (None, [C.POINTER(sbi_grid)]),
    "sbi_workspace_bytes": (C.c_size_t, [C.POINTER(sbi_grid), C.c_int32]),
    "sbi_init": (C.c_int, [C.POINTER(C.c_void_p), C.POINTER(sbi_grid), C.c_int32, C.POINTER(C.c_double),
                           C.c_double, C.c_void_p, C.c_size_t, C.c_void_p]),
    "sbi_vertical_velocity": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.POINTER(C.c_double), C.c_double,
                                        C.c_void_p, C.c_void_p, C.POINTER(sbi_solve_info)]),
    "sbi_vertical_velocity_noalloc": (C.c_int, [C.POINTER(sbi_grid), C.c_int32, C.POINTER(C.c_double), C.c_double,
                                                C.c_void_p, C.c_void_p, C.c_double, C.c_void_p, C.c_void_p,
                                                C.POINTER(sbi_solve_info), C.c_void_p]),
    "sbi_step": (C.c_int, [C.c_void_p, C.POINTER(sbi_state), C.c_double, C.c_int32, C.c_double,
                           C.POINTER(sbi_step_info)]),
    "sbi_step_adaptive": (C.c_int, [C.c_void_p, C.POINTER(sbi_state), C.c_double, C.c_double, C.c_double,
                                    C.c_double, C.c_int32, C.POINTER(sbi_adapt_info)]),
    "sbi_diagnostics": (C.c_int, [C.c_void_p, C.POINTER(sbi_state), C.c_double, C.POINTER(C.c_double),
                                  C.POINTER(C.c_double)]),
    "sbi_set_relaxation": (C.c_int, [C.c_void_p, C.POINTER(C.c_double), C.c_int32]),
    "sbi_set_wavemaker": (C.c_int, [C.c_void_p, C.POINTER(C.c_double), C.c_int32, C.c_double, C.c_double,
                                    C.c_double]),
    "sbi_set_depth": (C.c_int, [C.c_void_p, C.POINTER(C.c_double), C.c_double]),
    "sbi_net_load": (C.c_int, [C.c_void_p, C.c_void_p, C.c_size_t]),
    "sbi_destroy": (C.c_int, [C.c_void_p]),
    "sbi_status_string": (C.c_char_p, [C.c_int]),
    "sbi_last_stats": (C.c_int32, [C.c_void_p, C.POINTER(C.c_double), C.c_int32]),
    "sbi_profile_enable": (C.c_int, [C.c_void_p, C.c_int32]),
    "sbi_profile_read": (C.c_int32, [C.c_void_p, C.POINTER(C.c_char_p), C.POINTER(C.c_double),
                                     C.POINTER(C.c_int64), C.c_int32]),
    # learned warm start (sbi_net.h)
    "sbi_net_param_count": (C.c_int32, []),
    "sbi_net_blob_bytes": (C.c_size_t, []),
    "sbi_net_features": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "sbi_net_infer": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p]),
    "sbi_last_correction": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p]),
    "sbi_net_hist_param_count": (C.c_int32, [C.c_int32, C.c_int32]),
    "sbi_net_hist_load": (C.c_int, [C.c_void_p, C.c_int32, C.c_int32, C.c_double, C.POINTER(C.c_float)]),
    "sbi_net_hist_train": (C.c_int, [C.c_void_p, C.c_int32]),
    "sbi_net_hist_gradient": (C.c_int, [C.c_void_p, C.POINTER(C.c_double), C.POINTER(C.c_int32),
                                        C.POINTER(C.c_double), C.POINTER(C.c_double)]),
    "sbi_net_hist_newton": (C.c_int, [C.c_void_p, C.c_double, C.POINTER(C.c_double), C.POINTER(C.c_int32)]),
    "sbi_net_hist_adam": (C.c_int, [C.c_void_p, C.c_float, C.POINTER(C.c_double), C.POINTER(C.c_int32)]),
    "sbi_net_hist_params": (C.c_int, [C.c_void_p, C.POINTER(C.c_float)]),
    "sbi_net_trainer_bytes": (C.c_size_t, [C.c_int32, C.c_int32, C.c_int32]),
    "sbi_net_trainer_init": (C.c_int, [C.POINTER(C.c_void_p), C.c_int32, C.c_int32, C.c_int32,
                                       C.POINTER(C.c_float), C.c_void_p, C.c_size_t, C.c_void_p]),
    "sbi_net_trainer_forward": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p]),
    "sbi_net_trainer_gradient": (C.c_int, [C.c_void_p, C.c_void_p, C.c_void_p, C.POINTER(C.c_double),
                                           C.POINTER(C.c_float)]),
    "sbi_net_trainer_adam": (C.c_int, [C.c_void_p, C.c_float]),
    "sbi_net_trainer_params": (C.c_int, [C.c_void_p, C.POINTER(C.c_float)]),
    "sbi_net_trainer_destroy": (C.c_int, [C.c_void_p]),
    # launch plans and the autotuner (sbi.h)
    "sbi_plan_variants": (C.c_int32, [C.c_void_p]),
    "sbi_plan_get": (C.c_int, [C.c_void_p, C.POINTER(sbi_plan)]),
    "sbi_plan_set": (C.c_int, [C.c_void_p, C.POINTER(sbi_plan)]),
    "sbi_autotune": (C.c_int, [C.c_void_p, C.c_int32, C.POINTER(sbi_plan)]),
    "sbi_tune_cache_load": (C.c_int, [C.c_char_p, C.POINTER(C.c_int32)]),
    "sbi_tune_cache_save": (C.c_int, [C.c_char_p, C.POINTER(C.c_int32)]),
    # ensembles of uneven grids (sbi_batch.h)
    "sbi_batch_workspace_bytes": (C.c_size_t, [C.c_int32, C.POINTER(sbi_grid)]),
    "sbi_batch_init": (C.c_int, [C.POINTER(C.c_void_p), C.c_int32, C.POINTER(sbi_grid),
                                 C.POINTER(C.POINTER(C.c_double)), C.c_double, C.c_void_p, C.c_size_t, C.c_void_p,
                                 C.c_int32]),
    "sbi_batch_step": (C.c_int, [C.c_void_p, C.POINTER(sbi_state), C.c_double, C.c_int32, C.c_double,
                                 C.POINTER(sbi_step_info)]),
    "sbi_batch_groups": (C.c_int32, [C.c_void_p, C.POINTER(C.c_int32), C.POINTER(C.c_int32), C.c_int32]),
    "sbi_batch_budgets": (C.c_int32, [C.c_void_p, C.POINTER(C.c_int32), C.c_int32]),
    "sbi_batch_plan": (C.c_int, [C.c_void_p, C.c_int32, C.POINTER(sbi_plan)]),
    "sbi_batch_destroy": (C.c_int, [C.c_void_p]),
    "sbi_batch_net_load": (C.c_int, [C.c_void_p, C.c_void_p, C.c_size_t]),
    "sbi_batch_net_hist_load": (C.c_int, [C.c_void_p, C.c_int32, C.c_int32, C.c_double, C.POINTER(C.c_float)]),
}

SBI_BATCH_GRAPH, SBI_BATCH_AUTOTUNE = 1, 2

SBI_NET_PARAMS = 12706


class sbi_net_header(C.Structure):
    _fields_ = [("magic", C.c_char * 4), ("version", C.c_uint32), ("cin", C.c_uint32), ("width", C.c_uint32),
                ("nparams", C.c_uint32), ("in_scale", C.c_float * 8), ("out_scale", C.c_float * 2),
                ("reserved", C.c_float * 1)]

_lib = None


def load(path: str | None = None):
    """Load libsbi.so; raises if it has not been built (there is no fallback)."""
    global _lib
    if _lib is not None and path is None:
        return _lib
    p = path or LIB_PATH
    if not os.path.exists(p):
        raise RuntimeError(f"{p} is missing: build it with `python -m paper_2310_19840_amd.build`")
    lib = C.CDLL(p)
    for name, (res, args) in SIGNATURES.items():
        f = getattr(lib, name)
        f.restype = res
        f.argtypes = args
    if path is None:
        _lib = lib
    return lib


def status_string(code: int) -> str:
    return load().sbi_status_string(code).decode()


class SBIError(RuntimeError):
    def __init__(self, code: int, where: str, info=None):
        super().__init__(f"{where}: {status_string(code)} ({code})")
        self.code = code
        self.info = info  # per-member solve info the call reported with the error, if any
