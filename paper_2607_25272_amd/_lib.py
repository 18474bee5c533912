"""ctypes declarations mirroring include/spcg.h (argument marshalling only).

torch is imported before the library is loaded so that the process uses a
single HIP runtime (torch's), which both sides then share.
"""
import ctypes
import os

import torch  # noqa: F401  (loads the HIP runtime first)

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libspcg.so")

SPCG_OK = 0
SPCG_W_NOT_CONVERGED = 1
SPCG_KT_TRANSFORM_FIRST, SPCG_KT_TRANSFORM_REST, SPCG_KT_PROD_S, SPCG_KT_PROD_G = 0, 1, 2, 3
SPCG_KT_PROD_SG, SPCG_KT_PHASE_A, SPCG_KT_PHASE_B, SPCG_KT_N = 4, 5, 6, 8
SPCG_E_INVALID_ARG = -1
SPCG_E_SHAPE = -2
SPCG_E_DTYPE = -3
SPCG_E_RANK = -4
SPCG_E_BREAKDOWN = -5
SPCG_E_HIP = -6
SPCG_E_NOMEM = -7

SPCG_F64, SPCG_F32, SPCG_BF16, SPCG_FP8E4M3 = 0, 1, 2, 3
SPCG_METHOD_SPCG, SPCG_METHOD_FULL_PCG = 0, 1
SPCG_SCHEDULE_PLAIN, SPCG_SCHEDULE_LEARNED = 0, 1
SPCG_SKETCH_SRHT, SPCG_SKETCH_COUNT = 0, 1
SPCG_A_FIXED, SPCG_A_THEORY = 0, 1
SPCG_MLP_F, SPCG_MLP_H, SPCG_MLP_O = 8, 64, 8
SPCG_MLP_PARAMS = (SPCG_MLP_H * SPCG_MLP_F + SPCG_MLP_H + SPCG_MLP_H * SPCG_MLP_H + SPCG_MLP_H
                   + SPCG_MLP_O * SPCG_MLP_H + SPCG_MLP_O)
SPCG_MLP_S_SCALE = 10.0
SPCG_MLP_LAMBDA = 0.5

c_i32, c_i64, c_u64, c_f64, c_vp = (ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64,
                                    ctypes.c_double, ctypes.c_void_p)


class SpcgMat(ctypes.Structure):
    _fields_ = [("data", c_vp), ("dtype", c_i32), ("reserved", c_i32), ("rows", c_i64),
                ("cols", c_i64), ("ld", c_i64), ("col_scale", c_vp)]


class SketchOpts(ctypes.Structure):
    _fields_ = [("seed", c_u64), ("m0", c_i64), ("m_max", c_i64), ("r", c_i64),
                ("growth", c_i32), ("hat_only", c_i32), ("stage_dtype", c_i32), ("transform_segment", c_i32),
                ("kind", c_i32), ("reserved", c_i32), ("m_list", ctypes.POINTER(c_i64)),
                ("m_list_len", c_i32), ("reserved2", c_i32)]


class SketchInfo(ctypes.Structure):
    _fields_ = [("N", c_i64), ("Np", c_i64), ("d", c_i64), ("k", c_i64), ("r", c_i64),
                ("K", c_i64), ("L", c_i32), ("sketch_dtype", c_i32), ("ld", c_i64),
                ("m", c_i64 * 64), ("kind", c_i32), ("reserved", c_i32)]


class PrecondOpts(ctypes.Structure):
    _fields_ = [("qr_passes", c_i32), ("reserved", c_i32)]


class StageOpts(ctypes.Structure):
    _fields_ = [("iters", c_i32), ("refresh_gradient", c_i32), ("tol", c_f64),
                ("check_every", c_i32), ("reserved", c_i32)]


class StageStats(ctypes.Structure):
    _fields_ = [("iters", c_i32), ("converged", c_i32), ("rho0", c_f64), ("rho", c_f64),
                ("ax_norm", c_f64), ("resid_norm2", c_f64)]


class SolveOpts(ctypes.Structure):
    _fields_ = [("sketch", SketchOpts), ("precond", PrecondOpts), ("method", c_i32),
                ("a", c_i32), ("T", c_i32), ("check_every", c_i32), ("tol", c_f64),
                ("a_list", ctypes.POINTER(c_i32)), ("a_list_len", c_i32),
                ("time_phases", c_i32), ("time_products", c_i32), ("stage_stride", c_i32),
                ("schedule", c_i32), ("schedule_weights", c_vp), ("schedule_margin", c_i32),
                ("record_features", c_i32), ("batch_direct", c_i32), ("batch_tasks_per_cu", c_i32),
                ("a_rule", c_i32), ("nested_gradient", c_i32), ("omega", c_f64), ("stage_limit", c_i32),
                ("batch_shape", c_i32), ("batch_one_launch", c_i32)]


class SolveStats(ctypes.Structure):
    _fields_ = [("K", c_i32), ("T_stage1", c_i32), ("T_stage2", c_i32), ("converged", c_i32),
                ("qr_passes", c_i32), ("product_launches", c_i32), ("rho_final", c_f64),
                ("ax_norm", c_f64), ("t_sketch_ms", c_f64), ("t_precond_ms", c_f64),
                ("t_stage1_ms", c_f64), ("t_stage2_ms", c_f64), ("t_total_ms", c_f64),
                ("product_ms_sum", c_f64), ("product_bytes", c_f64), ("host_syncs", c_i32),
                ("policy_a", c_i32), ("policy_stride", c_i32), ("unchecked_iters", c_i32),
                ("fallback", c_i32), ("s_pred", ctypes.c_float), ("rho_ii0", c_f64),
                ("ax2_ii0", c_f64), ("resid2_ii0", c_f64), ("features_pre", ctypes.c_float * 8),
                ("features_ii", ctypes.c_float * 8), ("out_pre", ctypes.c_float * 8),
                ("out_ii", ctypes.c_float * 8), ("batch_tasks_per_cu", c_i32), ("batch_graphs", c_i32),
                ("kernel_ms", c_f64 * 8), ("kernel_bytes", c_f64 * 8), ("kernel_launches", c_i32 * 8),
                ("stages_planned", c_i32), ("stage_iters", c_i32 * 64), ("stage_features", ctypes.c_float * 128),
                ("stage_out", ctypes.c_float * 128), ("batch_shapes", c_i32 * 16),
                ("batch_tune_ms", ctypes.c_float * 64)]


P = ctypes.POINTER
# (name, restype, argtypes) for every symbol declared in include/spcg.h
SIGNATURES = [
    ("spcg_version", ctypes.c_char_p, []),
    ("spcg_ctx_create", c_i32, [ctypes.c_int, c_vp, P(c_vp)]),
    ("spcg_ctx_destroy", c_i32, [c_vp]),
    ("spcg_last_error", ctypes.c_char_p, [c_vp]),
    ("spcg_sketch", c_i32, [c_vp, P(SpcgMat), P(SpcgMat), P(SketchOpts), P(c_vp)]),
    ("spcg_sketch_get_info", c_i32, [c_vp, P(SketchInfo)]),
    ("spcg_sketch_view", c_i32, [c_vp, ctypes.c_int, P(SpcgMat), P(SpcgMat), P(c_f64)]),
    ("spcg_sketch_export", c_i32, [c_vp, c_vp, c_vp, c_vp, c_vp, c_vp]),
    ("spcg_sketch_free", None, [c_vp]),
    ("spcg_sketch_tables_host", c_i32, [c_u64, c_i32, c_i64, c_i64, c_vp, c_vp, c_vp, c_vp]),
    ("spcg_precond_build", c_i32, [c_vp, c_vp, P(PrecondOpts), P(c_vp)]),
    ("spcg_precond_from_r", c_i32, [c_vp, c_vp, c_i64, P(c_vp)]),
    ("spcg_precond_export", c_i32, [c_vp, c_vp, c_vp, P(c_i32)]),
    ("spcg_precond_free", None, [c_vp]),
    ("spcg_pcg_stage", c_i32, [c_vp, P(SpcgMat), P(SpcgMat), c_f64, c_vp, c_vp, P(StageOpts),
                               P(StageStats)]),
    ("spcg_pcg_stage_noalloc", c_i32, [c_vp, P(SpcgMat), P(SpcgMat), c_f64, c_vp, c_vp, P(StageOpts),
                               P(StageStats)]),
    ("spcg_solve", c_i32, [c_vp, P(SpcgMat), P(SpcgMat), P(SolveOpts), c_vp, P(SolveStats)]),
    ("spcg_solve_batched", c_i32, [c_vp, ctypes.c_int, P(SpcgMat), P(SpcgMat), P(SolveOpts), P(c_vp),
                                   P(SolveStats)]),
    ("spcg_solve_opts_default", None, [P(SolveOpts)]),
    ("spcg_mlp_forward", c_i32, [c_vp, c_vp, c_vp, c_i64, c_vp]),
    ("spcg_mlp_loss_grad", c_i32, [c_vp, c_vp, c_vp, c_vp, c_vp, c_vp, c_vp, c_vp, c_i64, c_vp, c_vp]),
    ("spcg_mlp_adam", c_i32, [c_vp, c_vp, c_vp, c_vp, c_vp, c_i64, c_i32, ctypes.c_float,
                              ctypes.c_float, ctypes.c_float, ctypes.c_float]),
]

_lib = None


def load():
    """Loads libspcg.so; raises if it has not been built (no fallback)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(
            f"{LIB_PATH} is missing: build it with `python -m paper_2607_25272_amd.build` "
            "(there is no CPU or PyTorch fallback for the SPCG path)")
    lib = ctypes.CDLL(LIB_PATH)
    for name, res, args in SIGNATURES:
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib
