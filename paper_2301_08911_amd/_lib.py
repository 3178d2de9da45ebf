"""Loader of the in-tree HIP library; there is no fallback implementation."""
from __future__ import annotations

import ctypes
import os

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libhmg.so")

SYMBOLS = (
    "hmg_create", "hmg_destroy", "hmg_set_density", "hmg_solve_cases", "hmg_elastic_tensor",
    "hmg_sensitivity", "hmg_oc_update", "hmg_filter", "hmg_get_displacement", "hmg_last_error",
    "hmg_num_levels", "hmg_level_dims", "hmg_level_omega", "hmg_apply_operator", "hmg_get_stencil",
    "hmg_load_vectors", "hmg_vcycle", "hmg_transfer", "hmg_profile", "hmg_profile_read",
    "hmg_element_constants", "hmg_filter_sensitivity", "hmg_symmetrize", "hmg_trig_init",
    "hmg_objective", "hmg_should_stop",
    "hmg_batch_create", "hmg_batch_destroy", "hmg_batch_set_density", "hmg_batch_tune",
    "hmg_batch_solve", "hmg_batch_elastic_tensors", "hmg_batch_last_error",
    # include/hmg_nn.h
    "hmg_nn_create", "hmg_nn_destroy", "hmg_nn_param_count", "hmg_nn_get_params",
    "hmg_nn_set_params", "hmg_nn_get_grads", "hmg_nn_forward", "hmg_nn_backward",
    "hmg_nn_zero_grad", "hmg_nn_adam_step", "hmg_nn_mse", "hmg_warm_start",
    "hmg_conv3d_forward", "hmg_conv3d_backward_data", "hmg_conv3d_backward_weight",
    "hmg_conv3d_workspace", "hmg_conv3d_backward_weight_noalloc",
    "hmg_conv3d_noalloc_scratch_floats",
)


class HmgConfig(ctypes.Structure):
    """Mirror of ``hmg_config`` in include/hmg.h."""
    _fields_ = [
        ("nx", ctypes.c_int32), ("ny", ctypes.c_int32), ("nz", ctypes.c_int32),
        ("E0", ctypes.c_double), ("nu", ctypes.c_double), ("penal", ctypes.c_double),
        ("Emin", ctypes.c_double), ("levels", ctypes.c_int32), ("omega", ctypes.c_double),
        ("nu_pre", ctypes.c_int32), ("nu_post", ctypes.c_int32), ("precision", ctypes.c_int32),
        ("replace_every", ctypes.c_int32), ("smoother", ctypes.c_int32),
        ("post_fp16", ctypes.c_int32), ("nondyadic", ctypes.c_int32),
    ]


class HmgNnConfig(ctypes.Structure):
    """Mirror of ``hmg_nn_config`` in include/hmg_nn.h."""
    _fields_ = [("levels", ctypes.c_int32), ("base_channels", ctypes.c_int32),
                ("in_channels", ctypes.c_int32), ("out_channels", ctypes.c_int32)]


_lib = None


def load() -> ctypes.CDLL:
    """Load libhmg.so (built by ``paper_2301_08911_amd.build``) and declare signatures."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(
            f"{LIB_PATH} is missing: build it with `python -m paper_2301_08911_amd.build` "
            "(the solver has no CPU fallback)")
    lib = ctypes.CDLL(LIB_PATH)
    vp, i32, f64, i64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_double, ctypes.c_int64
    P = ctypes.POINTER
    sig = {
        "hmg_create": ([P(HmgConfig), vp, P(vp)], i32),
        "hmg_destroy": ([vp], i32),
        "hmg_set_density": ([vp, vp], i32),
        "hmg_solve_cases": ([vp, f64, i32, i32, vp, P(i32), P(f64)], i32),
        "hmg_elastic_tensor": ([vp, P(f64)], i32),
        "hmg_sensitivity": ([vp, P(f64), vp], i32),
        "hmg_oc_update": ([vp, vp, vp, f64, f64, f64, f64, P(f64)], i32),
        "hmg_filter": ([vp, vp, vp, f64, i32], i32),
        "hmg_get_displacement": ([vp, vp], i32),
        "hmg_filter_sensitivity": ([vp, vp, vp, vp, f64], i32),
        "hmg_symmetrize": ([vp, vp, vp, i32], i32),
        "hmg_trig_init": ([vp, i32, P(f64), P(f64), i32, f64, f64, f64, vp, P(f64)], i32),
        "hmg_objective": ([i32, P(f64), i32, P(f64), P(f64), P(f64)], i32),
        "hmg_should_stop": ([P(f64), i32, f64, i32, i32, P(i32)], i32),
        "hmg_last_error": ([vp], ctypes.c_char_p),
        "hmg_num_levels": ([vp, P(i32)], i32),
        "hmg_level_dims": ([vp, i32, P(i32)], i32),
        "hmg_level_omega": ([vp, i32, P(f64)], i32),
        "hmg_element_constants": ([f64, P(f64), P(f64), P(f64), P(f64)], i32),
        "hmg_apply_operator": ([vp, i32, vp, vp], i32),
        "hmg_get_stencil": ([vp, i32, vp], i32),
        "hmg_load_vectors": ([vp, vp], i32),
        "hmg_vcycle": ([vp, vp, vp], i32),
        "hmg_transfer": ([vp, i32, i32, vp, vp], i32),
        "hmg_profile": ([vp, i32], i32),
        "hmg_profile_read": ([vp, i32, P(ctypes.c_int64), P(f64), P(f64)], i32),
        "hmg_batch_create": ([P(HmgConfig), i32, P(i32), vp, P(vp)], i32),
        "hmg_batch_destroy": ([vp], i32),
        "hmg_batch_set_density": ([vp, i32, vp], i32),
        "hmg_batch_tune": ([vp, P(i32), P(i32)], i32),
        "hmg_batch_solve": ([vp, f64, i32, P(i32), P(f64)], i32),
        "hmg_batch_elastic_tensors": ([vp, P(f64)], i32),
        "hmg_batch_last_error": ([vp], ctypes.c_char_p),
        "hmg_nn_create": ([P(HmgNnConfig), vp, ctypes.c_uint64, P(vp)], i32),
        "hmg_nn_destroy": ([vp], i32),
        "hmg_nn_param_count": ([vp, P(i64)], i32),
        "hmg_nn_get_params": ([vp, vp, i64], i32),
        "hmg_nn_set_params": ([vp, vp, i64], i32),
        "hmg_nn_get_grads": ([vp, vp, i64], i32),
        "hmg_nn_forward": ([vp, vp, i32, i32, vp], i32),
        "hmg_nn_backward": ([vp, vp], i32),
        "hmg_nn_zero_grad": ([vp], i32),
        "hmg_nn_adam_step": ([vp, f64, f64, f64, f64, i32], i32),
        "hmg_nn_mse": ([vp, vp, vp, i64, vp, P(f64)], i32),
        "hmg_warm_start": ([vp, vp, f64, P(f64), P(i32)], i32),
        "hmg_conv3d_forward": ([vp, vp, vp, vp, vp, i32, i32, i32, i32, i32, i32, i32], i32),
        "hmg_conv3d_backward_data": ([vp, vp, vp, vp, i32, i32, i32, i32, i32, i32], i32),
        "hmg_conv3d_backward_weight": ([vp, vp, vp, vp, vp, vp, i32, i32, i32, i32, i32, i32],
                                       i32),
        "hmg_conv3d_workspace": ([i32, i32, i32, i32, i32, i32], i64),
        "hmg_conv3d_backward_weight_noalloc": ([vp, vp, vp, vp, vp, i32, i32, i32, i32, i32, i32],
                                               i32),
        "hmg_conv3d_noalloc_scratch_floats": ([], i64),
    }
    for name, (args, ret) in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = ret
    _lib = lib
    return lib
