"""ctypes declarations of the C ABI in include/fms.h (argument marshalling only)."""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libfms.so")

FMS_OK = 0
FMS_ERR_INVALID_ARG = -1
FMS_ERR_UNSUPPORTED = -2
FMS_ERR_BAD_INPUT = -3
FMS_ERR_CAPACITY = -4
FMS_ERR_HIP = -5

FMS_PREC_FP32 = 0
FMS_PREC_BF16_REFINE = 1
FMS_PREC_BF16_SPLIT = 2

# Every entry point declared in include/fms.h.
EXPORTS = ("fms_default_params", "fms_create", "fms_destroy", "fms_cluster", "fms_cluster_batch",
           "fms_shift_seeds", "fms_shift_seeds_noalloc", "fms_unroll", "fms_unroll_backward", "fms_autotune", "fms_autotune_batch",
           "fms_clear_tuning",
           "fms_seed_order", "fms_status_string")


class FmsParams(ctypes.Structure):
    _fields_ = [
        ("bandwidth", ctypes.c_double),
        ("conv_tol", ctypes.c_double),
        ("gamma", ctypes.c_double),
        ("big_l", ctypes.c_double),
        ("big_h", ctypes.c_double),
        ("p_target", ctypes.c_double),
        ("seed", ctypes.c_uint64),
        ("n_initial", ctypes.c_int32),
        ("n_state_in", ctypes.c_int32),
        ("max_iter", ctypes.c_int32),
        ("max_rounds", ctypes.c_int32),
        ("precision", ctypes.c_int32),
        ("refine_iters", ctypes.c_int32),
        ("timing", ctypes.c_int32),
        ("tile_seeds", ctypes.c_int32),
        ("tile_items", ctypes.c_int32),
        ("tile_chunks", ctypes.c_int32),
        ("tile_waves", ctypes.c_int32),
        ("graphs", ctypes.c_int32),
    ]


class FmsFrame(ctypes.Structure):
    _fields_ = [
        ("emb", ctypes.c_void_p),
        ("pixel_stride", ctypes.c_int64),
        ("channel_stride", ctypes.c_int64),
        ("mask", ctypes.c_void_p),
        ("height", ctypes.c_int32),
        ("width", ctypes.c_int32),
        ("bandwidth", ctypes.c_double),
        ("n_state_in", ctypes.c_int32),
        ("labels", ctypes.c_void_p),
    ]


class FmsTuneEntry(ctypes.Structure):
    _fields_ = [
        ("precision", ctypes.c_int32),
        ("dim_padded", ctypes.c_int32),
        ("n_fg", ctypes.c_int32),
        ("seeds", ctypes.c_int32),
        ("tile_seeds", ctypes.c_int32),
        ("tile_items", ctypes.c_int32),
        ("tile_waves", ctypes.c_int32),
        ("us_per_step", ctypes.c_float),
        ("us_default", ctypes.c_float),
    ]

    def as_dict(self):
        return {name: getattr(self, name) for name, _ in self._fields_}


class FmsTuneReport(ctypes.Structure):
    _fields_ = [
        ("ms_default", ctypes.c_float),
        ("ms_tuned", ctypes.c_float),
        ("kept", ctypes.c_int32),
    ]


class FmsStats(ctypes.Structure):
    _fields_ = [
        ("seed_pixel_updates", ctypes.c_int64),
        ("n_min", ctypes.c_double),
        ("n_fg", ctypes.c_int32),
        ("rounds", ctypes.c_int32),
        ("seeds_used", ctypes.c_int32),
        ("iterations_total", ctypes.c_int32),
        ("refine_steps", ctypes.c_int32),
        ("n_discarded", ctypes.c_int32),
        ("n_uncovered", ctypes.c_int32),
        ("n_state_out", ctypes.c_int32),
        ("refine_unconverged", ctypes.c_int32),
        ("refine_step_diff", ctypes.c_int32),
        ("refine_updates", ctypes.c_int64),
        ("refine_gamma_cut", ctypes.c_int32),
        ("step_ms", ctypes.c_double * 2),
        ("step_updates", ctypes.c_int64 * 2),
        ("step_launches", ctypes.c_int32 * 2),
        ("step_pixels", ctypes.c_int64 * 2),
    ]

    def as_dict(self):
        out = {}
        for name, _ in self._fields_:
            if name == "reserved":
                continue
            v = getattr(self, name)
            out[name] = list(v) if hasattr(v, "__len__") else v
        return out


_lib = None


def load(path: str = LIB_PATH):
    """Load libfms.so and declare its signatures.  Raises if it is missing:
    there is no fallback path."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"libfms.so is not built ({path}); run __graft_entry__.build() or "
                           "python paper_2007_14283_amd/build.py")
    lib = ctypes.CDLL(path)
    vp, i32, i64, u64 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64
    lib.fms_default_params.argtypes = [ctypes.POINTER(FmsParams)]
    lib.fms_default_params.restype = None
    lib.fms_create.argtypes = [ctypes.POINTER(vp), i32]
    lib.fms_create.restype = ctypes.c_int
    lib.fms_destroy.argtypes = [vp]
    lib.fms_destroy.restype = ctypes.c_int
    lib.fms_cluster.argtypes = [vp, vp, vp, i64, i64, vp, i32, i32, i32, ctypes.POINTER(FmsParams),
                                vp, vp, i32, ctypes.POINTER(i32), vp, ctypes.POINTER(FmsStats)]
    lib.fms_cluster.restype = ctypes.c_int
    lib.fms_cluster_batch.argtypes = [vp, vp, i32, ctypes.POINTER(FmsFrame), i32, ctypes.POINTER(FmsParams),
                                      vp, vp, i32, ctypes.POINTER(i32), ctypes.POINTER(FmsStats)]
    lib.fms_cluster_batch.restype = ctypes.c_int
    lib.fms_shift_seeds.argtypes = [vp, vp, vp, i64, i64, vp, i32, i32, i32, vp, i32,
                                    ctypes.POINTER(FmsParams), vp, vp, vp, vp, ctypes.POINTER(FmsStats)]
    lib.fms_shift_seeds.restype = ctypes.c_int
    lib.fms_shift_seeds_noalloc.argtypes = lib.fms_shift_seeds.argtypes
    lib.fms_shift_seeds_noalloc.restype = ctypes.c_int
    f64 = ctypes.c_double
    lib.fms_unroll.argtypes = [vp, vp, vp, i64, i64, vp, i32, i32, i32, vp, i32, i32, f64, vp, vp, vp]
    lib.fms_unroll.restype = ctypes.c_int
    lib.fms_unroll_backward.argtypes = [vp, vp, vp, i64, i64, vp, i32, i32, i32, i32, f64, vp, vp, vp, vp, vp]
    lib.fms_unroll_backward.restype = ctypes.c_int
    lib.fms_autotune.argtypes = [vp, vp, ctypes.POINTER(FmsFrame), i32, ctypes.POINTER(FmsParams),
                                 ctypes.POINTER(FmsTuneEntry), i32, ctypes.POINTER(i32), ctypes.POINTER(FmsTuneReport)]
    lib.fms_autotune.restype = ctypes.c_int
    lib.fms_autotune_batch.argtypes = [vp, vp, i32, ctypes.POINTER(FmsFrame), i32, ctypes.POINTER(FmsParams),
                                       ctypes.POINTER(FmsTuneEntry), i32, ctypes.POINTER(i32),
                                       ctypes.POINTER(FmsTuneReport)]
    lib.fms_autotune_batch.restype = ctypes.c_int
    lib.fms_clear_tuning.argtypes = [vp]
    lib.fms_clear_tuning.restype = ctypes.c_int
    lib.fms_seed_order.argtypes = [vp, vp, i32, u64, vp]
    lib.fms_seed_order.restype = ctypes.c_int
    lib.fms_status_string.argtypes = [ctypes.c_int]
    lib.fms_status_string.restype = ctypes.c_char_p
    _lib = lib
    return lib
