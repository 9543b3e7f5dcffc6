"""ctypes declarations of the C ABI in include/gi.h (libgi.so, built in place).

There is no fallback: if the library is missing or does not load, every call raises.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
# GI_LIB: load another build of the library (for example one with host-side sanitizers)
LIB_PATH = os.environ.get("GI_LIB") or os.path.join(HERE, "libgi.so")

GI_OK = 0
GI_ERR_INVALID_ARG = -1
GI_ERR_CAPACITY = -2
GI_ERR_HIP = -3
GI_ERR_NONFINITE = -4
GI_ERR_UNSUPPORTED = -5
GI_ERR_NO_DEVICE = -6

GI_FLAG_KEY_OVERFLOW = 1
GI_FLAG_NONFINITE = 2
GI_FLAG_SCAN_STALL = 4
GI_FLAG_BAD_CODE = 8

GI_OPT_SYNC = 1
GI_OPT_SORT_BITS = 2
GI_OPT_FWD_PIXELS = 3
GI_OPT_BINNING = 4
GI_OPT_TIMING = 5
GI_OPT_TILE_ORDER = 7
GI_OPT_FIT_WAVES = 8
GI_OPT_COVARIANCE = 6

GI_BLEND_SUM = 1
GI_BLEND_ALPHA = 2

GI_COV_CHOLESKY = 0
GI_COV_ROTATION_SCALE = 1

GI_STAGE_BINNING = 0
GI_STAGE_RASTER_FWD = 1
GI_STAGE_RASTER_BWD = 2
GI_STAGE_RASTER_FIT = 3
GI_STAGE_UPDATE = 4

# limits of gi_render_noalloc (include/gi.h)
GI_NOALLOC_SCRATCH_BYTES = 64 << 20
GI_NOALLOC_MAX_GAUSSIANS = 1 << 18
GI_NOALLOC_MAX_TILES = 2048

# every symbol that include/gi.h declares
EXPORTS = (
    "gi_create", "gi_destroy", "gi_set_option", "gi_reserve", "gi_query", "gi_status_string",
    "gi_last_error", "gi_render", "gi_grad", "gi_fit_step", "gi_render_batched",
    "gi_grad_batched", "gi_fit_step_batched", "gi_fit_graph_create", "gi_fit_graph_launch",
    "gi_fit_graph_destroy", "gi_binning", "gi_scan_u32", "gi_sort_pairs", "gi_timing",
    "gi_get_option", "gi_autotune", "gi_fit_graph_query", "gi_codec_decode", "gi_render_codec",
    "gi_render_opacity", "gi_grad_opacity", "gi_fit_step_opacity", "gi_fit_step_recipe",
    "gi_recipe_params", "gi_qat_init", "gi_fit_step_qat", "gi_qat_encode",
    "gi_fit_graph_create_recipe", "gi_fit_graph_create_qat", "gi_render_noalloc",
    "gi_autotune_save", "gi_autotune_load",
)


class gi_adam(ctypes.Structure):
    _fields_ = [("lr_mu", ctypes.c_float), ("lr_l", ctypes.c_float), ("lr_c", ctypes.c_float),
                ("beta1", ctypes.c_float), ("beta2", ctypes.c_float), ("eps", ctypes.c_float),
                ("l_min", ctypes.c_float)]


class gi_schedule(ctypes.Structure):
    _fields_ = [("binning", ctypes.c_int32), ("fwd_pixels", ctypes.c_int32),
                ("sort_bits", ctypes.c_int32), ("tile_order", ctypes.c_int32),
                ("fit_waves", ctypes.c_int32), ("ms_per_step", ctypes.c_float)]


class gi_batch(ctypes.Structure):
    _fields_ = [("count", ctypes.c_int32),
                ("height_host", ctypes.POINTER(ctypes.c_int32)),
                ("width_host", ctypes.POINTER(ctypes.c_int32)),
                ("gauss_off_host", ctypes.POINTER(ctypes.c_int64))]


class gi_adan(ctypes.Structure):
    _fields_ = [("lr", ctypes.c_float), ("beta1", ctypes.c_float), ("beta2", ctypes.c_float),
                ("beta3", ctypes.c_float), ("eps", ctypes.c_float),
                ("weight_decay", ctypes.c_float), ("halve_every", ctypes.c_int32)]


class gi_qat(ctypes.Structure):
    _fields_ = [("quant_dev", ctypes.c_void_p), ("quant_m_dev", ctypes.c_void_p),
                ("quant_v_dev", ctypes.c_void_p), ("bits", ctypes.c_int32),
                ("stages", ctypes.c_int32), ("codebook_size", ctypes.c_int32),
                ("lambda_", ctypes.c_float), ("lr_q", ctypes.c_float),
                ("ema_dev", ctypes.c_void_p), ("decay", ctypes.c_float)]


class gi_codec(ctypes.Structure):
    _fields_ = [("mu_dev", ctypes.c_void_p), ("codes_dev", ctypes.c_void_p),
                ("index_dev", ctypes.c_void_p), ("codebook_dev", ctypes.c_void_p),
                ("gamma", ctypes.c_float * 3), ("beta", ctypes.c_float * 3),
                ("bits", ctypes.c_int32), ("stages", ctypes.c_int32),
                ("codebook_size", ctypes.c_int32)]


class GiError(RuntimeError):
    def __init__(self, status: int, what: str, detail: str = ""):
        self.status = status
        msg = f"{what}: {status_string(status)} ({status})"
        if detail:
            msg += f": {detail}"
        super().__init__(msg)


_lib = None

P = ctypes.c_void_p
I64 = ctypes.c_int64
I32 = ctypes.c_int32


def lib():
    """Load libgi.so; raises when it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                               "`python paper_2403_08551_amd/build.py` (hipcc, gfx950)")
        L = ctypes.CDLL(LIB_PATH)
        sig = {
            "gi_create": ([ctypes.POINTER(P), ctypes.c_int], ctypes.c_int),
            "gi_destroy": ([P], ctypes.c_int),
            "gi_set_option": ([P, ctypes.c_int, I64], ctypes.c_int),
            "gi_reserve": ([P, I64, I64, I64], ctypes.c_int),
            "gi_query": ([P, ctypes.POINTER(I64), ctypes.POINTER(ctypes.c_uint32), ctypes.c_int],
                         ctypes.c_int),
            "gi_status_string": ([ctypes.c_int], ctypes.c_char_p),
            "gi_last_error": ([P], ctypes.c_char_p),
            "gi_render": ([P, P, I64, I32, I32, P, P], ctypes.c_int),
            "gi_render_noalloc": ([P, I64, I32, I32, P, P, P], ctypes.c_int),
            "gi_grad": ([P, P, I64, I32, I32, P, P, P], ctypes.c_int),
            "gi_fit_step": ([P, P, P, P, P, I64, I32, I32, ctypes.POINTER(gi_adam), P, P, P, P],
                            ctypes.c_int),
            "gi_render_batched": ([P, P, ctypes.POINTER(gi_batch), P, P], ctypes.c_int),
            "gi_grad_batched": ([P, P, ctypes.POINTER(gi_batch), P, P, P], ctypes.c_int),
            "gi_fit_step_batched": ([P, P, P, P, P, ctypes.POINTER(gi_batch),
                                     ctypes.POINTER(gi_adam), P, P, P, P], ctypes.c_int),
            "gi_fit_graph_create": ([P, P, P, P, P, I64, I32, I32, ctypes.POINTER(gi_batch),
                                     ctypes.POINTER(gi_adam), P, P, P, P, ctypes.POINTER(P)],
                                    ctypes.c_int),
            "gi_fit_graph_launch": ([P, I32, P], ctypes.c_int),
            "gi_fit_graph_destroy": ([P], ctypes.c_int),
            "gi_fit_graph_query": ([P, ctypes.POINTER(I64), ctypes.POINTER(ctypes.c_uint32),
                                    ctypes.c_int], ctypes.c_int),
            "gi_binning": ([P, P, I64, I32, I32, P, P, P, P, P, I64, ctypes.POINTER(I64), P],
                           ctypes.c_int),
            "gi_scan_u32": ([P, P, P, I64, P, P], ctypes.c_int),
            "gi_sort_pairs": ([P, P, P, P, P, I64, I32, P], ctypes.c_int),
            "gi_get_option": ([P, ctypes.c_int, ctypes.POINTER(I64)], ctypes.c_int),
            "gi_autotune": ([P, P, P, I64, I32, I32, ctypes.POINTER(gi_batch), I32, P,
                             ctypes.POINTER(gi_schedule)], ctypes.c_int),
            "gi_autotune_save": ([P, ctypes.c_char_p], ctypes.c_int),
            "gi_autotune_load": ([P, ctypes.c_char_p, ctypes.POINTER(I32)], ctypes.c_int),
            "gi_fit_step_opacity": ([P, P, P, P, P, P, P, P, I64, I32, I32, I32,
                                     ctypes.POINTER(gi_adam), P, P, P, P], ctypes.c_int),
            "gi_fit_step_recipe": ([P, P, P, P, I64, I32, I32, ctypes.POINTER(gi_adan), P, P, P,
                                    P], ctypes.c_int),
            "gi_recipe_params": ([P, P, I64, I32, I32, P, P], ctypes.c_int),
            "gi_qat_init": ([P, P, I64, ctypes.POINTER(gi_qat), I32, P], ctypes.c_int),
            "gi_fit_step_qat": ([P, P, P, P, P, I64, I32, I32, ctypes.POINTER(gi_adam),
                                 ctypes.POINTER(gi_qat), P, P, P, P], ctypes.c_int),
            "gi_qat_encode": ([P, P, I64, ctypes.POINTER(gi_qat), P, P, P, P], ctypes.c_int),
            "gi_fit_graph_create_recipe": ([P, P, P, P, I64, I32, I32, ctypes.POINTER(gi_adan),
                                            P, P, P, P, ctypes.POINTER(P)], ctypes.c_int),
            "gi_fit_graph_create_qat": ([P, P, P, P, P, I64, I32, I32, ctypes.POINTER(gi_adam),
                                         ctypes.POINTER(gi_qat), P, P, P, P, ctypes.POINTER(P)],
                                        ctypes.c_int),
            "gi_render_opacity": ([P, P, P, I64, I32, I32, I32, P, P], ctypes.c_int),
            "gi_grad_opacity": ([P, P, P, I64, I32, I32, I32, P, P, P, P], ctypes.c_int),
            "gi_codec_decode": ([P, ctypes.POINTER(gi_codec), I64, P, P], ctypes.c_int),
            "gi_render_codec": ([P, ctypes.POINTER(gi_codec), I64, I32, I32, P, P], ctypes.c_int),
            "gi_timing": ([P, ctypes.c_int, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(I64),
                           ctypes.c_int], ctypes.c_int),
        }
        for name, (args, res) in sig.items():
            fn = getattr(L, name)
            fn.argtypes = args
            fn.restype = res
        _lib = L
    return _lib


def status_string(status: int) -> str:
    try:
        return lib().gi_status_string(status).decode()
    except Exception:  # library missing: plain text
        return str(status)
