"""ctypes loader for the C/OpenMP FP64 oracle in ``cpu_ref.c``.

TEST INFRASTRUCTURE: see the package docstring.  ``build()`` compiles the library in place with
gcc; ``lib()`` loads it, building first when it is missing.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "cpu_ref.c")
# GI_ORACLE_SO: load another build of the same source (the sanitizer test's instrumented one)
SO = os.environ.get("GI_ORACLE_SO") or os.path.join(HERE, "liboracle_cpu.so")

_P = ctypes.c_void_p
_I64 = ctypes.c_int64
_I32 = ctypes.c_int32
_lib = None


def build() -> str:
    """Compile ``cpu_ref.c`` into ``liboracle_cpu.so`` (float64, OpenMP, no FP contraction)."""
    tmp = SO + f".tmp{os.getpid()}"
    subprocess.run(["gcc", "-O3", "-march=x86-64-v3", "-ffp-contract=off", "-fopenmp", "-shared",
                    "-fPIC", SRC, "-lm", "-o", tmp], check=True)
    os.replace(tmp, SO)
    return SO


def lib():
    global _lib
    if _lib is None:
        if not os.environ.get("GI_ORACLE_SO") and (not os.path.exists(SO) or
                                                   os.path.getmtime(SO) < os.path.getmtime(SRC)):
            build()
        L = ctypes.CDLL(SO)
        L.or_tile_rects.argtypes = [_P, _I64, _I32, _I32, _P, _P]
        L.or_tile_rects.restype = _I64
        L.or_tile_lists.argtypes = [_P, _I64, _I32, _I32, _P, _P, _I64]
        L.or_tile_lists.restype = _I64
        L.or_render_culled.argtypes = [_P, _I64, _I32, _I32, _P, _P]
        L.or_render_pixels.argtypes = [_P, _I64, _I32, _I32, _P, _I64, _P, _P]
        L.or_grads_culled.argtypes = [_P, _I64, _I32, _I32, _P, _P, _P]
        L.or_grads_subset.argtypes = [_P, _I64, _I32, _I32, _P, _P, _I64, _P, _P]
        L.or_fit_step.argtypes = [_P, _P, _P, _P, _P, _I64, _I32, _I32, _P, _I64, _P]
        L.or_fit_step.restype = ctypes.c_double
        L.or_num_threads.restype = ctypes.c_int
        _lib = L
    return _lib


def _ptr(a):
    return a.ctypes.data_as(_P) if a is not None else None


def _f32(a):
    return np.ascontiguousarray(a, dtype=np.float32)


def tile_rects(params, height, width):
    p = _f32(params).reshape(-1, 8)
    rect = np.zeros((p.shape[0], 4), np.int64)
    count = np.zeros(p.shape[0], np.int64)
    lib().or_tile_rects(_ptr(p), p.shape[0], height, width, _ptr(rect), _ptr(count))
    return rect, count


def tile_lists(params, height, width):
    p = _f32(params).reshape(-1, 8)
    t = (-(-width // 16)) * (-(-height // 16))
    ranges = np.zeros((t, 2), np.int64)
    K = lib().or_tile_lists(_ptr(p), p.shape[0], height, width, _ptr(ranges), None, 0)
    ids = np.zeros(max(K, 1), np.int64)
    lib().or_tile_lists(_ptr(p), p.shape[0], height, width, _ptr(ranges), _ptr(ids), K)
    return ranges, ids[:K]


def render_culled(params, height, width, with_abs=False):
    p = _f32(params).reshape(-1, 8)
    img = np.zeros((height, width, 3))
    aimg = np.zeros((height, width, 3)) if with_abs else None
    lib().or_render_culled(_ptr(p), p.shape[0], height, width, _ptr(img), _ptr(aimg))
    return (img, aimg) if with_abs else img


def render_pixels(params, height, width, pix, with_abs=False):
    """Selected pixels (linear indices y * W + x); returns float64 [m, 3] (and |.| sums)."""
    p = _f32(params).reshape(-1, 8)
    pix = np.ascontiguousarray(pix, np.int64)
    out = np.zeros((pix.size, 3))
    aout = np.zeros((pix.size, 3)) if with_abs else None
    lib().or_render_pixels(_ptr(p), p.shape[0], height, width, _ptr(pix), pix.size, _ptr(out),
                           _ptr(aout))
    return (out, aout) if with_abs else out


def grads(params, height, width, dl_dimage, with_abs=False):
    p = _f32(params).reshape(-1, 8)
    G = _f32(dl_dimage)
    d = np.zeros((p.shape[0], 8))
    ad = np.zeros((p.shape[0], 8)) if with_abs else None
    lib().or_grads_culled(_ptr(p), p.shape[0], height, width, _ptr(G), _ptr(d), _ptr(ad))
    return (d, ad) if with_abs else d


def grads_subset(params, height, width, dl_dimage, which, with_abs=False):
    p = _f32(params).reshape(-1, 8)
    G = _f32(dl_dimage)
    which = np.ascontiguousarray(which, np.int64)
    d = np.zeros((which.size, 8))
    ad = np.zeros((which.size, 8)) if with_abs else None
    lib().or_grads_subset(_ptr(p), p.shape[0], height, width, _ptr(G), _ptr(which), which.size,
                          _ptr(d), _ptr(ad))
    return (d, ad) if with_abs else d


def fit_step(params, m, v, target, step, hp, want_image=False):
    """One FP64 fit step from float32 params; returns (params64, m, v, loss[, image])."""
    p = _f32(params).reshape(-1, 8)
    n = p.shape[0]
    h, w = target.shape[0], target.shape[1]
    out = np.zeros((n, 8))
    m = np.array(m, np.float64).reshape(n, 8)
    v = np.array(v, np.float64).reshape(n, 8)
    hpv = np.array([hp["lr_mu"], hp["lr_l"], hp["lr_c"], hp["beta1"], hp["beta2"], hp["eps"],
                    hp["l_min"]], np.float64)
    img = np.zeros((h, w, 3)) if want_image else None
    T = _f32(target)
    loss = lib().or_fit_step(_ptr(p), _ptr(out), _ptr(m), _ptr(v), _ptr(T), n, h, w, _ptr(hpv),
                             step, _ptr(img))
    if want_image:
        return out, m, v, loss, img
    return out, m, v, loss


def num_threads() -> int:
    return int(lib().or_num_threads())
