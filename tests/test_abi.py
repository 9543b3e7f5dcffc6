"""The C ABI without a GPU: the library loads, exports every symbol that include/gi.h declares,
and rejects bad arguments before touching the device."""
import ctypes
import os
import re

import pytest

from paper_2403_08551_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    src = open(os.path.join(ROOT, "include", "gi.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(gi_[a-z0-9_]+)\s*\(", src)))


def test_header_and_binding_agree():
    assert declared_symbols() == sorted(_lib.EXPORTS)


def test_library_exports_every_declared_symbol():
    L = _lib.lib()
    for name in declared_symbols():
        assert hasattr(L, name), name


def test_status_strings():
    L = _lib.lib()
    assert L.gi_status_string(0) == b"ok"
    assert L.gi_status_string(-1) == b"invalid argument"
    assert L.gi_status_string(12345) == b"unknown status"


def test_null_context_and_bad_sizes_are_rejected_without_a_device():
    L = _lib.lib()
    nul = ctypes.c_void_p(0)
    buf = (ctypes.c_float * 64)()
    img = ctypes.cast(buf, ctypes.c_void_p)
    assert L.gi_render(nul, img, 1, 16, 16, img, nul) == _lib.GI_ERR_INVALID_ARG
    assert L.gi_grad(nul, img, 1, 16, 16, img, img, nul) == _lib.GI_ERR_INVALID_ARG
    assert L.gi_create(None, 0) == _lib.GI_ERR_INVALID_ARG
    assert L.gi_destroy(nul) == _lib.GI_OK
    assert L.gi_set_option(nul, 1, 0) == _lib.GI_ERR_INVALID_ARG
    assert L.gi_reserve(nul, 1, 1, 1) == _lib.GI_ERR_INVALID_ARG
    assert L.gi_fit_graph_launch(nul, 1, nul) == _lib.GI_ERR_INVALID_ARG
    assert L.gi_fit_graph_destroy(nul) == _lib.GI_OK
    assert L.gi_scan_u32(nul, img, img, 4, nul, nul) == _lib.GI_ERR_INVALID_ARG
    assert L.gi_sort_pairs(nul, img, img, img, img, 4, 8, nul) == _lib.GI_ERR_INVALID_ARG
    assert L.gi_last_error(nul) == b""


def test_create_without_gfx950_reports_no_device():
    torch = pytest.importorskip("torch")
    if torch.cuda.is_available():
        pytest.skip("a GPU is visible")
    h = ctypes.c_void_p()
    assert _lib.lib().gi_create(ctypes.byref(h), 0) == _lib.GI_ERR_NO_DEVICE
    assert not h.value


def test_product_path_has_no_cpu_fallback(tmp_path, monkeypatch):
    # with the library path pointing nowhere, the binding raises instead of computing anything
    monkeypatch.setattr(_lib, "_lib", None)
    monkeypatch.setattr(_lib, "LIB_PATH", str(tmp_path / "missing.so"))
    with pytest.raises(RuntimeError, match="missing"):
        _lib.lib()


def test_header_constants_match_the_binding():
    src = open(os.path.join(ROOT, "include", "gi.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    found = dict(re.findall(r"\b(GI_[A-Z0-9_]+)\s*=\s*(-?\d+)", src))
    found.update(re.findall(r"#define\s+(GI_FLAG_[A-Z_]+)\s+(\d+)u", src))
    assert len(found) > 20
    for name, value in found.items():
        if hasattr(_lib, name):
            assert getattr(_lib, name) == int(value), name
    for name in ("GI_OPT_COVARIANCE", "GI_COV_CHOLESKY", "GI_COV_ROTATION_SCALE",
                 "GI_FLAG_SCAN_STALL", "GI_STAGE_UPDATE"):
        assert name in found and hasattr(_lib, name), name


def test_noalloc_render_rejects_bad_sizes_without_a_device():
    L = _lib.lib()
    nul = ctypes.c_void_p(0)
    buf = (ctypes.c_float * 64)()
    p = ctypes.cast(buf, ctypes.c_void_p)
    assert L.gi_render_noalloc(p, 1, 16, 16, nul, nul, nul) == _lib.GI_ERR_INVALID_ARG
    assert L.gi_render_noalloc(nul, 1, 16, 16, p, nul, nul) == _lib.GI_ERR_INVALID_ARG
    assert L.gi_render_noalloc(p, 1, 0, 16, p, nul, nul) == _lib.GI_ERR_INVALID_ARG
    big = _lib.GI_NOALLOC_MAX_GAUSSIANS + 1
    assert L.gi_render_noalloc(p, big, 16, 16, p, nul, nul) == _lib.GI_ERR_CAPACITY
    # 2 x 1025 tiles is two tiles over the limit
    assert L.gi_render_noalloc(p, 1, 32, 16 * 1025, p, nul, nul) == _lib.GI_ERR_CAPACITY
