"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only; no GPU code is
instrumented).

* The FP64 C oracle (`oracle/cpu_ref.c`) built with -fsanitize=address,undefined runs its whole
  interface on small ragged cases (Gaussians off the image, degenerate and non-finite records,
  one-pixel and empty images) in a child process; any report ends it with an error, and its
  results must equal the plain build's bit for bit.
* The library's host code (`libgi.so` with the sanitizers on the host side only) runs the C ABI's
  argument checks, which need no device, in a child process.
"""
import os
import subprocess
import sys

import numpy as np
import pytest

import synth
from oracle import cref

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _runtime(name):
    p = subprocess.run(["gcc", f"-print-file-name={name}"], capture_output=True, text=True)
    path = p.stdout.strip()
    return path if os.path.isabs(path) and os.path.exists(path) else None


def cases():
    out = []
    p = synth.gaussians(150, 45, 70, seed=2, l_lo=0.5, l_hi=12.0)
    p[:4, 0] = [-30.0, 200.0, 35.0, 0.0]
    p[4] = [np.nan, 1, 1, 0, 1, 1, 1, 1]
    p[5, 2] = 0.0
    out.append((p, 45, 70))
    out.append((synth.gaussians(5, 1, 1, seed=3), 1, 1))
    out.append((np.zeros((0, 8), np.float32), 17, 33))
    out.append((synth.gaussians(300, 64, 48, seed=4, l_lo=0.5, l_hi=32.0), 64, 48))
    return out


CHILD = r'''
import sys, numpy as np
sys.path.insert(0, ROOT)
import test_sanitizers as T
from oracle import cref, ref
res = {}
for k, (p, h, w) in enumerate(T.cases()):
    res[f"rects{k}"], res[f"counts{k}"] = cref.tile_rects(p, h, w)[:2]
    img, A = cref.render_culled(p, h, w, with_abs=True)
    res[f"img{k}"], res[f"A{k}"] = img, A
    G = np.random.default_rng(k).uniform(-1, 1, (h, w, 3))
    g, Ag = cref.grads(p, h, w, G, with_abs=True)
    res[f"g{k}"], res[f"Ag{k}"] = g, Ag
    if p.shape[0]:
        z = np.zeros((p.shape[0], 8))
        q = cref.fit_step(np.nan_to_num(p), z, z, np.full((h, w, 3), 0.5), 1, dict(ref.DEFAULT_ADAM))
        res[f"fit{k}"] = np.asarray(q[0] if isinstance(q, tuple) else q, dtype=np.float64)
np.savez(OUT, **{k: np.asarray(v) for k, v in res.items()})
'''


def _oracle_results(env, out):
    code = CHILD.replace("ROOT", repr(ROOT)).replace("OUT", repr(out))
    r = subprocess.run([sys.executable, "-c", code], env=env, capture_output=True, text=True,
                       cwd=os.path.join(ROOT, "tests"), timeout=600)
    assert r.returncode == 0, r.stderr[-3000:]
    assert "ERROR: AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr, \
        r.stderr[-3000:]
    return dict(np.load(out))


def test_oracle_under_address_and_undefined_behaviour_sanitizers(tmp_path):
    asan, ubsan = _runtime("libasan.so"), _runtime("libubsan.so")
    if not asan or not ubsan:
        pytest.skip("gcc sanitizer runtimes not installed")
    so = str(tmp_path / "liboracle_cpu_san.so")
    subprocess.run(["gcc", "-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
                    "-fno-sanitize-recover=undefined", "-ffp-contract=off", "-fopenmp", "-shared",
                    "-fPIC", cref.SRC, "-lm", "-o", so], check=True)
    base = dict(os.environ, OMP_NUM_THREADS="2")
    plain = _oracle_results(base, str(tmp_path / "plain.npz"))
    env = dict(base, GI_ORACLE_SO=so, LD_PRELOAD=f"{asan} {ubsan}",
               ASAN_OPTIONS="detect_leaks=0:halt_on_error=1:abort_on_error=0",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    san = _oracle_results(env, str(tmp_path / "san.npz"))
    assert sorted(san) == sorted(plain)
    for k in plain:
        np.testing.assert_array_equal(san[k], plain[k], err_msg=k)


ABI_CHILD = r'''
import ctypes, sys
sys.path.insert(0, ROOT)
from paper_2403_08551_amd import _lib
L = _lib.lib()
nul = ctypes.c_void_p(0)
buf = (ctypes.c_float * 64)()
p = ctypes.cast(buf, ctypes.c_void_p)
checks = [
    L.gi_render(nul, p, 1, 16, 16, p, nul) == _lib.GI_ERR_INVALID_ARG,
    L.gi_grad(nul, p, 1, 16, 16, p, p, nul) == _lib.GI_ERR_INVALID_ARG,
    L.gi_render_noalloc(p, 1, 16, 16, nul, nul, nul) == _lib.GI_ERR_INVALID_ARG,
    L.gi_render_noalloc(p, _lib.GI_NOALLOC_MAX_GAUSSIANS + 1, 16, 16, p, nul, nul) == _lib.GI_ERR_CAPACITY,
    L.gi_render_noalloc(p, 1, 32, 16 * 1025, p, nul, nul) == _lib.GI_ERR_CAPACITY,
    L.gi_autotune_save(nul, b"/nonexistent/x") == _lib.GI_ERR_INVALID_ARG,
    L.gi_autotune_load(nul, b"/nonexistent/x", None) == _lib.GI_ERR_INVALID_ARG,
    L.gi_fit_graph_launch(nul, 1, nul) == _lib.GI_ERR_INVALID_ARG,
    L.gi_fit_graph_destroy(nul) == _lib.GI_OK,
    L.gi_scan_u32(nul, p, p, 4, nul, nul) == _lib.GI_ERR_INVALID_ARG,
    L.gi_status_string(-3) == b"HIP runtime error",
]
print("checks", checks)
sys.exit(0 if all(checks) else 3)
'''


def test_library_host_code_under_address_sanitizer(tmp_path):
    clang_rt = None
    base = "/opt/rocm/llvm/lib/clang"
    if os.path.isdir(base):
        for v in sorted(os.listdir(base)):
            c = os.path.join(base, v, "lib", "linux", "libclang_rt.asan-x86_64.so")
            if os.path.exists(c):
                clang_rt = c
    if not clang_rt:
        pytest.skip("clang AddressSanitizer runtime not installed")
    src = os.path.join(ROOT, "paper_2403_08551_amd", "csrc")
    srcs = sorted(os.path.join(src, f) for f in os.listdir(src) if f.endswith(".hip"))
    so = str(tmp_path / "libgi_hostsan.so")
    subprocess.run(["/opt/rocm/bin/hipcc", "-O1", "-g", "-std=c++17", "--offload-arch=gfx950",
                    "-fPIC", "-shared", "-Xclang", "-target-feature", "-Xclang",
                    "-packed-fp32-ops", "-Xarch_host", "-fsanitize=address",
                    "-Xarch_host", "-fno-omit-frame-pointer", *srcs, "-o", so],
                   check=True, capture_output=True)
    env = dict(os.environ, GI_LIB=so, LD_PRELOAD=clang_rt,
               ASAN_OPTIONS="detect_leaks=0:halt_on_error=1")
    r = subprocess.run([sys.executable, "-c", ABI_CHILD.replace("ROOT", repr(ROOT))], env=env,
                       capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, (r.stdout + r.stderr)[-3000:]
    assert "AddressSanitizer" not in r.stderr, r.stderr[-3000:]
