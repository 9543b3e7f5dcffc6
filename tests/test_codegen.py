"""Code generation guards of the library's gfx950 kernels (CPU only: hipcc cross-compiles).

Every source under paper_2403_08551_amd/csrc is compiled to gfx950 assembly with the library's
own flags, and every kernel in it is checked for
- no packed FP32 arithmetic: the build turns the packed-fp32 feature off, and hand-written or
  compiler-made packed FP32 instructions have given wrong results on this part;
- no flat memory instructions: a flat access counts against both the vector-memory and the LDS
  wait counters, so an LDS wait after it also waits for memory (the raster forward's chunk
  prefetch had turned into one and every LDS wait of the chunk waited for it);
- no private (scratch) memory (the fine-tuning's per-stage codebook indices, indexed by the
  runtime stage count, are kept in registers by unrolling the stages to their maximum);
- no calls: every device function of a kernel is inlined (a call spills the caller's registers).
"""
import os
import re
import shutil
import subprocess
import sys
import tempfile

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
CSRC = os.path.join(ROOT, "paper_2403_08551_amd", "csrc")
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")

# kernels allowed private memory, with the reason in the module docstring
# the kernels of the hot path, which must exist under these names
HOT = ("k_raster_fit", "k_raster_fwd", "k_raster_bwd", "k_project_hist", "k_chained_scan",
       "k_fused_scatter", "k_adam")


def _flags():
    from paper_2403_08551_amd import build
    return [f for f in build.FLAGS if f not in ("-fPIC", "-shared")] + [
        "--cuda-device-only", "-S", "-I" + os.path.join(ROOT, "include"), "-I" + CSRC]


@pytest.fixture(scope="module")
def kernels():
    if not os.path.exists(HIPCC):
        pytest.skip("hipcc is not installed")
    srcs = sorted(f for f in os.listdir(CSRC) if f.endswith(".hip"))
    tmp = tempfile.mkdtemp()
    try:
        procs = [(s, subprocess.Popen([HIPCC, *_flags(), os.path.join(CSRC, s), "-o",
                                       os.path.join(tmp, s + ".s")],
                                      stdout=subprocess.DEVNULL, stderr=subprocess.PIPE))
                 for s in srcs]
        out = {}
        for s, p in procs:
            _, err = p.communicate(timeout=600)
            assert p.returncode == 0, f"{s}: {err.decode()[-2000:]}"
            asm = open(os.path.join(tmp, s + ".s")).read()
            for m in re.finditer(r"^\s+\.amdhsa_kernel (\S+)$", asm, re.M):
                name = m.group(1)
                start = asm.index(f"\n{name}:") + 1
                end = asm.index(".Lfunc_end", start)
                info = asm.index("; Kernel info:", end)
                scratch = int(re.search(r"; ScratchSize: (\d+)", asm[info:]).group(1))
                out[name] = (s, asm[start:end], scratch)
        return out
    finally:
        shutil.rmtree(tmp, ignore_errors=True)


def _short(name):
    m = re.search(r"(k_[a-z0-9_]+)", name)
    return m.group(1) if m else name


def _instructions(body):
    for line in body.splitlines():
        t = line.split(";")[0].strip()
        if t and not t.startswith(".") and not t.endswith(":"):
            yield t.split()[0]


def test_hot_path_kernels_are_built(kernels):
    names = {_short(k) for k in kernels}
    for k in HOT:
        assert k in names, k


def test_no_packed_fp32_arithmetic(kernels):
    packed = re.compile(r"v_pk_(fma|mul|add)_f32")
    bad = sorted({_short(k) for k, (_, body, _) in kernels.items()
                  if any(packed.match(op) for op in _instructions(body))})
    assert not bad, bad


def test_no_flat_memory_instructions(kernels):
    bad = sorted({_short(k) for k, (_, body, _) in kernels.items()
                  if any(op.startswith("flat_") for op in _instructions(body))})
    assert not bad, bad


def test_no_private_memory(kernels):
    bad = sorted({_short(k) for k, (_, _, scratch) in kernels.items() if scratch})
    assert not bad, bad


def test_no_calls(kernels):
    bad = sorted({_short(k) for k, (_, body, _) in kernels.items()
                  if any(op == "s_swappc_b64" for op in _instructions(body))})
    assert not bad, bad
