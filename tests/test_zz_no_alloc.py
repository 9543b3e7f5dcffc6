"""gi_render_noalloc, the render that allocates nothing (every buffer in the library's static
device array), through the C ABI against gi_render: the same kernels, so the images must be
bit-identical, on consecutive calls whose sizes shrink (the array keeps the last call's contents);
the small case also against the FP64 oracle at the forward bar (1e-5 A(p)).  Also: size limits
rejected before anything is enqueued, key overflow reported through the flags word and cleared
for the next call, and an empty set giving a zero image."""
import ctypes

import numpy as np
import pytest

import synth
from oracle import ref

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

FWD_RTOL = 1e-5


def dev(a, dtype=torch.float32):
    return torch.as_tensor(np.ascontiguousarray(a)).to(dtype=dtype, device="cuda")


def run_noalloc(P, pd, h, w):
    img = torch.full((h, w, 3), float("nan"), device="cuda")
    flags = torch.full((1,), -1, dtype=torch.int32, device="cuda")
    P.render_noalloc(pd, h, w, img, flags)
    torch.cuda.synchronize()
    return img, int(flags.item())


def test_noalloc_matches_render_on_consecutive_calls():
    import paper_2403_08551_amd as P
    kodak = synth.kodak_like(70_000)
    small = synth.plain_256()
    cases = [("kodak-768x512-70k", kodak.params(), kodak.height, kodak.width),
             ("plain-256x256-2k", small.params(), small.height, small.width),
             ("ragged-45x70", synth.gaussians(150, 45, 70, seed=2, l_lo=0.5, l_hi=12.0), 45, 70)]
    ctx = P.Context(0)
    try:
        for name, p, h, w in cases:
            print(f"case {name}", flush=True)
            pd = dev(p)
            want = ctx.render(pd, h, w)
            got, flags = run_noalloc(P, pd, h, w)
            assert flags == 0, f"{name}: flags {flags}"
            assert torch.equal(got, want), f"{name}: differs from gi_render"
        # the last (smallest) case against the oracle as well
        o, A = ref.render_culled(p, h, w, with_abs=True)
        g = got.cpu().numpy()
        assert np.all(np.abs(g - o) <= FWD_RTOL * A + 1e-30)
    finally:
        ctx.close()


def test_noalloc_size_limits_enqueue_nothing():
    import paper_2403_08551_amd as P
    L = P._lib.lib()
    img = torch.full((1024, 1024, 3), 7.0, device="cuda")
    p = torch.zeros((P._lib.GI_NOALLOC_MAX_GAUSSIANS + 1, 8), device="cuda")
    st = L.gi_render_noalloc(ctypes.c_void_p(p.data_ptr()), p.shape[0], 64, 64,
                             ctypes.c_void_p(img.data_ptr()), None, None)
    assert st == P._lib.GI_ERR_CAPACITY
    # 64 x 64 tiles = 4096 > 2048
    st = L.gi_render_noalloc(ctypes.c_void_p(p.data_ptr()), 10, 1024, 1024,
                             ctypes.c_void_p(img.data_ptr()), None, None)
    assert st == P._lib.GI_ERR_CAPACITY
    st = L.gi_render_noalloc(ctypes.c_void_p(p.data_ptr()), 10, 64, 64, None, None, None)
    assert st == P._lib.GI_ERR_INVALID_ARG
    torch.cuda.synchronize()
    assert bool((img == 7.0).all())


def test_noalloc_overflow_is_flagged_then_cleared():
    import paper_2403_08551_amd as P
    h = w = 256
    rng = np.random.default_rng(5)
    n = 20_000
    # every Gaussian covers all 256 tiles: 5.1M keys, more than the array holds
    big = np.zeros((n, 8), np.float32)
    big[:, 0:2] = rng.uniform(100, 156, (n, 2))
    big[:, 2] = 150.0
    big[:, 4] = 150.0
    big[:, 5:8] = rng.uniform(0, 1, (n, 3))
    _, flags = run_noalloc(P, dev(big), h, w)
    assert flags & P._lib.GI_FLAG_KEY_OVERFLOW
    small = synth.plain_256()
    pd = dev(small.params())
    got, flags = run_noalloc(P, pd, h, w)
    assert flags == 0
    ctx = P.Context(0)
    try:
        assert torch.equal(got, ctx.render(pd, h, w))
    finally:
        ctx.close()


def test_noalloc_empty_set_and_nonfinite_flag():
    import paper_2403_08551_amd as P
    img, flags = run_noalloc(P, torch.zeros((0, 8), device="cuda"), 33, 17)
    assert flags == 0
    assert bool((img == 0).all())
    p = synth.gaussians(40, 40, 40, seed=9)
    p[3] = [np.nan, 1, 1, 0, 1, 1, 1, 1]
    pd = dev(p)
    got, flags = run_noalloc(P, pd, 40, 40)
    assert flags == P._lib.GI_FLAG_NONFINITE
    ctx = P.Context(0)
    try:
        assert torch.equal(got, ctx.render(pd, 40, 40))
    finally:
        ctx.close()


def test_noalloc_render_replays_from_a_captured_graph():
    # the call recorded into a HIP graph (kernel nodes only) and replayed four times, with other
    # renders (through gi_render, and no-allocation renders of another size that overwrite the
    # shared array) and host waits between the replays: every replay equals the eager image
    import paper_2403_08551_amd as P
    w = synth.kodak_like(30_000)
    h, wd = w.height, w.width
    pd = dev(w.params())
    want, flags = run_noalloc(P, pd, h, wd)
    assert flags == 0
    other = synth.plain_256()
    po = dev(other.params())
    img = torch.full((h, wd, 3), float("nan"), device="cuda")
    fl = torch.full((1,), -1, dtype=torch.int32, device="cuda")
    g = torch.cuda.CUDAGraph()
    side = torch.cuda.Stream()
    side.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(side):
        with torch.cuda.graph(g, stream=side):
            P.render_noalloc(pd, h, wd, img, fl)
    torch.cuda.current_stream().wait_stream(side)
    ctx = P.Context(0)
    try:
        for i in range(4):
            img.fill_(float("nan"))
            fl.fill_(-1)
            g.replay()
            torch.cuda.synchronize()
            assert int(fl.item()) == 0, f"replay {i}: flags {int(fl.item())}"
            assert torch.equal(img, want), f"replay {i} differs from the eager image"
            ctx.render(po, other.height, other.width)
            small, f2 = run_noalloc(P, po, other.height, other.width)
            assert f2 == 0
    finally:
        ctx.close()
        del g
