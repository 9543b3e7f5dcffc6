"""Parity of the HIP path (through the C ABI) with the FP64 oracle.

Bars: tile rects, counts, offsets, key counts, tile ranges and per-tile id lists bit-exact;
forward |gpu - oracle| <= 1e-5 A(p) + 1e-30 with A(p) = sum |c'| exp(-sigma) over the same
support; gradients |gpu - oracle| <= 1e-4 A_theta + 1e-30 with A_theta the sum of absolute
per-pixel contributions; fit steps as stated in their tests.
"""
import math

import numpy as np
import pytest

import parity_util as pu
import synth
from oracle import cref, ref

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

FWD_RTOL = 1e-5
GRAD_RTOL = 1e-4


@pytest.fixture(scope="module")
def gi():
    import paper_2403_08551_amd as P
    ctx = P.Context(0)
    yield ctx
    ctx.close()


def dev(a, dtype=torch.float32):
    return torch.as_tensor(np.ascontiguousarray(a)).to(dtype=dtype, device="cuda")


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def ragged_case():
    h, w = 45, 70
    p = synth.gaussians(150, h, w, seed=2, l_lo=0.5, l_hi=12.0)
    p[:4, 0] = [-30.0, 200.0, 35.0, 0.0]
    p[:4, 1] = [10.0, 10.0, -40.0, 0.0]
    p[4] = [np.nan, 1, 1, 0, 1, 1, 1, 1]
    p[5, 2] = 0.0
    p[6, 5:8] = [-2.0, 3.0, -0.5]
    return p, h, w


def cases():
    out = {}
    w = synth.plain_256()
    out["plain-256x256-2k"] = (w.params(), w.height, w.width)
    out["ragged-45x70"] = ragged_case()
    out["one-pixel"] = (synth.gaussians(5, 1, 1, seed=3), 1, 1)
    out["empty"] = (np.zeros((0, 8), np.float32), 33, 17)
    out["wide-l-100x120"] = (synth.gaussians(400, 100, 120, seed=8, l_lo=0.5, l_hi=32.0), 100, 120)
    out["off-image"] = (synth.gaussians(50, 40, 40, seed=9) + np.array([500, 500, 0, 0, 0, 0, 0, 0],
                                                                         np.float32), 40, 40)
    return out


CASES = cases()


def assert_forward(g, o, A, what):
    bad = np.abs(g - o) > FWD_RTOL * A + 1e-30
    if bad.any():
        i = np.argmax(np.abs(g - o) / (A + 1e-300))
        raise AssertionError(f"{what}: {bad.sum()} values off; worst gpu {g.flat[i]} oracle "
                             f"{o.flat[i]} A {A.flat[i]}")


def assert_grads(g, o, A, what):
    bad = np.abs(g - o) > GRAD_RTOL * A + 1e-30
    if bad.any():
        i = np.argmax(np.abs(g - o) / (A + 1e-300))
        raise AssertionError(f"{what}: {bad.sum()} values off; worst gpu {g.flat[i]} oracle "
                             f"{o.flat[i]} A {A.flat[i]} at {np.unravel_index(i, g.shape)}")


# ------------------------------------------------------------------ binning (bit-exact)

@pytest.fixture(params=[1, 2, 3], ids=["radix", "one-pass", "rows"])
def mode(request, gi):
    import paper_2403_08551_amd as P
    gi.set_option(P._lib.GI_OPT_BINNING, request.param)
    yield request.param
    gi.set_option(P._lib.GI_OPT_BINNING, 0)


@pytest.mark.parametrize("name", list(CASES))
def test_binning_bit_exact(gi, name, mode):
    p, h, w = CASES[name]
    b = gi.binning(dev(p), h, w)
    rect, count = ref.tile_rects(p, h, w)
    ranges, ids = ref.tile_lists(p, h, w)
    if p.shape[0]:
        np.testing.assert_array_equal(host(b["rects"]), rect)
        np.testing.assert_array_equal(host(b["counts"]), count)
        np.testing.assert_array_equal(host(b["offsets"]), np.concatenate([[0], np.cumsum(count)[:-1]]))
    assert b["keys"] == int(count.sum())
    np.testing.assert_array_equal(host(b["ranges"]), ranges)
    np.testing.assert_array_equal(host(b["ids"]), ids)


@pytest.mark.parametrize("bits", [1, 3, 5, 8, 11])
def test_binning_independent_of_digit_width(gi, bits):
    import paper_2403_08551_amd as P
    p, h, w = CASES["wide-l-100x120"]
    ranges, ids = ref.tile_lists(p, h, w)
    gi.set_option(P._lib.GI_OPT_SORT_BITS, bits)
    gi.set_option(P._lib.GI_OPT_BINNING, 1)
    try:
        b = gi.binning(dev(p), h, w)
    finally:
        gi.set_option(P._lib.GI_OPT_SORT_BITS, 0)
        gi.set_option(P._lib.GI_OPT_BINNING, 0)
    np.testing.assert_array_equal(host(b["ranges"]), ranges)
    np.testing.assert_array_equal(host(b["ids"]), ids)


def test_binning_paths_give_identical_results(gi):
    # the one-pass counting sort, the row binning and the radix sort produce the same tile
    # order, so renders, gradients and fit steps agree bit for bit
    import paper_2403_08551_amd as P
    w = synth.plain_256()
    p0, T = w.params(), dev(w.target())
    G = dev(synth.upstream_gradient(w.height, w.width, 9))
    out = {}
    for m in (1, 2, 3):
        gi.set_option(P._lib.GI_OPT_BINNING, m)
        try:
            p = dev(p0)
            img = host(gi.render(p, w.height, w.width))
            d = host(gi.grad(p, w.height, w.width, G))
            mm, vv = torch.zeros_like(p), torch.zeros_like(p)
            st = torch.ones(1, dtype=torch.int32, device="cuda")
            for _ in range(3):
                gi.fit_step(p, mm, vv, T, st)
            out[m] = (img, d, host(p))
        finally:
            gi.set_option(P._lib.GI_OPT_BINNING, 0)
    for m in (2, 3):
        for a, b in zip(out[1], out[m]):
            np.testing.assert_array_equal(a, b)


# ------------------------------------------------------------------ sort and scan primitives

@pytest.mark.parametrize("n,bits", [(1, 1), (100, 4), (4096, 8), (4097, 11), (70001, 13),
                                    (300000, 21), (123457, 32)])
def test_sort_pairs_is_a_stable_sort(gi, n, bits):
    rng = np.random.default_rng(n + bits)
    keys = rng.integers(0, 2 ** 32, n, dtype=np.uint64).astype(np.uint32)
    keys_masked = keys & np.uint32((1 << bits) - 1) if bits < 32 else keys
    if bits >= 4:  # many equal keys, to exercise stability
        keys[::3] = keys[0]
        keys_masked = keys & np.uint32((1 << bits) - 1) if bits < 32 else keys
    vals = np.arange(n, dtype=np.uint32)
    ko, vo = gi.sort_pairs(dev(keys.view(np.int32), torch.int32), dev(vals.view(np.int32), torch.int32), bits)
    order = np.argsort(keys_masked, kind="stable")
    np.testing.assert_array_equal(host(vo).view(np.uint32), vals[order])
    np.testing.assert_array_equal(host(ko).view(np.uint32), keys[order])


@pytest.mark.parametrize("n", [1, 17, 16384, 16385, 65536, 65537, 1 << 20])
def test_scan_u32(gi, n):
    x = np.random.default_rng(n).integers(0, 1000, n).astype(np.int32)
    out, total = gi.scan_u32(dev(x, torch.int32))
    want = np.concatenate([[0], np.cumsum(x.astype(np.int64))[:-1]])
    np.testing.assert_array_equal(host(out).astype(np.int64), want)
    assert int(host(total)[0]) == int(x.astype(np.int64).sum())


# ------------------------------------------------------------------ forward

@pytest.mark.parametrize("name", list(CASES))
def test_render_matches_oracle(gi, name, mode):
    p, h, w = CASES[name]
    img = host(gi.render(dev(p), h, w))
    o, A = ref.render_culled(p, h, w, with_abs=True)
    assert_forward(img, o, A, name)


def test_render_is_deterministic_and_independent_of_pixels_per_lane(gi):
    import paper_2403_08551_amd as P
    p, h, w = CASES["plain-256x256-2k"]
    pd = dev(p)
    base = host(gi.render(pd, h, w))
    np.testing.assert_array_equal(host(gi.render(pd, h, w)), base)
    for px in (1, 2, 4):
        gi.set_option(P._lib.GI_OPT_FWD_PIXELS, px)
        try:
            np.testing.assert_array_equal(host(gi.render(pd, h, w)), base)
        finally:
            gi.set_option(P._lib.GI_OPT_FWD_PIXELS, 0)


def test_render_is_permutation_invariant(gi):
    p, h, w = CASES["plain-256x256-2k"]
    perm = np.random.default_rng(0).permutation(p.shape[0])
    a = host(gi.render(dev(p), h, w))
    b = host(gi.render(dev(p[perm]), h, w))
    _, A = ref.render_culled(p, h, w, with_abs=True)
    assert np.all(np.abs(a - b) <= 2 * FWD_RTOL * A + 1e-30)


# ------------------------------------------------------------------ backward

@pytest.mark.parametrize("name", list(CASES))
def test_grad_matches_oracle(gi, name, mode):
    p, h, w = CASES[name]
    G = synth.upstream_gradient(h, w, 17)
    if p.shape[0] == 0:
        d = gi.grad(dev(p), h, w, dev(G))
        assert d.shape == (0, 8)
        return
    d = host(gi.grad(dev(p), h, w, dev(G)))
    o, A = ref.grads(p, h, w, G, with_abs=True)
    assert_grads(d, o, A, name)


def test_grad_is_deterministic(gi):
    p, h, w = CASES["plain-256x256-2k"]
    G = dev(synth.upstream_gradient(h, w, 4))
    a = host(gi.grad(dev(p), h, w, G))
    b = host(gi.grad(dev(p), h, w, G))
    np.testing.assert_array_equal(a, b)


def test_autograd_function_matches_oracle(gi):
    import paper_2403_08551_amd as P
    p, h, w = CASES["ragged-45x70"]
    p = p[6:]  # finite, active Gaussians
    G = synth.upstream_gradient(h, w, 5)
    pt = dev(p).requires_grad_(True)
    img = P.render(pt, h, w, gi)
    (img * dev(G)).sum().backward()
    o, A = ref.grads(p, h, w, G, with_abs=True)
    assert_grads(host(pt.grad), o, A, "autograd")


# ------------------------------------------------------------------ fit steps

def _hp32(hp):
    # the ABI takes float32 hyper-parameters: give the oracle the same numbers
    return {k: float(np.float32(v)) for k, v in hp.items()}


def test_fit_steps_match_oracle(gi):
    import paper_2403_08551_amd as P
    w = synth.plain_256()
    p0, T = w.params(), w.target()
    hp = dict(ref.DEFAULT_ADAM)
    cfg = P.AdamConfig(**hp)
    pd, md, vd = dev(p0), torch.zeros(p0.shape, device="cuda"), torch.zeros(p0.shape, device="cuda")
    step = torch.ones(1, dtype=torch.int32, device="cuda")
    img = torch.empty(w.height, w.width, 3, device="cuda")
    loss = torch.empty(1, device="cuda")
    po, mo, vo = p0.astype(np.float64), np.zeros_like(p0, np.float64), np.zeros_like(p0, np.float64)
    hp32 = _hp32(hp)
    lr = np.array([hp32["lr_mu"]] * 2 + [hp32["lr_l"]] * 3 + [hp32["lr_c"]] * 3)
    for t in range(1, 4):
        pin = host(pd).copy()
        gi.fit_step(pd, md, vd, dev(T), step, cfg, image_out=img, loss_out=loss)
        o, A = ref.render_culled(pin, w.height, w.width, with_abs=True)
        assert_forward(host(img), o, A, f"fit step {t} image")
        np.testing.assert_allclose(host(loss)[0], ref.mse(o, T), rtol=1e-5)
        G = ref.mse_grad(o, T)
        g, Ag = ref.grads(pin, w.height, w.width, G, with_abs=True)
        po, mo, vo = ref.adam_step(pin, mo, vo, g, t, hp32)
        got = host(pd)
        # the Adam step divides by sqrt(v): where |g| is within the gradient tolerance of zero the
        # direction is not determined by the gradient, so only the step bound applies there
        firm = np.abs(g) > 10 * GRAD_RTOL * Ag + 1e-20
        tol = 1e-4 * lr + 1e-6 * np.abs(po)
        assert np.all(np.abs(got - po)[firm] <= np.broadcast_to(tol, po.shape)[firm]), t
        assert np.all(np.abs(got - po) <= 2.0 * lr + 1e-6 * np.abs(po))
        assert firm.mean() > 0.95
        assert int(host(step)[0]) == t + 1


@pytest.mark.parametrize("which", ["plain-256x256-2k", "kodak-768x512-10k", "kodak-768x512-30k",
                                   "kodak-768x512-70k"])
def test_fit_step_gradients_element_by_element(gi, which):
    # Adam with beta1 = beta2 = 0 and eps = 1: the first moment the fused fit kernel's update
    # writes is its gradient (L2 loss scale 2 / (3 H W) included), compared element by element
    # with the oracle's at the gradient bar; the step is then lr g / (|g| + 1), checked too
    import paper_2403_08551_amd as P
    w = synth.plain_256() if which.startswith("plain") else synth.kodak_like(
        int(which.rsplit("-", 1)[1][:-1]) * 1000)
    orc = ref if which.startswith("plain") else cref
    h, wd = w.height, w.width
    p0, T = w.params(), w.target()
    o, A = orc.render_culled(p0, h, wd, with_abs=True)
    g, bound = pu.grad_bound(orc.grads, p0, h, wd, ref.mse_grad(o, T), A)
    hp = pu.linear_hp(pu.lr_for(p0, bound, [0, 1]), pu.lr_for(p0, bound, [2, 3, 4]),
                      pu.lr_for(p0, bound, [5, 6, 7]))
    pd = dev(p0)
    md, vd = torch.zeros_like(pd), torch.zeros_like(pd)
    step = torch.ones(1, dtype=torch.int32, device="cuda")
    img = torch.empty(h, wd, 3, device="cuda")
    loss = torch.empty(1, device="cuda")
    gi.query(clear=True)  # flags other tests left on the shared context
    gi.fit_step(pd, md, vd, dev(T), step, P.AdamConfig(**hp), image_out=img, loss_out=loss)
    assert_forward(host(img), o, A, f"{which} fit image")
    np.testing.assert_allclose(host(loss)[0], ref.mse(o, T), rtol=1e-5)
    pu.assert_gradient(host(md), g, bound, f"{which} fused gradient")
    lr = np.array([hp["lr_mu"]] * 2 + [hp["lr_l"]] * 3 + [hp["lr_c"]] * 3)
    pu.assert_linear_step(p0, host(pd), g, bound, lr, f"{which} linear step")
    assert gi.query(clear=True)[1] == 0


@pytest.mark.parametrize("n", [1, 15, 16, 17, 31, 33, 63, 64, 65, 127, 128, 129, 161, 193, 255,
                               257, 320])
def test_adjoint_round_tails(gi, n):
    # one 16x16 tile whose list holds every Gaussian: n covers whole rounds of 128 Gaussians
    # and remainders taken by rounds of 2, 4, 8 and 16 lanes per Gaussian; the standalone
    # gradient (gi_grad) and the fused fit kernel's (first moment at beta1 = 0) against the oracle
    import paper_2403_08551_amd as P
    h = wd = 16
    p0 = synth.gaussians(n, h, wd, seed=500 + n)
    T = synth.target_noise_rects(h, wd, seed=600 + n)
    G = synth.upstream_gradient(h, wd, 700 + n)
    b = gi.binning(dev(p0), h, wd)
    assert host(b["ranges"]).tolist() == [[0, n]]
    d = host(gi.grad(dev(p0), h, wd, dev(G)))
    og, Ag = ref.grads(p0, h, wd, G, with_abs=True)
    assert_grads(d, og, Ag, f"one tile, {n} Gaussians")
    o, A = ref.render_culled(p0, h, wd, with_abs=True)
    g, bound = pu.grad_bound(ref.grads, p0, h, wd, ref.mse_grad(o, T), A)
    hp = pu.linear_hp(pu.lr_for(p0, bound, [0, 1]), pu.lr_for(p0, bound, [2, 3, 4]),
                      pu.lr_for(p0, bound, [5, 6, 7]))
    pd = dev(p0)
    md, vd = torch.zeros_like(pd), torch.zeros_like(pd)
    step = torch.ones(1, dtype=torch.int32, device="cuda")
    gi.query(clear=True)
    gi.fit_step(pd, md, vd, dev(T), step, P.AdamConfig(**hp))
    pu.assert_gradient(host(md), g, bound, f"one tile, {n} Gaussians, fused gradient")
    assert gi.query(clear=True)[1] == 0


# ------------------------------------------------------------------ batched == plain

def small_batch():
    rng = np.random.default_rng(12)
    hs = [int(x) for x in rng.integers(20, 90, 5)]
    ws = [int(x) for x in rng.integers(20, 90, 5)]
    ns = [int(h * w // 12) for h, w in zip(hs, ws)]
    ps = [synth.gaussians(n, h, w, seed=100 + i) for i, (n, h, w) in enumerate(zip(ns, hs, ws))]
    ts = [synth.target_noise_rects(h, w, seed=200 + i) for i, (h, w) in enumerate(zip(hs, ws))]
    return hs, ws, ps, ts


def test_batched_render_and_grad_equal_plain(gi):
    import paper_2403_08551_amd as P
    hs, ws, ps, ts = small_batch()
    off = np.concatenate([[0], np.cumsum([p.shape[0] for p in ps])])
    batch = P.Batch(hs, ws, off)
    allp = dev(np.concatenate(ps))
    imgs = gi.render_batched(allp, batch)
    Gs = [synth.upstream_gradient(h, w, 30 + i) for i, (h, w) in enumerate(zip(hs, ws))]
    Gall = dev(np.concatenate([g.reshape(-1, 3) for g in Gs]))
    dall = host(gi.grad_batched(allp, batch, Gall))
    for b in range(len(hs)):
        single = host(gi.render(dev(ps[b]), hs[b], ws[b]))
        np.testing.assert_array_equal(host(batch.image(imgs, b)), single)
        ds = host(gi.grad(dev(ps[b]), hs[b], ws[b], dev(Gs[b])))
        np.testing.assert_array_equal(dall[off[b]:off[b + 1]], ds)


@pytest.mark.parametrize("binning", [1, 3], ids=["radix", "rows"])
def test_batched_with_empty_images_and_blocks_spanning_images(gi, binning):
    # eight small images, two without Gaussians, so that one block of 256 Gaussians spans
    # several images and an empty one between them; batched render and gradient against each
    # image alone (default binning), bit for bit
    import paper_2403_08551_amd as P
    hs = [40, 33, 57, 20, 64, 18, 45, 30]
    ws = [36, 70, 25, 44, 50, 90, 31, 27]
    ns = [120, 0, 90, 60, 0, 150, 75, 40]
    ps = [synth.gaussians(n, h, w, seed=300 + i) for i, (n, h, w) in enumerate(zip(ns, hs, ws))]
    off = np.concatenate([[0], np.cumsum(ns)])
    batch = P.Batch(hs, ws, off)
    allp = dev(np.concatenate(ps))
    Gs = [synth.upstream_gradient(h, w, 60 + i) for i, (h, w) in enumerate(zip(hs, ws))]
    Gall = dev(np.concatenate([g.reshape(-1, 3) for g in Gs]))
    gi.set_option(P._lib.GI_OPT_BINNING, binning)
    try:
        imgs = gi.render_batched(allp, batch)
        dall = host(gi.grad_batched(allp, batch, Gall))
    finally:
        gi.set_option(P._lib.GI_OPT_BINNING, 0)
    for b in range(len(hs)):
        pb = dev(ps[b]) if ns[b] else dev(np.zeros((0, 8), np.float32))
        single = host(gi.render(pb, hs[b], ws[b]))
        np.testing.assert_array_equal(host(batch.image(imgs, b)), single)
        if ns[b]:
            ds = host(gi.grad(pb, hs[b], ws[b], dev(Gs[b])))
            np.testing.assert_array_equal(dall[off[b]:off[b + 1]], ds)


def test_row_binning_equals_radix_on_the_64_image_batch(gi):
    # the batch of uneven images (95k tiles, 1.1M Gaussians) rendered and differentiated with
    # row binning and with the radix sort of all keys: the same images and gradients, bit for bit
    import paper_2403_08551_amd as P
    ws = synth.batch_small(64)
    ps = [w.params() for w in ws]
    off = np.concatenate([[0], np.cumsum([p.shape[0] for p in ps])])
    batch = P.Batch([w.height for w in ws], [w.width for w in ws], off)
    allp = dev(np.concatenate(ps))
    G = dev(np.concatenate([synth.upstream_gradient(w.height, w.width, 500 + i).reshape(-1, 3)
                            for i, w in enumerate(ws)]))
    out = {}
    for mode in (1, 3):
        gi.set_option(P._lib.GI_OPT_BINNING, mode)
        try:
            img = host(gi.render_batched(allp, batch))
            d = host(gi.grad_batched(allp, batch, G))
        finally:
            gi.set_option(P._lib.GI_OPT_BINNING, 0)
        out[mode] = (img, d)
    np.testing.assert_array_equal(out[1][0], out[3][0])
    np.testing.assert_array_equal(out[1][1], out[3][1])


def test_batch_with_blocks_over_too_many_tile_rows_falls_back_to_the_radix_sort(gi):
    # three tall images (1024 tile rows each, 6144 tiles in all) whose 300 Gaussians share one
    # block of 256: its images hold 3072 tile rows, more than row binning takes, so the radix
    # path bins them; the batched render equals each image rendered alone
    import paper_2403_08551_amd as P
    hs, ws, ns = [16384] * 3, [32] * 3, [100] * 3
    ps = [synth.gaussians(n, h, w, seed=600 + i) for i, (n, h, w) in enumerate(zip(ns, hs, ws))]
    off = np.concatenate([[0], np.cumsum(ns)])
    batch = P.Batch(hs, ws, off)
    imgs = gi.render_batched(dev(np.concatenate(ps)), batch)
    for b in range(3):
        np.testing.assert_array_equal(host(batch.image(imgs, b)),
                                      host(gi.render(dev(ps[b]), hs[b], ws[b])))


def test_batched_fit_equals_plain_fit(gi):
    import paper_2403_08551_amd as P
    hs, ws, ps, ts = small_batch()
    off = np.concatenate([[0], np.cumsum([p.shape[0] for p in ps])])
    batch = P.Batch(hs, ws, off)
    allp = dev(np.concatenate(ps))
    m = torch.zeros_like(allp)
    v = torch.zeros_like(allp)
    T = dev(np.concatenate([t.reshape(-1, 3) for t in ts]))
    step = torch.ones(1, dtype=torch.int32, device="cuda")
    loss = torch.empty(len(hs), device="cuda")
    for _ in range(3):
        gi.fit_step_batched(allp, m, v, T, batch, step, loss_out=loss)
    for b in range(len(hs)):
        pb = dev(ps[b])
        mb, vb = torch.zeros_like(pb), torch.zeros_like(pb)
        sb = torch.ones(1, dtype=torch.int32, device="cuda")
        lb = torch.empty(1, device="cuda")
        for _ in range(3):
            gi.fit_step(pb, mb, vb, dev(ts[b]), sb, loss_out=lb)
        np.testing.assert_array_equal(host(allp)[off[b]:off[b + 1]], host(pb))
        np.testing.assert_allclose(host(loss)[b], host(lb)[0], rtol=1e-6)


# ------------------------------------------------------------------ captured steps

@pytest.mark.parametrize("binning", [0, 3], ids=["auto", "rows"])
def test_graph_replay_matches_eager_steps(gi, binning):
    # the captured steps bin with the option given (eager steps: the default one-pass path)
    w = synth.plain_256()
    p0, T = w.params(), dev(w.target())
    pa, pb = dev(p0), dev(p0)
    ma, va, mb, vb = (torch.zeros_like(pa) for _ in range(4))
    sa = torch.ones(1, dtype=torch.int32, device="cuda")
    sb = torch.ones(1, dtype=torch.int32, device="cuda")
    for _ in range(4):
        gi.fit_step(pa, ma, va, T, sa)
    import paper_2403_08551_amd as P
    g = P.Context(0)
    g.set_option(P._lib.GI_OPT_BINNING, binning)
    graph = g.fit_graph(pb, mb, vb, T, sb)
    for _ in range(2):  # eager work and synchronisation between replays
        graph.launch(2)
        torch.cuda.synchronize()
        _ = torch.zeros(10, device="cuda").sum().item()
    graph.close()
    g.close()
    np.testing.assert_array_equal(host(pb), host(pa))
    assert int(host(sb)[0]) == 5


def test_tile_order_from_the_previous_step(gi):
    # tile order 3: each fit step's update writes the next step's longest-first order; eager
    # steps, a run of 16 captured steps and a change of image size on the same context all give
    # the bits of the index order
    import paper_2403_08551_amd as P
    w = synth.plain_256()
    p0, T = w.params(), dev(w.target())
    small = synth.gaussians(400, 40, 72, seed=7)
    Ts = dev(synth.target_noise_rects(40, 72, seed=8))

    def run(order, captured):
        ctx = P.Context(0)
        ctx.set_option(P._lib.GI_OPT_TILE_ORDER, order)
        try:
            p = dev(p0)
            m, v = torch.zeros_like(p), torch.zeros_like(p)
            st = torch.ones(1, dtype=torch.int32, device="cuda")
            if captured:
                g = ctx.fit_graph(p, m, v, T, st)
                g.launch(3)
                g.launch(17)
                torch.cuda.synchronize()
                g.close()
            else:
                for _ in range(20):
                    ctx.fit_step(p, m, v, T, st)
            # another size on the same context, then the first size again
            q = dev(small)
            mq, vq = torch.zeros_like(q), torch.zeros_like(q)
            sq = torch.ones(1, dtype=torch.int32, device="cuda")
            for _ in range(3):
                ctx.fit_step(q, mq, vq, Ts, sq)
            img = host(ctx.render(p, w.height, w.width))
            ctx.fit_step(p, m, v, T, st)
            assert ctx.query(clear=True)[1] == 0
            return host(p), host(m), host(q), img
        finally:
            ctx.close()

    want = run(1, False)
    for order, captured in ((3, False), (3, True), (2, True)):
        got = run(order, captured)
        for a, b in zip(got, want):
            np.testing.assert_array_equal(a, b, err_msg=f"order {order}, captured {captured}")


def test_tile_order_above_the_update_kernels_limit(gi):
    # more than 16384 tiles: order 3 sorts once per tile count and keeps that order (the update
    # kernel writes none); fit steps give the bits of the index order
    import paper_2403_08551_amd as P
    h, w = 2080, 2064  # 130 x 129 = 16770 tiles
    p0 = synth.gaussians(3000, h, w, seed=31)
    T = dev(synth.target_noise_rects(h, w, seed=32))
    out = []
    for order in (1, 3):
        ctx = P.Context(0)
        ctx.set_option(P._lib.GI_OPT_TILE_ORDER, order)
        try:
            p = dev(p0)
            m, v = torch.zeros_like(p), torch.zeros_like(p)
            st = torch.ones(1, dtype=torch.int32, device="cuda")
            for _ in range(3):
                ctx.fit_step(p, m, v, T, st)
            assert ctx.query(clear=True)[1] == 0
            out.append((host(p), host(m), host(v)))
        finally:
            ctx.close()
    for a, b in zip(out[0], out[1]):
        np.testing.assert_array_equal(a, b)


def test_graph_runs_of_sixteen_steps_match_eager_steps(gi):
    # 37 steps in launches of 37 and 3: runs of 16 go out as one launch of the 16-step graph,
    # the rest one step per launch; the result equals 40 eager steps bit for bit
    w = synth.plain_256()
    p0, T = w.params(), dev(w.target())
    pa, pb = dev(p0), dev(p0)
    ma, va, mb, vb = (torch.zeros_like(pa) for _ in range(4))
    sa = torch.ones(1, dtype=torch.int32, device="cuda")
    sb = torch.ones(1, dtype=torch.int32, device="cuda")
    loss_a = torch.empty(1, device="cuda")
    loss_b = torch.empty(1, device="cuda")
    for _ in range(40):
        gi.fit_step(pa, ma, va, T, sa, loss_out=loss_a)
    import paper_2403_08551_amd as P
    g = P.Context(0)
    graph = g.fit_graph(pb, mb, vb, T, sb, loss_out=loss_b)
    try:
        graph.launch(37)
        torch.cuda.synchronize()
        _ = torch.zeros(10, device="cuda").sum().item()
        graph.launch(3)
        torch.cuda.synchronize()
        assert graph.query()[1] == 0
    finally:
        graph.close()
        g.close()
    np.testing.assert_array_equal(host(pb), host(pa))
    np.testing.assert_array_equal(host(mb), host(ma))
    np.testing.assert_array_equal(host(vb), host(va))
    np.testing.assert_array_equal(host(loss_b), host(loss_a))
    assert int(host(sb)[0]) == 41


def test_graph_launch_starts_from_the_parameters_as_they_are(gi):
    # every launch of a captured step bins the parameters as they are then, so parameters
    # changed between launches are the ones fitted
    w = synth.plain_256()
    p0, T = w.params(), dev(w.target())
    pa, pb = dev(p0), dev(p0)
    ma, va, mb, vb = (torch.zeros_like(pa) for _ in range(4))
    sa = torch.ones(1, dtype=torch.int32, device="cuda")
    sb = torch.ones(1, dtype=torch.int32, device="cuda")
    import paper_2403_08551_amd as P
    g = P.Context(0)
    graph = g.fit_graph(pb, mb, vb, T, sb)
    try:
        graph.launch(2)
        torch.cuda.synchronize()
        for _ in range(2):
            gi.fit_step(pa, ma, va, T, sa)
        torch.cuda.synchronize()
        for p in (pa, pb):  # every Gaussian one pixel to the right, half a pixel up
            p[:, 0] += 1.0
            p[:, 1] -= 0.5
        torch.cuda.synchronize()
        graph.launch(3)
        torch.cuda.synchronize()
        for _ in range(3):
            gi.fit_step(pa, ma, va, T, sa)
        assert graph.query()[1] == 0
    finally:
        graph.close()
        g.close()
    np.testing.assert_array_equal(host(pb), host(pa))
    assert int(host(sb)[0]) == 6


@pytest.mark.parametrize("binning", [1, 2, 3], ids=["radix", "one-pass", "rows"])
def test_renders_between_steps_leave_fit_and_grad_unchanged(binning):
    # a render's binning skips the key slots (only the adjoint reads them): steps, gradients and
    # captured steps after renders on the same context bin again and give the same bits
    import paper_2403_08551_amd as P
    w = synth.plain_256()
    h, wd = w.height, w.width
    p0, T = w.params(), dev(w.target())
    o = dev(np.random.default_rng(5).uniform(0.2, 1.0, p0.shape[0]))
    dl = dev(np.random.default_rng(6).normal(size=(h, wd, 3)))
    pa, pb = dev(p0), dev(p0)
    ma, va, mb, vb = (torch.zeros_like(pa) for _ in range(4))
    sa = torch.ones(1, dtype=torch.int32, device="cuda")
    sb = torch.ones(1, dtype=torch.int32, device="cuda")
    ca, cb = P.Context(0), P.Context(0)
    graph = None
    try:
        for c in (ca, cb):
            c.set_option(P._lib.GI_OPT_BINNING, binning)
        for _ in range(3):
            ca.fit_step(pa, ma, va, T, sa)
        ga = host(ca.grad(pa, h, wd, dl))
        for _ in range(3):
            cb.render(pb, h, wd)
            cb.fit_step(pb, mb, vb, T, sb)
            cb.render_opacity(pb, o, h, wd, blend="alpha")
        cb.render(pb, h, wd)
        np.testing.assert_array_equal(host(pb), host(pa))
        np.testing.assert_array_equal(host(cb.grad(pb, h, wd, dl)), ga)
        for _ in range(2):
            ca.fit_step(pa, ma, va, T, sa)
        graph = cb.fit_graph(pb, mb, vb, T, sb)
        for _ in range(2):  # a render between the launches of the captured step
            graph.launch(1)
            cb.render(pb, h, wd)
            torch.cuda.synchronize()
        np.testing.assert_array_equal(host(pb), host(pa))
        assert int(host(sb)[0]) == int(host(sa)[0]) == 6
    finally:
        if graph is not None:
            graph.close()
        ca.close()
        cb.close()


# ------------------------------------------------------------------ flags and edge cases

def test_nonfinite_flag(gi):
    p, h, w = CASES["ragged-45x70"]
    gi.query(clear=True)
    gi.render(dev(p), h, w)
    _, flags = gi.query(clear=True)
    assert flags & 2


@pytest.mark.parametrize("binning", [1, 2, 3])
def test_key_overflow_skips_the_update(binning):
    import paper_2403_08551_amd as P
    ctx = P.Context(0)
    try:
        ctx.set_option(P._lib.GI_OPT_BINNING, binning)
        ctx.set_option(P._lib.GI_OPT_SYNC, 0)
        ctx.reserve(2000, 256, 4096)  # cfg1 needs ~15k keys
        w = synth.plain_256()
        p = dev(w.params())
        p_before = host(p).copy()
        m, v = torch.zeros_like(p), torch.zeros_like(p)
        step = torch.ones(1, dtype=torch.int32, device="cuda")
        ctx.fit_step(p, m, v, dev(w.target()), step)
        keys, flags = ctx.query(clear=True)
        assert flags & 1
        assert keys > 4096
        np.testing.assert_array_equal(host(p), p_before)
    finally:
        ctx.close()


# ------------------------------------------------------------------ full-size workloads, sampled

@pytest.mark.parametrize("n", [70_000])
def test_kodak_size_full_images_and_gradients(gi, n):
    # the metric's workload whole: tile lists key for key, every pixel of the render and every
    # gradient element (gi_grad with a seeded dL/dC) against the C oracle
    w = synth.kodak_like(n)
    p, h, wd = w.params(), w.height, w.width
    pd = dev(p)
    b = gi.binning(pd, h, wd)
    ranges, ids = cref.tile_lists(p, h, wd)
    assert b["keys"] == ids.size
    np.testing.assert_array_equal(host(b["ranges"]), ranges)
    np.testing.assert_array_equal(host(b["ids"]), ids)
    img = host(gi.render(pd, h, wd))
    o, A = cref.render_culled(p, h, wd, with_abs=True)
    assert_forward(img, o, A, "kodak full image")
    G = synth.upstream_gradient(h, wd, 3)
    d = host(gi.grad(pd, h, wd, dev(G)))
    od, Ad = cref.grads(p, h, wd, G, with_abs=True)
    assert_grads(d, od, Ad, "kodak full gradients")


@pytest.mark.parametrize("n", [100_000, 300_000])
def test_div2k_size_full_images(gi, n):
    # 2040x1356 (row binning): counts exactly, every pixel of the render against the C oracle;
    # gradients whole at 100k, on a seeded sample of Gaussians at 300k
    w = synth.div2k_full(n)
    p, h, wd = w.params(), w.height, w.width
    pd = dev(p)
    rect, count = cref.tile_rects(p, h, wd)
    b = gi.binning(pd, h, wd)
    assert b["keys"] == int(count.sum())
    np.testing.assert_array_equal(host(b["counts"]), count)
    img = host(gi.render(pd, h, wd))
    o, A = cref.render_culled(p, h, wd, with_abs=True)
    assert_forward(img, o, A, f"div2k {n} full image")
    G = synth.upstream_gradient(h, wd, 4)
    d = host(gi.grad(pd, h, wd, dev(G)))
    if n <= 100_000:
        od, Ad = cref.grads(p, h, wd, G, with_abs=True)
        assert_grads(d, od, Ad, f"div2k {n} full gradients")
    else:
        which = np.random.default_rng(2).choice(n, 2000, replace=False)
        od, Ad = cref.grads_subset(p, h, wd, G, which, with_abs=True)
        assert_grads(d[which], od, Ad, f"div2k {n} sampled gradients")


def binning_in_mode(gi, mode, pd, h, wd):
    import paper_2403_08551_amd as P
    gi.set_option(P._lib.GI_OPT_BINNING, mode)
    try:
        b = gi.binning(pd, h, wd)
        return b["keys"], host(b["ranges"]), host(b["ids"]), host(b["offsets"])
    finally:
        gi.set_option(P._lib.GI_OPT_BINNING, 0)


@pytest.mark.parametrize("n", [300_000])
def test_row_binning_equals_radix_at_full_size(gi, n):
    # 2040x1356, 10880 tiles: the row binning (the default at this size) against the radix
    # sort, key for key; the radix path is itself checked against the oracle above
    w = synth.div2k_full(n)
    pd = dev(w.params())
    rows = binning_in_mode(gi, 3, pd, w.height, w.width)
    radix = binning_in_mode(gi, 1, pd, w.height, w.width)
    assert rows[0] == radix[0]
    for a, b in zip(rows[1:], radix[1:]):
        np.testing.assert_array_equal(a, b)


def test_row_binning_matches_oracle_on_wide_rows(gi):
    # one image 1024 tiles wide (the widest row binning takes) and one tile high, and a
    # 1025-tile-wide one (radix then); tile lists against the oracle
    for wd in (16 * 1024, 16 * 1024 + 5):
        h = 20
        p = synth.gaussians(3000, h, wd, seed=wd, l_lo=0.5, l_hi=40.0)
        ranges, ids = cref.tile_lists(p, h, wd)
        k, r, i, _ = binning_in_mode(gi, 3, dev(p), h, wd)
        assert k == ids.size
        np.testing.assert_array_equal(r, ranges)
        np.testing.assert_array_equal(i, ids)


# ------------------------------------------------------------------ autotuner

def test_autotune_reads_but_never_writes_and_keeps_results_exact(gi):
    import paper_2403_08551_amd as P
    w = synth.plain_256()
    p = dev(w.params())
    T = dev(w.target())
    before = host(p).copy()
    ref_img = host(gi.render(p, w.height, w.width))
    sc = gi.autotune(p, T, reps=2)
    assert sc["binning"] in (1, 2, 3) and sc["fwd_pixels"] in (1, 2, 4)
    assert sc["sort_bits"] in (0, 4, 6, 8, 11) and sc["tile_order"] in (1, 2, 3)
    assert sc["fit_waves"] in (4, 6) and sc["ms_per_step"] > 0
    np.testing.assert_array_equal(host(p), before)
    for opt in (P._lib.GI_OPT_FWD_PIXELS, P._lib.GI_OPT_BINNING, P._lib.GI_OPT_TILE_ORDER,
                P._lib.GI_OPT_FIT_WAVES):
        assert gi.get_option(opt) == 0  # explicit options untouched
    np.testing.assert_array_equal(host(gi.render(p, w.height, w.width)), ref_img)


def _schedules(tiles, rows_ok=True):
    """Every schedule the autotuner can choose for a workload with this many tiles."""
    out = []
    paths = ([2] if tiles <= 2048 else []) + ([3] if rows_ok else []) + [1]
    for b in paths:
        for px in (1, 2, 4):
            for order in (1, 2, 3):
                for waves in (4, 6):
                    out.append((b, px, 0, order, waves))
        if b == 1:
            out += [(1, 4, d, 2, 4) for d in (4, 6, 8, 11)]
    return out


def _run_schedule(P, sched, p0, T, h, w, G, batch=None):
    ctx = P.Context(0)
    try:
        b, px, digit, order, waves = sched
        ctx.set_option(P._lib.GI_OPT_BINNING, b)
        ctx.set_option(P._lib.GI_OPT_FIT_WAVES, waves)
        ctx.set_option(P._lib.GI_OPT_FWD_PIXELS, px)
        ctx.set_option(P._lib.GI_OPT_SORT_BITS, digit)
        ctx.set_option(P._lib.GI_OPT_TILE_ORDER, order)
        pd = dev(p0)
        if batch is None:
            img = host(ctx.render(pd, h, w))
            g = host(ctx.grad(pd, h, w, dev(G)))
        else:
            img = host(ctx.render_batched(pd, batch))
            g = host(ctx.grad_batched(pd, batch, dev(G)))
        m, v = torch.zeros_like(pd), torch.zeros_like(pd)
        st = torch.ones(1, dtype=torch.int32, device="cuda")
        for _ in range(2):
            if batch is None:
                ctx.fit_step(pd, m, v, T, st)
            else:
                ctx.fit_step_batched(pd, m, v, T, batch, st)
        assert ctx.query()[1] == 0
        return img, g, host(pd), host(m), host(v)
    finally:
        ctx.close()


def test_every_schedule_gives_the_same_bits_single_image():
    # each knob the autotuner sets (binning path, radix digit, pixels per lane, tile order, fit
    # kernel waves per SIMD) leaves the render, the gradient and two fit steps bit for bit as
    # the default schedule
    import paper_2403_08551_amd as P
    w = synth.plain_256()
    p0, T = w.params(), dev(w.target())
    G = synth.upstream_gradient(w.height, w.width, 3)
    want = _run_schedule(P, (0, 0, 0, 0, 0), p0, T, w.height, w.width, G)
    for sched in _schedules(256):
        got = _run_schedule(P, sched, p0, T, w.height, w.width, G)
        for a, b, what in zip(got, want, ("image", "gradient", "params", "m", "v")):
            np.testing.assert_array_equal(a, b, err_msg=f"{what} under schedule {sched}")


def test_every_schedule_gives_the_same_bits_batch():
    import paper_2403_08551_amd as P
    dims = [(96, 160), (200, 72), (33, 257)]
    ps = [synth.gaussians(300 + 100 * i, h, w, seed=40 + i) for i, (h, w) in enumerate(dims)]
    off = np.concatenate([[0], np.cumsum([p.shape[0] for p in ps])])
    batch = P.Batch([h for h, _ in dims], [w for _, w in dims], off)
    p0 = np.concatenate(ps)
    T = dev(np.full((sum(h * w for h, w in dims), 3), 0.5, np.float32))
    G = np.concatenate([synth.upstream_gradient(h, w, 60 + i).reshape(-1, 3)
                        for i, (h, w) in enumerate(dims)])
    tiles = sum(((h + 15) // 16) * ((w + 15) // 16) for h, w in dims)
    want = _run_schedule(P, (0, 0, 0, 0, 0), p0, T, 0, 0, G, batch=batch)
    for sched in _schedules(tiles):
        got = _run_schedule(P, sched, p0, T, 0, 0, G, batch=batch)
        for a, b, what in zip(got, want, ("images", "gradient", "params", "m", "v")):
            np.testing.assert_array_equal(a, b, err_msg=f"{what} under schedule {sched}")


def test_autotune_cache_round_trip(tmp_path):
    import paper_2403_08551_amd as P
    w = synth.plain_256()
    p, T = dev(w.params()), dev(w.target())
    a = P.Context(0)
    b = P.Context(0)
    try:
        sc = a.autotune(p, T, reps=1)
        path = str(tmp_path / "tune.jsonl")
        a.autotune_save(path)
        lines = open(path).read().splitlines()
        assert len(lines) == 1 and '"arch": "gfx950"' in lines[0]
        assert f'"binning": {sc["binning"]}' in lines[0]
        # an entry of another architecture is skipped; the file's own entry is taken
        with open(path, "a") as f:
            f.write(lines[0].replace('"arch": "gfx950"', '"arch": "gfx000"') + "\n")
        assert b.autotune_load(path) == 1
        # b now renders with the loaded schedule: same bits as a's tuned render
        np.testing.assert_array_equal(host(b.render(p, w.height, w.width)),
                                      host(a.render(p, w.height, w.width)))
        bad = str(tmp_path / "bad.jsonl")
        with open(bad, "w") as f:
            f.write(lines[0].replace('"fwd_pixels": ', '"fwd_pixels": 3') + "\n")
        with pytest.raises(P.GiError):
            b.autotune_load(bad)
        with pytest.raises(P.GiError):
            b.autotune_load(str(tmp_path / "missing.jsonl"))
    finally:
        a.close()
        b.close()


def test_graphs_survive_later_growth_of_the_context(gi):
    # a graph keeps its own workspace: a larger graph or call afterwards must not move it
    import paper_2403_08551_amd as P
    small = synth.plain_256(500)
    big = synth.kodak_like(10_000)
    ctx = P.Context(0)
    try:
        p_s, T_s = dev(small.params()), dev(small.target())
        m_s, v_s = torch.zeros_like(p_s), torch.zeros_like(p_s)
        st_s = torch.ones(1, dtype=torch.int32, device="cuda")
        g_small = ctx.fit_graph(p_s, m_s, v_s, T_s, st_s)
        p_b, T_b = dev(big.params()), dev(big.target())
        m_b, v_b = torch.zeros_like(p_b), torch.zeros_like(p_b)
        st_b = torch.ones(1, dtype=torch.int32, device="cuda")
        g_big = ctx.fit_graph(p_b, m_b, v_b, T_b, st_b)
        ctx.render(p_b, big.height, big.width)  # grows the context's own workspace too
        g_small.launch(3)
        g_big.launch(1)
        # eager reference of the small fit
        p_e = dev(small.params())
        m_e, v_e = torch.zeros_like(p_e), torch.zeros_like(p_e)
        st_e = torch.ones(1, dtype=torch.int32, device="cuda")
        for _ in range(3):
            gi.fit_step(p_e, m_e, v_e, T_s, st_e)
        np.testing.assert_array_equal(host(p_s), host(p_e))
        assert g_small.query()[1] == 0 and g_big.query()[1] == 0
        g_small.close()
        g_big.close()
    finally:
        ctx.close()


def test_large_batch_subset_gradients_and_finite_differences(gi):
    # 16 images shaped like the 256-image workload (sides 512-2048, 20k-200k Gaussians), one
    # batched gradient call; per image, 32 sampled Gaussians against the oracle's analytic
    # gradient and 4 of them against a local central finite difference
    import paper_2403_08551_amd as P
    ws = synth.batch_large(16)
    ps = [w.params() for w in ws]
    Gs = [synth.upstream_gradient(w.height, w.width, 700 + i) for i, w in enumerate(ws)]
    off = np.concatenate([[0], np.cumsum([p.shape[0] for p in ps])])
    batch = P.Batch([w.height for w in ws], [w.width for w in ws], off)
    d = host(gi.grad_batched(dev(np.concatenate(ps)), batch,
                             dev(np.concatenate([g.reshape(-1, 3) for g in Gs]))))
    rng = np.random.default_rng(3)
    for b, w in enumerate(ws):
        which = rng.choice(ps[b].shape[0], 32, replace=False)
        o, A = cref.grads_subset(ps[b], w.height, w.width, Gs[b], which, with_abs=True)
        got = d[off[b]:off[b + 1]][which]
        assert_grads(got, o, A, f"batch image {b}")
        rect0, _ = ref.tile_rects(ps[b], w.height, w.width)
        for n in which[:4]:
            fd = ref.fd_local(ps[b], w.height, w.width, Gs[b], int(n))
            scale = np.abs(o).max() + 1e-30
            k = int(np.nonzero(which == n)[0][0])
            assert np.all(np.abs(got[k] - fd) <= 1e-4 * A[k] + 1e-5 * scale), (b, n, got[k], fd)
