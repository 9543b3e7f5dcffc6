"""Parity of the rotation-scale covariance form (Sec. 3.1, Eq. RSSR) on the HIP path with the
FP64 oracle: records (mu_x, mu_y, s1, s2, theta, c0, c1, c2), Sigma = (R S)(R S)^T.

Bars as for the Cholesky form: tile rects, counts, ranges and lists bit-exact (the box rule uses
only s1^2 and s2^2, so the decision is exact on both sides); forward within 1e-5 A(p); gradients
within 1e-4 A_theta; fit steps as in their test.
"""
import math

import numpy as np
import pytest

import parity_util as pu
import synth
from oracle import ref

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

FWD_RTOL = 1e-5
GRAD_RTOL = 1e-4


@pytest.fixture(scope="module")
def gi():
    import paper_2403_08551_amd as P
    ctx = P.Context(0, covariance="rotation_scale")
    yield ctx
    ctx.close()


def dev(a):
    return torch.as_tensor(np.ascontiguousarray(a)).to(dtype=torch.float32, device="cuda")


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def ragged_case():
    h, w = 45, 70
    p = synth.gaussians_rs(160, h, w, seed=41, s_lo=0.5, s_hi=12.0)
    p[:4, 0] = [-30.0, 200.0, 35.0, 0.0]
    p[:4, 1] = [10.0, 10.0, -40.0, 0.0]
    p[4] = [np.nan, 1, 1, 1, 0, 1, 1, 1]
    p[5, 2] = 0.0                        # s1 = 0: inactive
    p[6, 4] = 3e7                        # |theta| > 2^24: inactive
    p[7, 2:5] = [-3.0, 2.0, 1.0]         # negative scale: same Sigma as +3
    p[8, 2:5] = [4.0, -1.5, 40.0]        # angle far outside (-pi, pi]
    p[9, 2:5] = [2.0, 2.0, 0.3]          # isotropic: no angle gradient
    p[10, 2:5] = [0.5, 24.0, 0.7]        # 48:1 elongation
    p[11, 2:5] = [2.0, 1.0, 0.0]         # 3 s1 = 6 exactly on the box rule
    return p, h, w


def cases():
    return {
        "rs-plain-256x256-2k": (synth.gaussians_rs(2000, 256, 256, seed=30, s_lo=1.0, s_hi=8.0,
                                                   c_lo=0.0, c_hi=1.0), 256, 256),
        "rs-ragged-45x70": ragged_case(),
        "rs-wide-100x120": (synth.gaussians_rs(400, 100, 120, seed=31, s_lo=0.5, s_hi=32.0),
                            100, 120),
        "rs-one-pixel": (synth.gaussians_rs(5, 1, 1, seed=32), 1, 1),
        "rs-empty": (np.zeros((0, 8), np.float32), 33, 17),
    }


CASES = cases()


def check(g, o, A, rtol, what):
    # plus an absolute floor far below any real error: where a value is exactly zero (theta of an
    # isotropic Gaussian) the oracle's float64 trigonometry leaves rounding noise of ~1e-18, and
    # the sum of absolute contributions is then noise of the same size
    bad = np.abs(g - o) > rtol * A + 1e-12 * np.abs(o).max(initial=0.0) + 1e-30
    if bad.any():
        i = np.argmax(np.abs(g - o) / (A + 1e-300))
        raise AssertionError(f"{what}: {bad.sum()} values off; worst gpu {g.flat[i]} oracle "
                             f"{o.flat[i]} A {A.flat[i]} at {np.unravel_index(i, g.shape)}")


@pytest.fixture(params=[1, 2, 3], ids=["radix", "one-pass", "rows"])
def mode(request, gi):
    import paper_2403_08551_amd as P
    gi.set_option(P._lib.GI_OPT_BINNING, request.param)
    yield request.param
    gi.set_option(P._lib.GI_OPT_BINNING, 0)


def test_option_round_trip(gi):
    import paper_2403_08551_amd as P
    assert gi.get_option(P._lib.GI_OPT_COVARIANCE) == P._lib.GI_COV_ROTATION_SCALE
    with pytest.raises(P.GiError):
        gi.set_option(P._lib.GI_OPT_COVARIANCE, 7)
    assert gi.get_option(P._lib.GI_OPT_COVARIANCE) == P._lib.GI_COV_ROTATION_SCALE


@pytest.mark.parametrize("name", list(CASES))
def test_rs_binning_bit_exact(gi, name, mode):
    p, h, w = CASES[name]
    b = gi.binning(dev(p), h, w)
    rect, count = ref.tile_rects(p, h, w, cov="rs")
    ranges, ids = ref.tile_lists(p, h, w, cov="rs")
    if p.shape[0]:
        np.testing.assert_array_equal(host(b["rects"]), rect)
        np.testing.assert_array_equal(host(b["counts"]), count)
    assert b["keys"] == int(count.sum())
    np.testing.assert_array_equal(host(b["ranges"]), ranges)
    np.testing.assert_array_equal(host(b["ids"]), ids)


@pytest.mark.parametrize("name", list(CASES))
def test_rs_render_matches_oracle(gi, name, mode):
    p, h, w = CASES[name]
    img = host(gi.render(dev(p), h, w))
    o, A = ref.render_culled(p, h, w, with_abs=True, cov="rs")
    check(img, o, A, FWD_RTOL, name)


@pytest.mark.parametrize("name", list(CASES))
def test_rs_grad_matches_oracle(gi, name, mode):
    p, h, w = CASES[name]
    G = synth.upstream_gradient(h, w, 18)
    if p.shape[0] == 0:
        assert gi.grad(dev(p), h, w, dev(G)).shape == (0, 8)
        return
    d = host(gi.grad(dev(p), h, w, dev(G)))
    o, A = ref.grads(p, h, w, G, with_abs=True, cov="rs")
    check(d, o, A, GRAD_RTOL, name)
    if name == "rs-ragged-45x70":
        assert d[9, 4] == 0.0  # s1 = s2: Sigma does not depend on theta
        assert np.all(d[[4, 5, 6]] == 0.0)


def test_rs_with_zero_angle_renders_the_cholesky_record_bitwise(gi):
    # theta = 0, s > 0: the rebuilt Cholesky factor is (s1, 0, s2) exactly, so the records agree
    import paper_2403_08551_amd as P
    p, h, w = CASES["rs-plain-256x256-2k"]
    p = p.copy()
    p[:, 4] = 0.0
    chol = p.copy()
    chol[:, 2], chol[:, 3], chol[:, 4] = p[:, 2], 0.0, p[:, 3]
    c = P.Context(0)
    try:
        np.testing.assert_array_equal(host(gi.render(dev(p), h, w)), host(c.render(dev(chol), h, w)))
    finally:
        c.close()


def test_rs_fit_steps_match_oracle(gi):
    import paper_2403_08551_amd as P
    h, w = 96, 128
    p0 = synth.gaussians_rs(600, h, w, seed=33, s_lo=0.6, s_hi=6.0, c_lo=0.0, c_hi=0.3)
    p0[:20, 2] = 0.52  # near the floor: some updates land below l_min and are raised to it
    T = synth.target_noise_rects(h, w, seed=34)
    hp = dict(ref.DEFAULT_ADAM)
    cfg = P.AdamConfig(**hp)
    pd = dev(p0)
    md, vd = torch.zeros_like(pd), torch.zeros_like(pd)
    step = torch.ones(1, dtype=torch.int32, device="cuda")
    img = torch.empty(h, w, 3, device="cuda")
    loss = torch.empty(1, device="cuda")
    hp32 = {k: float(np.float32(v)) for k, v in hp.items()}
    lr = np.array([hp32["lr_mu"]] * 2 + [hp32["lr_l"]] * 3 + [hp32["lr_c"]] * 3)
    mo, vo = np.zeros_like(p0, np.float64), np.zeros_like(p0, np.float64)
    for t in range(1, 4):
        pin = host(pd).copy()
        gi.fit_step(pd, md, vd, dev(T), step, cfg, image_out=img, loss_out=loss)
        o, A = ref.render_culled(pin, h, w, with_abs=True, cov="rs")
        check(host(img), o, A, FWD_RTOL, f"fit step {t} image")
        np.testing.assert_allclose(host(loss)[0], ref.mse(o, T), rtol=1e-5)
        g, Ag = ref.grads(pin, h, w, ref.mse_grad(o, T), with_abs=True, cov="rs")
        po, mo, vo = ref.adam_step(pin, mo, vo, g, t, hp32, cov="rs")
        got = host(pd)
        firm = np.abs(g) > 10 * GRAD_RTOL * Ag + 1e-20
        tol = 1e-4 * lr + 1e-6 * np.abs(po)
        assert np.all(np.abs(got - po)[firm] <= np.broadcast_to(tol, po.shape)[firm]), t
        assert np.all(np.abs(got - po) <= 2.0 * lr + 1e-6 * np.abs(po))
        assert firm.mean() > 0.9
        assert np.all(np.abs(got[:, 2:4]) >= np.float32(hp32["l_min"]))
    assert int(host(step)[0]) == 4


def test_rs_fit_step_gradients_element_by_element(gi):
    # Adam with beta1 = beta2 = 0, eps = 1: the first moment is the fused kernel's gradient in
    # (mu, s1, s2, theta, c'), compared element by element with the oracle's at the gradient bar
    import paper_2403_08551_amd as P
    h, w = 96, 128
    p0 = synth.gaussians_rs(600, h, w, seed=35, s_lo=0.6, s_hi=6.0, c_lo=0.0, c_hi=0.3)
    T = synth.target_noise_rects(h, w, seed=36)
    o, A = ref.render_culled(p0, h, w, with_abs=True, cov="rs")

    def grads_rs(p, hh, ww, G, with_abs):
        return ref.grads(p, hh, ww, G, with_abs=with_abs, cov="rs")

    g, bound = pu.grad_bound(grads_rs, p0, h, w, ref.mse_grad(o, T), A)
    hp = pu.linear_hp(pu.lr_for(p0, bound, [0, 1]), pu.lr_for(p0, bound, [2, 3, 4]),
                      pu.lr_for(p0, bound, [5, 6, 7]))
    pd = dev(p0)
    md, vd = torch.zeros_like(pd), torch.zeros_like(pd)
    step = torch.ones(1, dtype=torch.int32, device="cuda")
    gi.fit_step(pd, md, vd, dev(T), step, P.AdamConfig(**hp))
    pu.assert_gradient(host(md), g, bound, "rotation-scale fused gradient")
    lr = np.array([hp["lr_mu"]] * 2 + [hp["lr_l"]] * 3 + [hp["lr_c"]] * 3)
    pu.assert_linear_step(p0, host(pd), g, bound, lr, "rotation-scale linear step")


def test_rs_batched_equals_plain_and_graph_equals_eager(gi):
    import paper_2403_08551_amd as P
    hs, ws = [40, 75, 23], [64, 31, 90]
    ps = [synth.gaussians_rs(h * w // 10, h, w, seed=50 + i) for i, (h, w) in enumerate(zip(hs, ws))]
    off = np.concatenate([[0], np.cumsum([p.shape[0] for p in ps])])
    batch = P.Batch(hs, ws, off)
    allp = dev(np.concatenate(ps))
    imgs = gi.render_batched(allp, batch)
    Gs = [synth.upstream_gradient(h, w, 60 + i) for i, (h, w) in enumerate(zip(hs, ws))]
    dall = host(gi.grad_batched(allp, batch, dev(np.concatenate([g.reshape(-1, 3) for g in Gs]))))
    for b in range(len(hs)):
        np.testing.assert_array_equal(host(batch.image(imgs, b)),
                                      host(gi.render(dev(ps[b]), hs[b], ws[b])))
        np.testing.assert_array_equal(dall[off[b]:off[b + 1]],
                                      host(gi.grad(dev(ps[b]), hs[b], ws[b], dev(Gs[b]))))
    # a captured step keeps the covariance form of the context it was made from
    h, w = hs[0], ws[0]
    T = dev(synth.target_sinusoids(h, w, seed=61))
    pa, pb = dev(ps[0]), dev(ps[0])
    ma, va, mb, vb = (torch.zeros_like(pa) for _ in range(4))
    sa = torch.ones(1, dtype=torch.int32, device="cuda")
    sb = torch.ones(1, dtype=torch.int32, device="cuda")
    for _ in range(3):
        gi.fit_step(pa, ma, va, T, sa)
    graph = gi.fit_graph(pb, mb, vb, T, sb)
    gi.set_option(P._lib.GI_OPT_COVARIANCE, P._lib.GI_COV_CHOLESKY)
    try:
        graph.launch(1)
        torch.cuda.synchronize()
        graph.launch(2)
        torch.cuda.synchronize()
    finally:
        gi.set_option(P._lib.GI_OPT_COVARIANCE, P._lib.GI_COV_ROTATION_SCALE)
        graph.close()
    np.testing.assert_array_equal(host(pb), host(pa))
    assert math.isclose(float(host(sb)[0]), 4.0)


def test_rs_kodak_size_sampled(gi):
    # 768x512 / 70k rotation-scale records: binning bit-exact, sampled pixels against the oracle's
    # per-pixel sum over the Gaussians of the pixel's tile list
    h, w = 512, 768
    p = synth.gaussians_rs(70_000, h, w, seed=2070, s_lo=1.0, s_hi=8.0, c_lo=0.0, c_hi=1.0)
    b = gi.binning(dev(p), h, w)
    ranges, ids = ref.tile_lists(p, h, w, cov="rs")
    np.testing.assert_array_equal(host(b["ranges"]), ranges)
    np.testing.assert_array_equal(host(b["ids"]), ids)
    img = host(gi.render(dev(p), h, w))
    inv = ref.inverse_covariance(p, cov="rs")
    pf = p.astype(np.float64)
    tw, _ = ref.grid_tiles(h, w)
    rng = np.random.default_rng(2071)
    for y, x in zip(rng.integers(0, h, 64), rng.integers(0, w, 64)):
        a, e_ = ranges[(y // 16) * tw + x // 16]
        sel = ids[a:e_]
        dx, dy = x + 0.5 - pf[sel, 0], y + 0.5 - pf[sel, 1]
        s = 0.5 * (inv[0][sel] * dx * dx + 2 * inv[1][sel] * dx * dy + inv[2][sel] * dy * dy)
        e = np.exp(-s)
        want = (e[:, None] * pf[sel, 5:8]).sum(0)
        A = (e[:, None] * np.abs(pf[sel, 5:8])).sum(0)
        assert np.all(np.abs(img[y, x] - want) <= FWD_RTOL * A + 1e-30), (y, x)
