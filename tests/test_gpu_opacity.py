"""Parity of the opacity renderings (Sec. 3.2: Eq. rasterization3 summation with a separate
opacity, Eq. rasterization1/2 alpha blending in index order) on the HIP path with the FP64
oracle.  Bars: forward within 1e-5 A(p), gradients (params and opacity) within 1e-4 of the sum of
absolute per-pixel contributions, as for the merged-colour path.
"""
import numpy as np
import pytest

import parity_util as pu
import synth
from oracle import blend, ref

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

FWD_RTOL = 1e-5
GRAD_RTOL = 1e-4


def dev(a):
    return torch.as_tensor(np.ascontiguousarray(a)).to(dtype=torch.float32, device="cuda")


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def opac(n, seed, lo=0.05, hi=0.95):
    return np.random.default_rng(seed).uniform(lo, hi, n).astype(np.float32)


def ragged_case():
    h, w = 45, 70
    p = synth.gaussians(150, h, w, seed=81, l_lo=0.5, l_hi=10.0)
    p[:3, 0] = [-30.0, 200.0, 35.0]
    p[:3, 1] = [10.0, 10.0, -40.0]
    p[3] = [np.nan, 1, 1, 0, 1, 1, 1, 1]
    p[4, 5:8] = [-2.0, 3.0, -0.5]
    o = opac(150, 82)
    o[5:9] = [1.6, 1.0, 0.0, -0.3]  # clamped near the centre, full, transparent, negative
    return p, o, h, w


def cases():
    w = synth.plain_256(1500)
    return {
        "plain-256x256": (w.params(), opac(1500, 80), 256, 256),
        "ragged-45x70": ragged_case(),
        "wide-l-100x120": (synth.gaussians(300, 100, 120, seed=83, l_lo=0.5, l_hi=32.0),
                           opac(300, 84), 100, 120),
        "one-pixel": (synth.gaussians(5, 1, 1, seed=85), opac(5, 86), 1, 1),
        "empty": (np.zeros((0, 8), np.float32), np.zeros(0, np.float32), 33, 17),
    }


CASES = cases()


def check(g, o, A, rtol, what):
    bad = np.abs(g - o) > rtol * A + 1e-30
    if bad.any():
        i = np.argmax(np.abs(g - o) / (A + 1e-300))
        raise AssertionError(f"{what}: {bad.sum()} values off; worst gpu {g.flat[i]} oracle "
                             f"{o.flat[i]} A {A.flat[i]} at {np.unravel_index(i, g.shape)}")


@pytest.fixture(scope="module")
def gi():
    import paper_2403_08551_amd as P
    ctx = P.Context(0)
    yield ctx
    ctx.close()


@pytest.fixture(params=[1, 2, 3], ids=["radix", "one-pass", "rows"])
def mode(request, gi):
    import paper_2403_08551_amd as P
    gi.set_option(P._lib.GI_OPT_BINNING, request.param)
    yield request.param
    gi.set_option(P._lib.GI_OPT_BINNING, 0)


@pytest.mark.parametrize("blend_mode", ["sum", "alpha"])
@pytest.mark.parametrize("name", list(CASES))
def test_render_matches_oracle(gi, name, blend_mode, mode):
    p, o, h, w = CASES[name]
    img = host(gi.render_opacity(dev(p), dev(o), h, w, blend_mode))
    want, A = blend.render_blend(p, o, h, w, blend_mode, with_abs=True)
    check(img, want, A, FWD_RTOL, f"{name} {blend_mode}")


@pytest.mark.parametrize("blend_mode", ["sum", "alpha"])
@pytest.mark.parametrize("name", list(CASES))
def test_grad_matches_oracle(gi, name, blend_mode, mode):
    p, o, h, w = CASES[name]
    G = synth.upstream_gradient(h, w, 87)
    dp, do = gi.grad_opacity(dev(p), dev(o), h, w, dev(G), blend_mode)
    dp, do = host(dp), host(do)
    if p.shape[0] == 0:
        assert dp.shape == (0, 8) and do.shape == (0,)
        return
    wp, wo, ap, ao = blend.grads_blend(p, o, h, w, G, blend_mode, with_abs=True)
    check(dp, wp, ap, GRAD_RTOL, f"{name} {blend_mode} params")
    check(do, wo, ao, GRAD_RTOL, f"{name} {blend_mode} opacity")


def test_sum_equals_render_of_merged_colours_bitwise(gi):
    p, o, h, w = CASES["plain-256x256"]
    merged = p.copy()
    merged[:, 5:8] = p[:, 5:8] * o[:, None]  # float32 products, as the projection forms them
    a = host(gi.render_opacity(dev(p), dev(o), h, w, "sum"))
    np.testing.assert_array_equal(a, host(gi.render(dev(merged), h, w)))


def test_alpha_blending_is_deterministic_and_order_dependent(gi):
    p, o, h, w = CASES["plain-256x256"]
    G = dev(synth.upstream_gradient(h, w, 88))
    a1 = host(gi.render_opacity(dev(p), dev(o), h, w, "alpha"))
    a2 = host(gi.render_opacity(dev(p), dev(o), h, w, "alpha"))
    np.testing.assert_array_equal(a1, a2)
    g1 = [host(t) for t in gi.grad_opacity(dev(p), dev(o), h, w, G, "alpha")]
    g2 = [host(t) for t in gi.grad_opacity(dev(p), dev(o), h, w, G, "alpha")]
    np.testing.assert_array_equal(g1[0], g2[0])
    np.testing.assert_array_equal(g1[1], g2[1])
    rev = host(gi.render_opacity(dev(p[::-1]), dev(o[::-1]), h, w, "alpha"))
    want, A = blend.render_blend(p[::-1], o[::-1], h, w, "alpha", with_abs=True)
    check(rev, want, A, FWD_RTOL, "reversed order")
    assert np.abs(rev - a1).max() > 1e-3


def test_rotation_scale_alpha(gi):
    import paper_2403_08551_amd as P
    h, w = 80, 96
    p = synth.gaussians_rs(500, h, w, seed=89)
    o = opac(500, 90)
    G = synth.upstream_gradient(h, w, 91)
    ctx = P.Context(0, covariance="rotation_scale")
    try:
        img = host(ctx.render_opacity(dev(p), dev(o), h, w, "alpha"))
        want, A = blend.render_blend(p, o, h, w, "alpha", cov="rs", with_abs=True)
        check(img, want, A, FWD_RTOL, "rs alpha")
        dp, do = ctx.grad_opacity(dev(p), dev(o), h, w, dev(G), "alpha")
        wp, wo, ap, ao = blend.grads_blend(p, o, h, w, G, "alpha", cov="rs", with_abs=True)
        check(host(dp), wp, ap, GRAD_RTOL, "rs alpha params")
        check(host(do), wo, ao, GRAD_RTOL, "rs alpha opacity")
    finally:
        ctx.close()


def test_kodak_size_alpha_sampled(gi):
    wl = synth.kodak_like(70_000)
    p = wl.params()
    o = opac(p.shape[0], 92)
    img = host(gi.render_opacity(dev(p), dev(o), wl.height, wl.width, "alpha"))
    # sampled pixels: blend the pixel's tile list in order with the oracle's float64 arithmetic
    ranges, ids = ref.tile_lists(p, wl.height, wl.width)
    inv = ref.inverse_covariance(p)
    pf = p.astype(np.float64)
    of = o.astype(np.float64)
    tw, _ = ref.grid_tiles(wl.height, wl.width)
    rng = np.random.default_rng(93)
    for y, x in zip(rng.integers(0, wl.height, 48), rng.integers(0, wl.width, 48)):
        a, b = ranges[(y // 16) * tw + x // 16]
        T, C, A = 1.0, np.zeros(3), np.zeros(3)
        for n in ids[a:b]:
            dx, dy = x + 0.5 - pf[n, 0], y + 0.5 - pf[n, 1]
            s = 0.5 * (inv[0][n] * dx * dx + 2 * inv[1][n] * dx * dy + inv[2][n] * dy * dy)
            al = min(of[n] * np.exp(-s), 0.99)
            C += pf[n, 5:8] * al * T
            A += np.abs(pf[n, 5:8]) * abs(al * T)
            T *= 1 - al
        assert np.all(np.abs(img[y, x] - C) <= FWD_RTOL * A + 1e-30), (y, x, img[y, x], C)


@pytest.mark.parametrize("blend_mode", ["sum", "alpha"])
def test_fit_steps_match_oracle(gi, blend_mode):
    import paper_2403_08551_amd as P
    h, w = 96, 128
    p0 = synth.gaussians(700, h, w, seed=94, l_lo=0.6, l_hi=6.0)
    o0 = opac(700, 95, 0.2, 0.9)
    T = synth.target_noise_rects(h, w, seed=96)
    hp = dict(ref.DEFAULT_ADAM)
    hp32 = {k: float(np.float32(v)) for k, v in hp.items()}
    lr = np.array([hp32["lr_mu"]] * 2 + [hp32["lr_l"]] * 3 + [hp32["lr_c"]] * 3)
    pd, od = dev(p0), dev(o0)
    md, vd = torch.zeros_like(pd), torch.zeros_like(pd)
    mo, vo = torch.zeros_like(od), torch.zeros_like(od)
    step = torch.ones(1, dtype=torch.int32, device="cuda")
    img = torch.empty(h, w, 3, device="cuda")
    loss = torch.empty(1, device="cuda")
    Mp, Vp = np.zeros_like(p0, np.float64), np.zeros_like(p0, np.float64)
    Mo, Vo = np.zeros(700), np.zeros(700)
    for t in range(1, 4):
        pin, oin = host(pd).copy(), host(od).copy()
        gi.fit_step_opacity(pd, od, md, vd, mo, vo, dev(T), step, blend_mode, P.AdamConfig(**hp),
                            image_out=img, loss_out=loss)
        want, A = blend.render_blend(pin, oin, h, w, blend_mode, with_abs=True)
        check(host(img), want, A, FWD_RTOL, f"step {t} image")
        np.testing.assert_allclose(host(loss)[0], ref.mse(want, T), rtol=1e-5)
        gp, go, ap, ao = blend.grads_blend(pin, oin, h, w, ref.mse_grad(want, T), blend_mode,
                                           with_abs=True)
        po, Mp, Vp = ref.adam_step(pin, Mp, Vp, gp, t, hp32)
        oo, Mo, Vo = blend.adam_opacity_step(oin, Mo, Vo, go, t, hp32)
        got_p, got_o = host(pd), host(od)
        firm = np.abs(gp) > 10 * GRAD_RTOL * ap + 1e-20
        tol = 1e-4 * lr + 1e-6 * np.abs(po)
        assert np.all(np.abs(got_p - po)[firm] <= np.broadcast_to(tol, po.shape)[firm]), t
        assert np.all(np.abs(got_p - po) <= 2.0 * lr + 1e-6 * np.abs(po))
        firm_o = np.abs(go) > 10 * GRAD_RTOL * ao + 1e-20
        tol_o = 1e-4 * hp32["lr_c"] + 1e-6 * np.abs(oo)
        assert np.all(np.abs(got_o - oo)[firm_o] <= tol_o[firm_o]), t
        assert np.all(np.abs(got_o - oo) <= 2.0 * hp32["lr_c"] + 1e-6)
        assert firm.mean() > 0.9 and firm_o.mean() > 0.9
    assert int(host(step)[0]) == 4


@pytest.mark.parametrize("blend_mode", ["sum", "alpha"])
def test_fit_step_gradients_element_by_element(gi, blend_mode):
    # Adam with beta1 = beta2 = 0, eps = 1: the first moments of records and opacities are the
    # fused kernel's gradients, compared element by element with the oracle's at the gradient
    # bar (plus what the forward bar allows through dL/dC)
    import paper_2403_08551_amd as P
    h, w = 96, 128
    p0 = synth.gaussians(700, h, w, seed=97, l_lo=0.6, l_hi=6.0)
    o0 = opac(700, 98, 0.2, 0.9)
    T = synth.target_noise_rects(h, w, seed=99)
    want, A = blend.render_blend(p0, o0, h, w, blend_mode, with_abs=True)
    G = ref.mse_grad(want, T)
    gp, go, ap, ao = blend.grads_blend(p0, o0, h, w, G, blend_mode, with_abs=True)
    Gp = (2.0 * pu.FWD_RTOL / (3.0 * h * w)) * A
    _, _, app, aop = blend.grads_blend(p0, o0, h, w, Gp, blend_mode, with_abs=True)
    bp = pu.GRAD_RTOL * ap + app + 1e-30
    bo = pu.GRAD_RTOL * ao + aop + 1e-30
    hp = pu.linear_hp(pu.lr_for(p0, bp, [0, 1]), pu.lr_for(p0, bp, [2, 3, 4]),
                      pu.lr_for(p0, bp, [5, 6, 7]))
    pd, od = dev(p0), dev(o0)
    md, vd = torch.zeros_like(pd), torch.zeros_like(pd)
    mo, vo = torch.zeros_like(od), torch.zeros_like(od)
    step = torch.ones(1, dtype=torch.int32, device="cuda")
    img = torch.empty(h, w, 3, device="cuda")
    gi.fit_step_opacity(pd, od, md, vd, mo, vo, dev(T), step, blend_mode, P.AdamConfig(**hp),
                        image_out=img)
    check(host(img), want, A, FWD_RTOL, "image")
    pu.assert_gradient(host(md), gp, bp, f"{blend_mode} record gradients")
    pu.assert_gradient(host(mo), go, bo, f"{blend_mode} opacity gradients")
    lr = np.array([hp["lr_mu"]] * 2 + [hp["lr_l"]] * 3 + [hp["lr_c"]] * 3)
    pu.assert_linear_step(p0, host(pd), gp, bp, lr, f"{blend_mode} linear step")
