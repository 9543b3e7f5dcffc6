"""Pins of the opacity-variant oracle (Sec. 3.2, Eqs. rasterization1-3) against closed forms, a
library density, the accumulated-summation oracle, the small-alpha limit and finite
differences.  CPU only."""
import math

import numpy as np
import pytest

import synth
from oracle import blend, ref


def opac(n, seed, lo=0.05, hi=0.95):
    return np.random.default_rng(seed).uniform(lo, hi, n).astype(np.float32)


def test_single_gaussian_is_colour_times_clamped_alpha():
    from scipy.stats import multivariate_normal
    h, w = 40, 40
    p = np.array([[20.3, 19.6, 3.0, 1.0, 2.0, 0.7, -0.2, 0.4]], np.float32)
    for o in (0.6, 2.5):
        img = blend.render_blend(p, np.array([o], np.float32), h, w, "alpha")
        q = p.astype(np.float64)[0]
        L = np.array([[q[2], 0], [q[3], q[4]]])
        ys, xs = np.meshgrid(np.arange(h) + 0.5, np.arange(w) + 0.5, indexing="ij")
        e = multivariate_normal(q[:2], L @ L.T).pdf(np.stack([xs, ys], -1)) * 2 * math.pi * q[2] * q[4]
        rect, _ = ref.tile_rects(p, h, w)
        mask = np.zeros((h, w), bool)
        tx0, ty0, tx1, ty1 = rect[0]
        mask[ty0 * 16:(ty1 + 1) * 16, tx0 * 16:(tx1 + 1) * 16] = True
        al = np.minimum(np.float32(o) * e, 0.99) * mask
        np.testing.assert_allclose(img, al[..., None] * q[5:8], rtol=1e-12, atol=1e-15)
        if o > 1:
            assert np.isclose(img[..., 0].max(), 0.99 * q[5])


def test_two_gaussians_blend_in_index_order():
    h, w = 32, 32
    p = np.array([[14.0, 15.0, 4.0, 0.5, 3.0, 1.0, 0.0, 0.5],
                  [18.0, 16.0, 3.0, -1.0, 4.0, 0.0, 1.0, 0.25]], np.float32)
    o = np.array([0.8, 0.7], np.float32)
    a = blend.render_blend(p, o, h, w, "alpha")
    b = blend.render_blend(p[::-1], o[::-1], h, w, "alpha")
    e = [ref.render_culled(np.concatenate([p[i:i + 1, :5], [[1, 1, 1]]], 1).astype(np.float32),
                           h, w)[..., 0] for i in range(2)]
    a1, a2 = o[0] * e[0], o[1] * e[1]
    c1, c2 = p[0, 5:8].astype(np.float64), p[1, 5:8].astype(np.float64)
    want_a = a1[..., None] * c1 + (a2 * (1 - a1))[..., None] * c2
    want_b = a2[..., None] * c2 + (a1 * (1 - a2))[..., None] * c1
    np.testing.assert_allclose(a, want_a, rtol=1e-12, atol=1e-15)
    np.testing.assert_allclose(b, want_b, rtol=1e-12, atol=1e-15)
    assert np.abs(a - b).max() > 0.05  # order matters for alpha blending ...
    s1 = blend.render_blend(p, o, h, w, "sum")
    s2 = blend.render_blend(p[::-1], o[::-1], h, w, "sum")
    np.testing.assert_allclose(s1, s2, rtol=1e-14)  # ... and not for the summation


def test_summation_with_opacity_equals_merged_colours():
    w = synth.plain_256(500)
    p = w.params()
    o = opac(p.shape[0], 3)
    merged = p.copy()
    merged[:, 5:8] = (p[:, 5:8].astype(np.float64) * o[:, None].astype(np.float64))
    got = blend.render_blend(p, o, w.height, w.width, "sum")
    # merged colours rounded to float32 by ref: compare within that rounding
    want, A = ref.render_culled(merged, w.height, w.width, with_abs=True)
    assert np.all(np.abs(got - want) <= 1e-7 * A + 1e-300)


def test_small_alpha_limit_is_the_summation():
    p = synth.gaussians(60, 48, 48, seed=4)
    for eps in (1e-3, 1e-4):
        o = np.full(60, eps, np.float32)
        a = blend.render_blend(p, o, 48, 48, "alpha")
        s, A = blend.render_blend(p, o, 48, 48, "sum", with_abs=True)
        # the difference is second order: |a - s| <= (sum alpha)^2 max |c|
        cnt = blend.render_blend(p, o, 48, 48, "sum", with_abs=True)[1].sum(-1) / 3
        assert np.all(np.abs(a - s) <= (A.max(-1) / 1.0 + cnt)[..., None] ** 2 + 1e-15)
        assert np.abs(a - s).max() <= 60 * 60 * eps * eps


@pytest.mark.parametrize("mode,cov", [("alpha", "chol"), ("sum", "chol"), ("alpha", "rs")])
def test_gradients_match_finite_differences(mode, cov):
    h, w = 30, 34
    if cov == "chol":
        p = synth.gaussians(8, h, w, seed=11, l_lo=1.5, l_hi=6.0)
    else:
        p = synth.gaussians_rs(8, h, w, seed=11, s_lo=1.5, s_hi=6.0)
    o = opac(8, 12)
    o[2] = 1.6  # clamped near its centre
    G = synth.upstream_gradient(h, w, 13)
    dp, do = blend.grads_blend(p, o, h, w, G, mode, cov)
    fp, fo = blend.fd_grads_blend(p, o, h, w, G, mode, cov)
    scale = np.abs(dp).max(axis=0) + 1e-12
    assert np.all(np.abs(dp - fp) <= 1e-6 * scale + 1e-9), (dp - fp) / scale
    np.testing.assert_allclose(do, fo, rtol=1e-6, atol=1e-9 * np.abs(do).max())


def test_alpha_gradient_of_the_front_gaussian_sees_what_it_hides():
    # one pixel column of two fully overlapping isotropic Gaussians: dC/dalpha_1 = c1 - alpha2 c2
    h, w = 16, 16
    p = np.array([[8.5, 8.5, 40.0, 0.0, 40.0, 1.0, 0.0, 0.0],
                  [8.5, 8.5, 40.0, 0.0, 40.0, 0.5, 0.0, 0.0]], np.float32)
    o = np.array([0.3, 0.6], np.float32)
    G = np.zeros((h, w, 3))
    G[8, 8, 0] = 1.0
    dp, do = blend.grads_blend(p, o, h, w, G, "alpha")
    e = 1.0  # the pixel centre is the mean
    a1, a2 = 0.3 * e, 0.6 * e
    np.testing.assert_allclose(do[0], e * (1.0 - a2 * 0.5), rtol=1e-6)
    np.testing.assert_allclose(do[1], e * (1 - a1) * 0.5, rtol=1e-6)
    np.testing.assert_allclose(dp[0, 5], a1, rtol=1e-6)
    np.testing.assert_allclose(dp[1, 5], a2 * (1 - a1), rtol=1e-6)


def test_opacity_adam_matches_the_colour_slot_update():
    # the opacity update is the colour-slot update of ref.adam_step run on the same numbers
    rng = np.random.default_rng(14)
    o = rng.uniform(0.1, 0.9, 50)
    g = rng.normal(size=50)
    m = rng.normal(size=50) * 0.01
    v = rng.uniform(0, 0.01, 50)
    got = blend.adam_opacity_step(o, m, v, g, 3)
    P = np.zeros((50, 8))
    P[:, 5] = o
    G = np.zeros((50, 8))
    G[:, 5] = g
    M = np.zeros((50, 8))
    M[:, 5] = m
    V = np.zeros((50, 8))
    V[:, 5] = v
    want = ref.adam_step(P, M, V, G, 3, dict(ref.DEFAULT_ADAM, l_min=0.0))
    for a, b in zip(got, want):
        np.testing.assert_allclose(a, b[:, 5], rtol=1e-15)
