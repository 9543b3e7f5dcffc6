"""Pins of the FP64 oracle against facts that do not come from the oracle itself: closed forms,
exact symmetries, library routines, finite differences, exact rational brute force and the
numbers the paper prints.  CPU only."""
import json
import math
import os
from fractions import Fraction

import numpy as np
import pytest

import synth
from oracle import cref, ref

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def one(mx, my, l1, l2, l3, c=(1.0, 1.0, 1.0)):
    return np.array([[mx, my, l1, l2, l3, *c]], np.float32)


# ----------------------------------------------------------------- the record (Sec. 3.2, Table 3)

def test_record_size_matches_paper_tables():
    g = json.load(open(os.path.join(GOLDEN, "paper_record_sizes.json")))
    assert synth.PARAMS_PER_GAUSSIAN == g["params_per_gaussian_merged"]
    n = g["table3_gaussians"]
    assert n * synth.PARAMS_PER_GAUSSIAN == g["table3_params_k_merged"] * 1000
    assert n * g["params_per_gaussian_basic"] == g["table3_params_k_unmerged"] * 1000
    per_3dgs = g["table3_params_k_3dgs"] * 1000 // n
    assert per_3dgs / synth.PARAMS_PER_GAUSSIAN == g["compression_ratio_vs_3dgs_merged"]
    assert math.floor(per_3dgs / g["params_per_gaussian_basic"] * 2) / 2 == \
        g["compression_ratio_vs_3dgs_basic"]


# ----------------------------------------------------------------- forward closed forms

@pytest.mark.parametrize("fn", ["full", "culled"])
def test_peak_equals_colour(fn):
    p = one(40.5, 33.5, 3.0, 0.7, 2.0, (0.25, -1.5, 2.0))
    img = ref.render_full(p, 80, 80) if fn == "full" else ref.render_culled(p, 80, 80)
    np.testing.assert_array_equal(img[33, 40], [0.25, -1.5, 2.0])
    assert np.all(np.abs(img) <= np.abs(img[33, 40]) + 1e-15)


@pytest.mark.parametrize("l", [(1.0, 0.0, 1.0), (2.0, 0.7, 1.3), (3.0, -1.25, 2.5), (1.5, 0.5, 4.0)])
def test_grid_sum_is_gaussian_integral(l):
    # Poisson summation: the pixel-grid sum of exp(-1/2 d^T S^-1 d) equals 2 pi sqrt(det S) up to
    # terms of order exp(-2 pi^2 lambda_min), below 1e-8 when lambda_min >= 1 px^2.
    l1, l2, l3 = l
    lam_min = np.linalg.eigvalsh(np.array([[l1 * l1, l1 * l2], [l1 * l2, l2 * l2 + l3 * l3]]))[0]
    assert lam_min >= 0.99
    c = (0.3, 1.0, -2.0)
    p = one(64.25, 63.6, l1, l2, l3, c)
    img = ref.render_full(p, 128, 128)
    want = 2 * math.pi * abs(l1 * l3) * np.array(c)
    np.testing.assert_allclose(img.sum(axis=(0, 1)), want, rtol=1e-7)


def test_forward_matches_library_density():
    # e^{-sigma} = 2 pi sqrt(det Sigma) * N(p; mu, Sigma), with the normal density from scipy
    # (eigen-decomposition based, independent of the oracle's inverse).  Dense E @ Cmat.
    from scipy.stats import multivariate_normal
    p = synth.gaussians(12, 24, 20, seed=3, l_lo=1.0, l_hi=5.0)
    h, w = 24, 20
    ys, xs = np.meshgrid(np.arange(h) + 0.5, np.arange(w) + 0.5, indexing="ij")
    pts = np.stack([xs.ravel(), ys.ravel()], axis=1)
    E = np.zeros((h * w, p.shape[0]))
    for n, q in enumerate(p.astype(np.float64)):
        S = np.array([[q[2] ** 2, q[2] * q[3]], [q[2] * q[3], q[3] ** 2 + q[4] ** 2]])
        E[:, n] = multivariate_normal(mean=q[:2], cov=S).pdf(pts) * 2 * math.pi * abs(q[2] * q[4])
    want = (E @ p[:, 5:8].astype(np.float64)).reshape(h, w, 3)
    np.testing.assert_allclose(ref.render_full(p, h, w), want, rtol=1e-12, atol=1e-300)


def _rot90_params(p, side):
    # rotate by +90 degrees about the image centre: d -> R d with R = [[0, -1], [1, 0]];
    # Sigma' = R Sigma R^T; the Cholesky factor is rebuilt exactly for Pythagorean entries.
    q = p.astype(np.float64).copy()
    ctr = side / 2.0
    q[:, 0] = ctr - (p[:, 1] - ctr)
    q[:, 1] = ctr + (p[:, 0] - ctr)
    for n in range(p.shape[0]):
        l1, l2, l3 = (float(v) for v in p[n, 2:5])
        s00, s01, s11 = l2 * l2 + l3 * l3, -l1 * l2, l1 * l1
        a = math.sqrt(s00)
        b = s01 / a
        c = math.sqrt(s11 - b * b)
        q[n, 2:5] = (a, b, c)
    out = q.astype(np.float32)
    assert np.array_equal(out.astype(np.float64), q), "test needs exactly representable rotations"
    return out


@pytest.mark.parametrize("fn", ["full", "culled"])
def test_exact_rotation_by_90_degrees(fn):
    # l vectors from Pythagorean triples so that the rotated Cholesky factor is exact
    rng = np.random.default_rng(11)
    shapes = [(5.0, 3.0, 4.0), (2.5, -1.5, 2.0), (1.25, 0.75, 1.0), (4.0, 0.0, 1.5),
              (10.0, 6.0, 8.0), (1.0, 0.0, 3.0)]
    side = 64
    n = 24
    p = np.zeros((n, 8), np.float32)
    p[:, 0] = rng.integers(0, side * 4, n) / 4.0
    p[:, 1] = rng.integers(0, side * 4, n) / 4.0
    p[:, 2:5] = np.array([shapes[i % len(shapes)] for i in range(n)])
    p[:, 5:8] = rng.uniform(-1, 1, (n, 3))
    q = _rot90_params(p, side)
    render = ref.render_full if fn == "full" else ref.render_culled
    a = render(p, side, side)
    b = render(q, side, side)
    np.testing.assert_allclose(b, np.rot90(a, -1, axes=(0, 1)), rtol=1e-12, atol=1e-14)


def test_rotation_invariance_of_peak_and_integral():
    for theta in np.linspace(0.1, 3.0, 5):
        R = np.array([[math.cos(theta), -math.sin(theta)], [math.sin(theta), math.cos(theta)]])
        S = R @ np.diag([9.0, 2.25]) @ R.T
        L = np.linalg.cholesky(S)
        p = one(70.5, 70.5, L[0, 0], L[1, 0], L[1, 1], (1.0, 2.0, 3.0))
        img = ref.render_full(p, 140, 140)
        np.testing.assert_allclose(img[70, 70], [1, 2, 3], rtol=0, atol=0)
        pf = p.astype(np.float64)
        want = 2 * math.pi * abs(pf[0, 2] * pf[0, 4]) * np.array([1.0, 2.0, 3.0])
        np.testing.assert_allclose(img.sum(axis=(0, 1)), want, rtol=1e-7)
        np.testing.assert_allclose(want / np.array([1.0, 2.0, 3.0]), 2 * math.pi * 4.5, rtol=1e-6)


def test_permutation_invariance_and_linearity():
    p = synth.gaussians(300, 70, 90, seed=5)
    a = ref.render_culled(p, 70, 90)
    perm = np.random.default_rng(1).permutation(300)
    b = ref.render_culled(p[perm], 70, 90)
    np.testing.assert_allclose(b, a, rtol=1e-13)
    q = p.copy()
    q[:, 5:8] *= -2.0
    np.testing.assert_allclose(ref.render_culled(q, 70, 90), -2.0 * a, rtol=1e-13)


# ----------------------------------------------------------------- the tile rule

def _exact_radius(l1, l2, l3):
    l1, l2, l3 = Fraction(float(l1)), Fraction(float(l2)), Fraction(float(l3))
    a, b, c = l1 * l1, l1 * l2, l2 * l2 + l3 * l3
    r = 0
    while True:  # least r with r^2 / 9 >= lambda_max, decided in exact rationals
        s = Fraction(r * r, 9)
        if 2 * s >= a + c and (s - a) * (s - c) >= b * b:
            return r
        r += 1


def test_radius_against_exact_rationals():
    p = synth.gaussians(400, 100, 100, seed=9, l_lo=0.5, l_hi=32.0)
    p[:5, 2:5] = [[1, 0, 1], [2, 0, 2], [1, 0, 3], [3, 4, 0.5], [0.5, 0.5, 0.5]]
    r = ref.radius(p)
    for n in range(p.shape[0]):
        assert r[n] == _exact_radius(*p[n, 2:5]), n
    assert r[0] == 3 and r[1] == 6 and r[2] == 9


def test_tile_membership_brute_force():
    h, w = 45, 70   # ragged: neither side a multiple of 16
    p = synth.gaussians(150, h, w, seed=2, l_lo=0.5, l_hi=12.0)
    p[:4, 0] = [-30.0, 200.0, 35.0, 0.0]   # off-image and on-edge means
    p[:4, 1] = [10.0, 10.0, -40.0, 0.0]
    p[4] = [np.nan, 1, 1, 0, 1, 1, 1, 1]
    p[5, 2] = 0.0
    rect, count = ref.tile_rects(p, h, w)
    tw, th = ref.grid_tiles(h, w)
    rads = [_exact_radius(*q[2:5]) if np.all(np.isfinite(q)) and q[2] != 0 and q[4] != 0 else None
            for q in p]
    for n in range(p.shape[0]):
        if rads[n] is None:
            assert count[n] == 0
            continue
        r = rads[n]
        mx, my = Fraction(float(p[n, 0])), Fraction(float(p[n, 1]))
        members = set()
        for ty in range(th):
            for tx in range(tw):
                # the tile's x-range [16 tx, 16 tx + 16) meets the closed interval [mx - r, mx + r]
                if (16 * tx <= mx + r and mx - r < 16 * tx + 16
                        and 16 * ty <= my + r and my - r < 16 * ty + 16):
                    members.add((tx, ty))
        got = set()
        if count[n]:
            tx0, ty0, tx1, ty1 = rect[n]
            got = {(x, y) for y in range(ty0, ty1 + 1) for x in range(tx0, tx1 + 1)}
        assert got == members, n
        assert count[n] == len(members)
    ranges, ids = ref.tile_lists(p, h, w)
    for t in range(tw * th):
        tx, ty = t % tw, t // tw
        want = [n for n in range(p.shape[0]) if count[n] and rect[n, 0] <= tx <= rect[n, 2]
                and rect[n, 1] <= ty <= rect[n, 3]]
        assert list(ids[ranges[t, 0]:ranges[t, 1]]) == want


def test_culling_drops_only_far_pairs():
    # every dropped (pixel, Gaussian) pair has sigma > 4.5, so full - culled is bounded by
    # e^{-4.5} sum |c'| over the dropped Gaussians
    h, w = 48, 64
    p = synth.gaussians(60, h, w, seed=4, l_lo=1.0, l_hi=8.0)
    full = ref.render_full(p, h, w)
    cull = ref.render_culled(p, h, w)
    rect, count = ref.tile_rects(p, h, w)
    i00, i01, i11 = ref.inverse_covariance(p)
    bound = np.zeros((h, w))
    pf = p.astype(np.float64)
    ys, xs = np.meshgrid(np.arange(h) + 0.5, np.arange(w) + 0.5, indexing="ij")
    tyy, txx = np.meshgrid(np.arange(h) // 16, np.arange(w) // 16, indexing="ij")
    for n in range(p.shape[0]):
        inside = ((txx >= rect[n, 0]) & (txx <= rect[n, 2]) & (tyy >= rect[n, 1])
                  & (tyy <= rect[n, 3]))
        dx, dy = xs - pf[n, 0], ys - pf[n, 1]
        sig = 0.5 * (i00[n] * dx * dx + 2 * i01[n] * dx * dy + i11[n] * dy * dy)
        assert np.all(sig[~inside] > 4.5)
        bound += np.where(inside, 0.0, np.abs(pf[n, 5:8]).sum())
    diff = np.abs(full - cull).max(axis=2)
    assert np.all(diff <= math.exp(-4.5) * bound + 1e-15)
    assert diff.max() > 0


# ----------------------------------------------------------------- gradients (App. A)

@pytest.mark.parametrize("culled", [True, False])
def test_gradients_match_finite_differences(culled):
    h, w = 36, 40
    p = synth.gaussians(7, h, w, seed=21, l_lo=1.5, l_hi=6.0)
    p[:, 5:8] -= 0.5
    G = synth.upstream_gradient(h, w, 8)
    an = ref.grads(p, h, w, G, culled=culled)
    fd = ref.fd_grads(p, h, w, G, culled=culled)
    scale = np.abs(an).max(axis=0) + 1e-12
    assert np.all(np.abs(an - fd) <= 1e-6 * scale + 1e-9 * np.abs(an).max()), (an - fd) / scale


def test_local_finite_differences_equal_global_ones():
    h, w = 40, 44
    p = synth.gaussians(9, h, w, seed=23, l_lo=1.5, l_hi=6.0)
    G = synth.upstream_gradient(h, w, 6)
    glob = ref.fd_grads(p, h, w, G, which=[2, 5])
    for n in (2, 5):
        np.testing.assert_allclose(ref.fd_local(p, h, w, G, n), glob[n], rtol=1e-6, atol=1e-9)


def test_gradient_closed_forms_for_one_gaussian():
    # S = sum over pixels of C^k for one Gaussian far from the border: S = 2 pi l1 l3 c^k
    # (Poisson error negligible), so dS/dc = 2 pi l1 l3, dS/dl1 = 2 pi l3 c, dS/dl3 = 2 pi l1 c,
    # dS/dl2 = 0, dS/dmu = 0.
    l1, l2, l3, c = 2.0, 0.6, 1.5, 0.75
    p = one(60.3, 59.7, l1, l2, l3, (c, 0.0, 0.0))
    G = np.zeros((120, 120, 3))
    G[:, :, 0] = 1.0
    d = ref.grads(p, 120, 120, G, culled=False)[0]
    two_pi = 2 * math.pi
    np.testing.assert_allclose(d[5], two_pi * l1 * l3, rtol=1e-7)
    np.testing.assert_allclose(d[2], two_pi * l3 * c, rtol=1e-7)
    np.testing.assert_allclose(d[4], two_pi * l1 * c, rtol=1e-7)
    assert abs(d[3]) < 1e-7 and abs(d[0]) < 1e-7 and abs(d[1]) < 1e-7
    assert d[6] == 0 and d[7] == 0


def test_gradients_match_autograd_float64():
    # reverse-mode autodiff of the same sum, written as plain torch float64 ops on the CPU
    torch = pytest.importorskip("torch")
    h, w = 30, 34
    p = synth.gaussians(9, h, w, seed=31, l_lo=1.0, l_hi=6.0)
    G = synth.upstream_gradient(h, w, 2)
    rect, count = ref.tile_rects(p, h, w)
    pt = torch.tensor(p.astype(np.float64), requires_grad=True)
    ys, xs = torch.meshgrid(torch.arange(h, dtype=torch.float64) + 0.5,
                            torch.arange(w, dtype=torch.float64) + 0.5, indexing="ij")
    img = torch.zeros(h, w, 3, dtype=torch.float64)
    for n in range(p.shape[0]):
        L = torch.stack([torch.stack([pt[n, 2], torch.zeros((), dtype=torch.float64)]),
                         torch.stack([pt[n, 3], pt[n, 4]])])
        S = L @ L.T
        d = torch.stack([xs - pt[n, 0], ys - pt[n, 1]], dim=-1)
        sol = torch.linalg.solve(S, d.reshape(-1, 2).T).T.reshape(h, w, 2)
        e = torch.exp(-0.5 * (d * sol).sum(-1))
        mask = torch.zeros(h, w, dtype=torch.float64)
        tx0, ty0, tx1, ty1 = rect[n]
        mask[ty0 * 16:(ty1 + 1) * 16, tx0 * 16:(tx1 + 1) * 16] = 1.0
        img = img + (mask * e)[..., None] * pt[n, 5:8]
    (img * torch.tensor(G, dtype=torch.float64)).sum().backward()
    np.testing.assert_allclose(ref.grads(p, h, w, G), pt.grad.numpy(), rtol=1e-10, atol=1e-12)


def test_adjoint_dot_product():
    # <G, J v> = <J^T G, v> with J v from a float64 central difference along v
    h, w = 32, 32
    p = synth.gaussians(6, h, w, seed=41, l_lo=1.5, l_hi=5.0)
    G = synth.upstream_gradient(h, w, 3)
    v = np.random.default_rng(0).normal(size=p.shape)
    eps = 1e-6
    rect0, _ = ref.tile_rects(p, h, w)
    plus = ref._render64(p.astype(np.float64) + eps * v, h, w, True, rect0, 0)
    minus = ref._render64(p.astype(np.float64) - eps * v, h, w, True, rect0, 0)
    jv = (plus - minus) / (2 * eps)
    lhs = np.sum(G * jv)
    rhs = np.sum(ref.grads(p, h, w, G) * v)
    np.testing.assert_allclose(lhs, rhs, rtol=1e-7)


# ----------------------------------------------------------------- loss and optimiser

def test_mse_and_gradient_match_torch():
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(3)
    a, b = rng.normal(size=(9, 7, 3)), rng.normal(size=(9, 7, 3))
    ta = torch.tensor(a, requires_grad=True)
    loss = torch.nn.functional.mse_loss(ta, torch.tensor(b))
    loss.backward()
    np.testing.assert_allclose(ref.mse(a, b), loss.item(), rtol=1e-14)
    np.testing.assert_allclose(ref.mse_grad(a, b), ta.grad.numpy(), rtol=1e-14)


def test_adam_matches_torch_optimizer():
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(4)
    p0 = synth.gaussians(20, 32, 32, seed=1).astype(np.float64)
    hp = dict(ref.DEFAULT_ADAM, l_min=0.0)
    groups = [(slice(0, 2), hp["lr_mu"]), (slice(2, 5), hp["lr_l"]), (slice(5, 8), hp["lr_c"])]
    tens = [torch.tensor(p0[:, s].copy(), requires_grad=True) for s, _ in groups]
    opt = torch.optim.Adam([{"params": [t], "lr": lr} for t, (_, lr) in zip(tens, groups)],
                           betas=(hp["beta1"], hp["beta2"]), eps=hp["eps"])
    p, m, v = p0.copy(), np.zeros_like(p0), np.zeros_like(p0)
    for step in range(1, 5):
        g = rng.normal(size=p0.shape) * 10.0 ** rng.integers(-4, 2, size=p0.shape)
        for t, (s, _) in zip(tens, groups):
            t.grad = torch.tensor(g[:, s].copy())
        opt.step()
        p, m, v = ref.adam_step(p, m, v, g, step, hp)
        got = np.concatenate([t.detach().numpy() for t in tens], axis=1)
        np.testing.assert_allclose(p, got, rtol=1e-13, atol=1e-15)


def test_adam_first_step_closed_form_and_floor():
    p0 = np.array([[10.0, 10.0, 0.55, 0.1, -0.52, 0.5, 0.5, 0.5]])
    g = np.array([[1.0, -2.0, 3.0, 0.0, -4.0, 1e-3, -1e-3, 0.0]])
    hp = dict(ref.DEFAULT_ADAM)
    p, m, v = ref.adam_step(p0, np.zeros_like(p0), np.zeros_like(p0), g, 1, hp)
    lr = np.array([hp["lr_mu"]] * 2 + [hp["lr_l"]] * 3 + [hp["lr_c"]] * 3)
    step = lr * g / (np.abs(g) + hp["eps"])
    want = p0 - step
    np.testing.assert_allclose(p, want, rtol=1e-12)
    assert p[0, 2] == pytest.approx(0.54) and p[0, 4] == pytest.approx(-0.51)
    p2, _, _ = ref.adam_step(np.array([[0, 0, 0.5, 0, 0.5, 0, 0, 0.0]]), np.zeros((1, 8)),
                             np.zeros((1, 8)), np.array([[0, 0, 1.0, 0, 1.0, 0, 0, 0]]), 1, hp)
    assert p2[0, 2] == 0.5 and p2[0, 4] == 0.5


# ----------------------------------------------------------------- the two oracles agree

def test_c_oracle_matches_numpy_oracle():
    w = synth.plain_256()
    p = w.params()
    h, wd = w.height, w.width
    r1, c1 = ref.tile_rects(p, h, wd)
    r2, c2 = cref.tile_rects(p, h, wd)
    assert np.array_equal(r1, r2) and np.array_equal(c1, c2)
    g1, i1 = ref.tile_lists(p, h, wd)
    g2, i2 = cref.tile_lists(p, h, wd)
    assert np.array_equal(g1, g2) and np.array_equal(i1, i2)
    a1, A1 = ref.render_culled(p, h, wd, with_abs=True)
    a2, A2 = cref.render_culled(p, h, wd, with_abs=True)
    assert np.all(np.abs(a1 - a2) <= 1e-13 * A1)
    np.testing.assert_allclose(A1, A2, rtol=1e-13)
    pix = np.array([0, 1, 255, 256 * 100 + 37, 256 * 256 - 1])
    np.testing.assert_allclose(cref.render_pixels(p, h, wd, pix), a1.reshape(-1, 3)[pix],
                               rtol=1e-13, atol=1e-300)
    G = synth.upstream_gradient(h, wd, 5)
    d1, D1 = ref.grads(p, h, wd, G, with_abs=True)
    d2, D2 = cref.grads(p, h, wd, G, with_abs=True)
    assert np.all(np.abs(d1 - d2) <= 1e-12 * D1 + 1e-300)
    which = np.array([0, 17, 1999])
    np.testing.assert_allclose(cref.grads_subset(p, h, wd, G, which), d2[which], rtol=1e-13)
    # fit step: loss, image, gradients and the Adam update together
    T = w.target()
    hp = dict(ref.DEFAULT_ADAM)
    zeros = np.zeros((p.shape[0], 8))
    pc, mc, vc, loss, img = cref.fit_step(p, zeros, zeros, T, 1, hp, want_image=True)
    np.testing.assert_allclose(img, a1, rtol=1e-13, atol=1e-300)
    np.testing.assert_allclose(loss, ref.mse(a1, T), rtol=1e-12)
    gr = ref.grads(p, h, wd, ref.mse_grad(a1, T))
    pn, mn, vn = ref.adam_step(p, zeros, zeros, gr, 1, hp)
    np.testing.assert_allclose(mc, mn, rtol=1e-9, atol=1e-300)
    assert np.mean(np.abs(pc - pn) <= 1e-9 * np.abs(pn) + 1e-12) > 0.999


def test_degenerate_gaussians_are_inactive():
    p = np.array([[10, 10, 0, 0, 1, 1, 1, 1],
                  [10, 10, 1, 0, 0, 1, 1, 1],
                  [10, 10, np.inf, 0, 1, 1, 1, 1],
                  [np.nan, 10, 1, 0, 1, 1, 1, 1],
                  [10, 10, 1, 0, 1, np.nan, 1, 1],
                  [10, 10, 1e-9, 0, 1, 1, 1, 1],
                  [3e7, 10, 1, 0, 1, 1, 1, 1],
                  [10, 10, 1, 0, 1, 1, 1, 1]], np.float32)
    rect, count = ref.tile_rects(p, 32, 32)
    assert list(count) == [0, 0, 0, 0, 0, 0, 0, 1]
    img = ref.render_culled(p, 32, 32)
    np.testing.assert_allclose(img, ref.render_culled(p[7:], 32, 32), rtol=0)


# ----------------------------------------------------------------- rotation-scale covariance
# Record (mu_x, mu_y, s1, s2, theta, c0, c1, c2), Sigma = (R S)(R S)^T (Sec. 3.1, Eq. RSSR).

def rs_gaussians(n, h, w, seed):
    return synth.gaussians_rs(n, h, w, seed)


def test_rs_radius_is_the_least_integer_covering_three_sigma():
    # exact rational check: r is the least integer with r^2 >= 9 max(s1^2, s2^2)
    from fractions import Fraction
    rng = np.random.default_rng(17)
    s = np.concatenate([np.exp(rng.uniform(-3, 5, (300, 2))),
                        np.array([[2.0, 1.0], [1.0, 2.0], [1 / 3, 0.25], [4.0 / 3, -5.0 / 3],
                                  [0.5, 0.5], [7.0, -7.0], [2 ** -24, 2 ** -24]])])
    p = np.zeros((s.shape[0], 8), np.float32)
    p[:, 2:4] = s
    p[:, 4] = rng.uniform(-4, 4, s.shape[0])
    got = ref.radius(p, cov="rs")
    for q, r in zip(p.astype(np.float64), got):
        m = max(Fraction(q[2]) ** 2, Fraction(q[3]) ** 2)
        assert r * r >= 9 * m and (r == 0 or (r - 1) ** 2 < 9 * m), (q[2:4], r)
    # the eigenvalue rule agrees with the characteristic-polynomial rule on the trigonometric
    # covariance away from rounding ties
    s00, s01, s11 = ref.covariance(p, cov="rs")
    lam = 0.5 * (s00 + s11) + np.sqrt(0.25 * (s00 - s11) ** 2 + s01 ** 2)
    far = np.abs(3 * np.sqrt(lam) - np.round(3 * np.sqrt(lam))) > 1e-9
    assert far.sum() > 250
    np.testing.assert_array_equal(got[far], np.ceil(3 * np.sqrt(lam[far])).astype(np.int64))


def test_rs_forward_matches_library_density():
    from scipy.spatial.transform import Rotation
    from scipy.stats import multivariate_normal
    h, w = 22, 26
    p = rs_gaussians(10, h, w, 5)
    ys, xs = np.meshgrid(np.arange(h) + 0.5, np.arange(w) + 0.5, indexing="ij")
    pts = np.stack([xs.ravel(), ys.ravel()], axis=1)
    want = np.zeros((h * w, 3))
    for q in p.astype(np.float64):
        R = Rotation.from_euler("z", q[4]).as_matrix()[:2, :2]  # library rotation
        S = R @ np.diag([q[2] ** 2, q[3] ** 2]) @ R.T
        dens = multivariate_normal(mean=q[:2], cov=S).pdf(pts) * 2 * math.pi * abs(q[2] * q[3])
        want += dens[:, None] * q[5:8]
    np.testing.assert_allclose(ref.render_full(p, h, w, cov="rs"), want.reshape(h, w, 3),
                               rtol=1e-11, atol=1e-14)


def test_rs_closed_forms_and_symmetries():
    s1, s2, th, c = 2.5, 1.5, 0.7, 0.8
    p = np.array([[60.3, 59.7, s1, s2, th, c, 0.0, 0.0]], np.float32)
    pf = p.astype(np.float64)[0]
    img = ref.render_full(p, 120, 120, cov="rs")
    np.testing.assert_allclose(img[..., 0].sum(), 2 * math.pi * pf[2] * pf[3] * pf[5], rtol=1e-8)
    G = np.zeros((120, 120, 3))
    G[..., 0] = 1.0
    d = ref.grads(p, 120, 120, G, culled=False, cov="rs")[0]
    np.testing.assert_allclose(d[2], 2 * math.pi * pf[3] * pf[5], rtol=1e-7)
    np.testing.assert_allclose(d[3], 2 * math.pi * pf[2] * pf[5], rtol=1e-7)
    assert abs(d[4]) < 1e-7 and abs(d[0]) < 1e-7 and abs(d[1]) < 1e-7
    # theta + pi and (s1, s2, theta) -> (s2, s1, theta + pi/2) describe the same Sigma
    q = rs_gaussians(20, 48, 48, 9).astype(np.float64)
    a = ref.render_full(q.astype(np.float32), 48, 48, cov="rs")
    q2 = q.copy()
    q2[:, 4] += math.pi
    q3 = q.copy()
    q3[:, 2], q3[:, 3], q3[:, 4] = q[:, 3], q[:, 2], q[:, 4] + math.pi / 2
    for alt in (q2, q3):
        b = np.zeros((48, 48, 3))
        for n in range(alt.shape[0]):  # float64 parameters, no float32 rounding of theta
            inv = tuple(v[0] for v in ref._inv_from(alt[n:n + 1], "rs"))
            s, _, _ = ref._sigma(alt[n], inv, np.arange(48.0), np.arange(48.0))
            b += np.exp(-s)[:, :, None] * alt[n, 5:8]
        np.testing.assert_allclose(b, a, rtol=1e-6, atol=1e-9)


def test_rs_with_zero_angle_reduces_to_the_cholesky_tile_rule():
    h, w = 70, 90
    p = rs_gaussians(200, h, w, 3)
    p[:, 4] = 0.0
    chol = p.copy()
    chol[:, 2], chol[:, 3], chol[:, 4] = p[:, 2], 0.0, p[:, 3]
    r1, c1 = ref.tile_rects(p, h, w, cov="rs")
    r2, c2 = ref.tile_rects(chol, h, w)
    assert np.array_equal(r1, r2) and np.array_equal(c1, c2)
    np.testing.assert_allclose(ref.render_culled(p, h, w, cov="rs"), ref.render_culled(chol, h, w),
                               rtol=1e-14, atol=1e-300)


@pytest.mark.parametrize("culled", [True, False])
def test_rs_gradients_match_finite_differences(culled):
    h, w = 36, 40
    p = rs_gaussians(7, h, w, 21)
    G = synth.upstream_gradient(h, w, 8)
    an = ref.grads(p, h, w, G, culled=culled, cov="rs")
    fd = ref.fd_grads(p, h, w, G, culled=culled, cov="rs")
    scale = np.abs(an).max(axis=0) + 1e-12
    assert np.all(np.abs(an - fd) <= 1e-6 * scale + 1e-9 * np.abs(an).max()), (an - fd) / scale
    if culled:  # the local difference covers the tile support only
        for n in (0, 3):
            np.testing.assert_allclose(ref.fd_local(p, h, w, G, n, cov="rs"), fd[n], rtol=1e-5,
                                       atol=1e-8)
