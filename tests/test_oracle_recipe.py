"""Pins of the fitting-recipe oracle (App. C parametrisation, Adan of Sec. 4.1) against closed
forms, finite differences through the parametrisation, and the special case in which Adan is
Adam.  CPU only."""
import math

import numpy as np
import pytest

import synth
from oracle import recipe, ref


def test_parametrisation_closed_forms():
    raw = np.array([[0.0, 0.0, 0.0, 0.3, 0.0, 1, 2, 3],
                    [20.0, -20.0, 1.5, -0.25, 2.0, 0, 0, 0]], np.float32)
    p = recipe.effective(raw, 100, 200)
    np.testing.assert_array_equal(p[0], [100.0, 50.0, 0.5, float(np.float32(0.3)), 0.5, 1, 2, 3])
    np.testing.assert_allclose(p[1, :2], [200.0, 0.0], atol=1e-12)
    np.testing.assert_array_equal(p[1, 2:5], [2.0, -0.25, 2.5])
    q = recipe.effective(raw, 100, 200, cov="rs")
    np.testing.assert_array_equal(q[0, 2:5], [0.5, float(np.float32(0.3)) + 0.5, 0.0])
    np.testing.assert_array_equal(q[1, 2:5], [2.0, 0.25, 2.0])


@pytest.mark.parametrize("cov", ["chol", "rs"])
def test_raw_gradients_match_finite_differences(cov):
    h, w = 24, 28
    rng = np.random.default_rng(3)
    raw = np.zeros((5, 8), np.float32)
    raw[:, 0:2] = np.arctanh(rng.uniform(-0.7, 0.7, (5, 2)))
    raw[:, 2:5] = rng.uniform(1.0, 4.0, (5, 3))
    if cov == "chol":
        raw[:, 3] = rng.uniform(-0.5, 0.5, 5)
    else:
        raw[:, 4] = rng.uniform(-3, 3, 5)
    raw[:, 5:8] = rng.uniform(-0.5, 1.0, (5, 3))
    G = synth.upstream_gradient(h, w, 4)
    p = recipe.effective(raw, h, w, cov).astype(np.float32)
    an = recipe.raw_grads(raw, ref.grads(p, h, w, G, culled=False, cov=cov), h, w)

    def loss(r64):
        p64 = r64.copy()
        p64[:, 0] = w * (np.tanh(r64[:, 0]) + 1) / 2
        p64[:, 1] = h * (np.tanh(r64[:, 1]) + 1) / 2
        p64[:, 2] += 0.5
        p64[:, 4 if cov == "chol" else 3] += 0.5
        return float((ref._render64(p64, h, w, False, None, None, cov) * G).sum())

    # the analytic gradient is taken at the float32-rounded effective record: difference there
    r0 = raw.astype(np.float64)
    fd = np.zeros_like(an)
    for n in range(5):
        for k in range(8):
            step = 1e-6 * max(abs(r0[n, k]), 1.0)
            a, b = r0.copy(), r0.copy()
            a[n, k] += step
            b[n, k] -= step
            fd[n, k] = (loss(a) - loss(b)) / (2 * step)
    scale = np.abs(an).max(axis=0) + 1e-12
    assert np.all(np.abs(an - fd) <= 2e-5 * scale), (an - fd) / scale


def test_adan_with_a_constant_gradient_moves_by_the_learning_rate_times_the_sign():
    hp = dict(recipe.DEFAULT_ADAN, halve_every=2, eps=0.0)
    g = np.array([0.3, -2.0, 1e-3])
    th = np.zeros(3)
    st = (np.zeros(3), np.zeros(3), np.zeros(3), np.zeros(3))
    lrs = []
    for k in range(1, 6):
        th, *st = recipe.adan_step(th, *st, g, k, hp)
        lrs.append(hp["lr"] * 0.5 ** ((k - 1) // 2))
    np.testing.assert_allclose(th, -sum(lrs) * np.sign(g), rtol=1e-12)


def test_adan_without_its_difference_term_is_adam():
    rng = np.random.default_rng(6)
    hp = dict(recipe.DEFAULT_ADAN, beta2=0.0, halve_every=0, lr=0.01)
    adam = dict(ref.DEFAULT_ADAM, lr_mu=0.01, lr_l=0.01, lr_c=0.01, beta1=hp["beta1"],
                beta2=hp["beta3"], eps=hp["eps"], l_min=0.0)
    th = rng.normal(size=(4, 8))
    a = th.copy()
    st = (np.zeros((4, 8)),) * 4
    am, av = np.zeros((4, 8)), np.zeros((4, 8))
    for k in range(1, 7):
        g = rng.normal(size=(4, 8))
        th, *st = recipe.adan_step(th, *st, g, k, hp)
        a, am, av = ref.adam_step(a, am, av, g, k, adam)
        np.testing.assert_allclose(th, a, rtol=1e-12, atol=1e-15)


def test_recipe_fit_step_lowers_the_loss():
    h, w = 32, 40
    rng = np.random.default_rng(8)
    raw = np.zeros((80, 8), np.float32)
    raw[:, 0:2] = np.arctanh(rng.uniform(-0.95, 0.95, (80, 2)))
    raw[:, 2:5] = rng.uniform(0.5, 3.0, (80, 3))
    raw[:, 3] = rng.uniform(-0.3, 0.3, 80)
    raw[:, 5:8] = rng.uniform(0, 0.5, (80, 3))
    T = synth.target_sinusoids(h, w, 9)
    st = tuple(np.zeros((80, 8)) for _ in range(4))
    hp = dict(recipe.DEFAULT_ADAN, lr=0.02)
    losses = []
    r = raw
    for k in range(1, 31):
        r, st, _, loss = recipe.fit_step(r, st, T, k, h, w, hp)
        r = r.astype(np.float32)
        losses.append(loss)
    assert losses[-1] < 0.5 * losses[0], losses[::6]


def test_adan_with_equal_first_two_rates_is_adam_on_the_nesterov_gradient():
    # Adan's reformulation: with b1 = b2 = b the numerator m_k + b v_k is an exponential average
    # of g_k + b (g_k - g_{k-1}), and n_k one of its square; so Adan equals Adam (the pinned
    # oracle) fed that gradient, with Adam's second rate b3, under a gradient that changes
    rng = np.random.default_rng(11)
    b, b3 = 0.9, 0.99
    hp = dict(recipe.DEFAULT_ADAN, beta1=b, beta2=b, beta3=b3, halve_every=0, lr=0.02)
    adam = dict(ref.DEFAULT_ADAM, lr_mu=0.02, lr_l=0.02, lr_c=0.02, beta1=b, beta2=b3,
                eps=hp["eps"], l_min=0.0)
    th = rng.normal(size=(5, 8))
    a = th.copy()
    st = (np.zeros((5, 8)),) * 4
    am, av = np.zeros((5, 8)), np.zeros((5, 8))
    g_prev = None
    for k in range(1, 9):
        g = rng.normal(size=(5, 8)) * (1.0 + k)
        nesterov = g if g_prev is None else g + b * (g - g_prev)
        th, *st = recipe.adan_step(th, *st, g, k, hp)
        a, am, av = ref.adam_step(a, am, av, nesterov, k, adam)
        np.testing.assert_allclose(th, a, rtol=1e-12, atol=1e-14)
        g_prev = g


def test_adan_moments_are_explicit_weighted_sums():
    # with the default rates (all different) the three moments after k steps are the unrolled
    # sums sum_j (1 - b) b^(k - j) x_j of their inputs (x = g, g - g_prev (0 at j = 1), and
    # (g + b2 (g - g_prev))^2), and the update divides the bias-corrected ones
    rng = np.random.default_rng(12)
    hp = dict(recipe.DEFAULT_ADAN, halve_every=0, lr=0.01)
    b1, b2, b3, eps = hp["beta1"], hp["beta2"], hp["beta3"], hp["eps"]
    gs = [rng.normal(size=6) for _ in range(7)]
    th = np.zeros(6)
    st = (np.zeros(6),) * 4
    for k in range(1, 8):
        before = th.copy()
        th, *st = recipe.adan_step(th, *st, gs[k - 1], k, hp)
        d = [np.zeros(6)] + [gs[j] - gs[j - 1] for j in range(1, k)]
        m = sum((1 - b1) * b1 ** (k - 1 - j) * gs[j] for j in range(k))
        v = sum((1 - b2) * b2 ** (k - 1 - j) * d[j] for j in range(k))
        n = sum((1 - b3) * b3 ** (k - 1 - j) * (gs[j] + b2 * d[j]) ** 2 for j in range(k))
        np.testing.assert_allclose(st[0], m, rtol=1e-12, atol=1e-15)
        np.testing.assert_allclose(st[1], v, rtol=1e-12, atol=1e-15)
        np.testing.assert_allclose(st[2], n, rtol=1e-12, atol=1e-15)
        step = (m / (1 - b1 ** k) + b2 * v / (1 - b2 ** k)) / (np.sqrt(n / (1 - b3 ** k)) + eps)
        np.testing.assert_allclose(before - th, 0.01 * step, rtol=1e-10, atol=1e-15)
