"""Pins of the quantisation-aware fine-tuning oracle (Sec. 3.3, Sec. 3.4) against closed forms
(binary16, LSQ+ rounding at representable points, K-means on separated clusters, the moving
average's geometric convergence), torch float64 autograd of the LSQ+ quantiser with a
straight-through round in all three branches, the commitment loss's minimiser, and the Adam
oracle.  CPU only."""
import numpy as np
import pytest

import synth
from oracle import qat, ref


def test_fake_quant_closed_forms():
    p = np.zeros((4, 8), np.float32)
    p[:, 0] = [0.5, 100.25, 1000.3, 2049.0]     # binary16: exact, exact, to 1000.5, tie to 2048
    p[:, 1] = [1.0, 2.0, 3.0, 4.0]
    p[:, 2] = [1.0, 1.125, 1.0625, 0.0]         # gamma 0.125, beta 1: codes 0, 1, tie 0.5 -> 0, clamp
    p[:, 3] = [0.0, 0.0, 0.0, 0.0]
    p[:, 4] = [2.0, 2.0, 2.0, 10.0]             # above the range: clamps to 63
    p[:, 5:8] = [[0.2, 0.3, 0.4]] * 4
    gamma, beta = np.array([0.125, 1.0, 0.125]), np.array([1.0, -0.5, 1.0])
    books = np.zeros((2, 8, 3))
    books[0, 3] = np.float32([0.2, 0.3, 0.4])
    q, x, code, idx, resids = qat.fake_quant(p, gamma, beta, books, 6)
    np.testing.assert_array_equal(q[:, 0], [0.5, 100.25, 1000.5, 2048.0])
    np.testing.assert_array_equal(code[:, 0], [0, 1, 0, 0])
    np.testing.assert_array_equal(q[:, 2], [1.0, 1.125, 1.0, 1.0])
    np.testing.assert_array_equal(code[:, 2], [8, 8, 8, 63])
    np.testing.assert_array_equal(q[:, 4], [2.0, 2.0, 2.0, 1.0 + 63 * 0.125])
    np.testing.assert_array_equal(idx[:, 0], [3, 3, 3, 3])
    np.testing.assert_array_equal(q[:, 5:8], np.float32([[0.2, 0.3, 0.4]] * 4))
    # the residual before stage 0 is the colour, before stage 1 what stage 0 left (nothing)
    np.testing.assert_array_equal(resids[0], np.float32([[0.2, 0.3, 0.4]] * 4))
    np.testing.assert_array_equal(resids[1], np.zeros((4, 3)))
    np.testing.assert_array_equal(idx[:, 1], [0, 0, 0, 0])


def test_lsq_init_spans_the_range():
    p = synth.gaussians(500, 64, 64, seed=3)
    g, b = qat.lsq_init(p, 6)
    q, x, code, _, _ = qat.fake_quant(p, g, b, np.zeros((1, 1, 3)), 6)
    assert np.all((x >= -1e-12) & (x <= 63 + 1e-12))
    assert code.min() == 0 and code.max() == 63
    assert np.all(np.abs(q[:, 2:5] - p[:, 2:5].astype(np.float64)) <= g / 2 + 1e-12)


def separated_points(seed, per=40):
    rng = np.random.default_rng(seed)
    centres = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0], [0, 0, 1], [1, 1, 0], [1, 0, 1],
                        [0, 1, 1], [1, 1, 1]], np.float64)
    # cluster j occupies indices [per j, per (j + 1)): the seeds floor(j n / k) = per j are one
    # per cluster, so Lloyd's iterations reach the cluster means and stay there
    lab = np.repeat(np.arange(8), per)
    return centres[lab] + rng.uniform(-0.05, 0.05, (8 * per, 3)), lab


def test_kmeans_recovers_separated_cluster_means():
    pts, lab = separated_points(4)
    got = qat.kmeans(pts, 8, 5)
    want = np.array([pts[lab == j].mean(axis=0) for j in range(8)])
    np.testing.assert_allclose(got, want, rtol=0, atol=1e-12)


def test_rvq_init_state_counts_each_cluster():
    # unequal separated clusters as colours: stage 0's running count of entry j is cluster j's
    # size and its running sum is that size times the float32 centroid (the cluster mean)
    rng = np.random.default_rng(14)
    sizes = [30, 45, 20, 60, 35, 50, 25, 40]
    centres = rng.uniform(0.1, 0.9, (8, 3))
    centres[:, 0] = np.linspace(0.05, 0.95, 8)     # separated along the first channel
    n = sum(sizes)
    # the seeds floor(j n / 8) take one point of each cluster; the other points in any order
    seeds = [(j * n) // 8 for j in range(8)]
    rest = rng.permutation(np.repeat(np.arange(8), np.array(sizes) - 1))
    lab = np.empty(n, np.int64)
    lab[seeds] = np.arange(8)
    lab[np.setdiff1d(np.arange(n), seeds)] = rest
    cols = centres[lab] + rng.uniform(-0.01, 0.01, (n, 3))
    p = np.zeros((n, 8), np.float32)
    p[:, 5:8] = cols
    books, ema = qat.rvq_init(p, 2, 8, 5)
    c32 = p[:, 5:8].astype(np.float64)
    want = np.array([c32[lab == j].mean(axis=0) for j in range(8)])
    np.testing.assert_allclose(books[0], want, rtol=0, atol=1e-7)
    np.testing.assert_array_equal(ema[0, :, 0], sizes)
    np.testing.assert_allclose(ema[0, :, 1:4], np.array(sizes)[:, None] * books[0], rtol=1e-7)
    assert ema[1, :, 0].sum() == n


def test_lsq_gradients_match_torch_autograd_in_all_three_branches():
    # the fake quantiser of slots 2..4 written with torch ops in float64 (clamp, scale and a
    # straight-through round x + (round(x) - x).detach()) and differentiated by autograd; the
    # record values straddle the code range so that every branch (below, inside, above) occurs
    torch = pytest.importorskip("torch")
    h, w = 28, 30
    n = 60
    p = synth.gaussians(n, h, w, seed=15, l_lo=1.5, l_hi=5.0)
    gamma = np.float32([0.05, 0.02, 0.04]).astype(np.float64)
    beta = np.float32([2.0, -0.4, 2.2]).astype(np.float64)
    books = qat.rvq_init(p, 2, 8)[0]
    T = synth.target_sinusoids(h, w, 16)
    dp, dg, db, _, img, _, _ = qat.qat_grads(p, gamma, beta, books, 6, h, w, T)
    q, x, _, _, _ = qat.fake_quant(p, gamma, beta, books, 6)
    assert (x < 0).sum() >= 5 and (x > 63).sum() >= 5 and ((x >= 0) & (x <= 63)).sum() >= 5
    up = ref.grads(q.astype(np.float32), h, w, ref.mse_grad(img, T))[:, 2:5]
    lt = torch.tensor(p[:, 2:5].astype(np.float64), requires_grad=True)
    gt = torch.tensor(gamma, requires_grad=True)
    bt = torch.tensor(beta, requires_grad=True)
    xc = torch.clamp((lt - bt) / gt, 0.0, 63.0)
    r = xc + (torch.round(xc) - xc).detach()
    lbar = r * gt + bt
    (lbar * torch.tensor(up)).sum().backward()
    np.testing.assert_allclose(dp[:, 2:5], lt.grad.numpy(), rtol=1e-12, atol=1e-18)
    np.testing.assert_allclose(dg, gt.grad.numpy(), rtol=1e-10, atol=1e-18)
    np.testing.assert_allclose(db, bt.grad.numpy(), rtol=1e-10, atol=1e-18)
    # the quantised values themselves agree with the torch forward
    np.testing.assert_array_equal(q[:, 2:5], lbar.detach().numpy())


def test_ste_gradients_are_the_image_gradient_at_the_quantised_record():
    h, w = 24, 24
    p = synth.gaussians(40, h, w, seed=7, l_lo=1.5, l_hi=5.0)
    g, b = qat.lsq_init(p, 6)
    books = qat.rvq_init(p, 2, 8)[0]
    T = synth.target_sinusoids(h, w, 8)
    dp, dg, db, _, img, _, _ = qat.qat_grads(p, g, b, books, 6, h, w, T)
    q, x, code, _, _ = qat.fake_quant(p, g, b, books, 6)
    want = ref.grads(q.astype(np.float32), h, w, ref.mse_grad(img, T))
    inside = (x >= 0) & (x <= 63)
    np.testing.assert_array_equal(dp[:, [0, 1, 5, 6, 7]], want[:, [0, 1, 5, 6, 7]])
    np.testing.assert_array_equal(dp[:, 2:5][inside], want[:, 2:5][inside])
    assert np.all(dp[:, 2:5][~inside] == 0)
    np.testing.assert_array_equal(db, np.zeros(3))


def _assignment(n, M, B, seed):
    rng = np.random.default_rng(seed)
    idx = rng.integers(0, B, (n, M))
    resids = rng.uniform(-1, 1, (M, n, 3))
    return idx, resids


def test_ema_converges_geometrically_to_constant_residuals():
    # every Gaussian chosen by entry j brings the same residual r_j in every step: with state
    # (N0, S0 = N0 C0) the closed form is C_t = (d^t N0 C0 + (1 - d^t) n r) / (d^t N0 + (1 - d^t) n)
    M, B, d = 2, 4, 0.9
    rng = np.random.default_rng(17)
    rj = rng.uniform(-1, 1, (M, B, 3)).astype(np.float32).astype(np.float64)
    counts = np.array([[5, 0, 9, 3], [7, 2, 0, 8]])
    n = counts.sum(axis=1)
    assert n[0] == n[1]
    idx = np.stack([np.repeat(np.arange(B), counts[m]) for m in range(M)], axis=1)
    resids = np.stack([rj[m][idx[:, m]] for m in range(M)])
    C0 = rng.uniform(-1, 1, (M, B, 3)).astype(np.float32).astype(np.float64)
    N0 = np.array([[4.0, 6.0, 1.0, 8.0], [3.0, 5.0, 2.0, 9.0]])
    ema = np.concatenate([N0[..., None], (N0[..., None] * C0).astype(np.float32)], axis=2)
    books = C0.copy()
    for t in range(1, 41):
        books, ema = qat.ema_update(books, ema, idx, resids, decay=d)
        a = d ** t
        want = (a * N0[..., None] * C0 + (1 - a) * counts[..., None] * rj) / (
            a * N0[..., None] + (1 - a) * counts[..., None])
        np.testing.assert_allclose(books, want, rtol=2e-5, atol=2e-6 * (t + 1))
    # after 40 steps the assigned entries sit within d^40 (relative) of their residual; an
    # entry nobody chose keeps its centroid (S and N decay together)
    used = counts > 0
    assert np.all(np.abs(books - rj)[used] <= 0.1 * np.abs(C0 - rj)[used] + 1e-5)
    np.testing.assert_allclose(books[~used], C0[~used], rtol=1e-5, atol=1e-6)


def test_ema_with_zero_decay_is_a_lloyd_update_and_minimises_the_commitment_loss():
    M, B, n = 2, 8, 300
    idx, resids = _assignment(n, M, B, 18)
    idx[:, 1] = np.where(idx[:, 1] == 5, 4, idx[:, 1])   # entry 5 of stage 1 left unused
    books0 = np.random.default_rng(19).uniform(-1, 1, (M, B, 3)).astype(np.float32)
    ema0 = np.ones((M, B, 4))
    books, ema = qat.ema_update(books0, ema0, idx, resids, decay=0.0)
    for m in range(M):
        for j in range(B):
            sel = idx[:, m] == j
            if sel.any():
                np.testing.assert_allclose(books[m, j], resids[m][sel].mean(axis=0), rtol=2e-7,
                                           atol=1e-7)
                assert ema[m, j, 0] == sel.sum()
            else:
                np.testing.assert_array_equal(books[m, j], books0[m, j])
                assert ema[m, j, 0] == 0
    # for these assignments no move of an entry lowers L_c (up to the float32 rounding of the
    # entries themselves)
    base = qat.commitment_loss(books, idx, resids)
    rng = np.random.default_rng(20)
    for _ in range(50):
        moved = books + rng.normal(0, 1e-3, books.shape)
        assert qat.commitment_loss(moved, idx, resids) >= base - 1e-12


def test_ema_fixed_point_and_decay_one():
    M, B, n = 1, 4, 80
    idx, resids = _assignment(n, M, B, 21)
    counts = np.array([(idx[:, 0] == j).sum() for j in range(B)], np.float64)
    means = np.array([resids[0][idx[:, 0] == j].mean(axis=0) for j in range(B)])
    books = means[None].astype(np.float32).astype(np.float64)
    ema = np.concatenate([counts[None, :, None], (counts[:, None] * books[0])[None]], axis=2)
    nb, ne = qat.ema_update(books, ema, idx, resids, decay=0.95)
    np.testing.assert_allclose(nb, books, rtol=1e-6, atol=1e-7)
    np.testing.assert_allclose(ne[..., 0], ema[..., 0], rtol=1e-7)
    # with decay 1 the state stays and the entries are S / N again (within float32 rounding)
    nb1, ne1 = qat.ema_update(books, ema, idx, resids, decay=1.0)
    np.testing.assert_allclose(nb1, books, rtol=2.5e-7, atol=1e-8)
    np.testing.assert_array_equal(ne1, ema.astype(np.float32))


def test_quantiser_adam_is_the_adam_oracle_and_the_loss_carries_lambda_lc():
    h, w = 20, 20
    p = synth.gaussians(30, h, w, seed=9)
    g, b = qat.lsq_init(p, 6)
    books, ema = qat.rvq_init(p, 2, 8)
    T = synth.target_sinusoids(h, w, 10)
    zeros = np.zeros((30, 8))
    out = qat.qat_step(p, zeros, zeros, (g, b, books), np.zeros(6), np.zeros(6), ema, T, 1, h, w,
                       6, lr_q=0.01, lam=2.5)
    dp, dg, db, _, img, idx, resids = qat.qat_grads(p, g, b, books, 6, h, w, T)
    flat = np.concatenate([g, b])
    gflat = np.concatenate([dg, db])
    hp = dict(ref.DEFAULT_ADAM, lr_mu=0.01, lr_l=0.01, lr_c=0.01, l_min=0.0)
    P = np.zeros((6, 8))
    P[:, 0] = flat
    G = np.zeros((6, 8))
    G[:, 0] = gflat
    want = ref.adam_step(P, np.zeros((6, 8)), np.zeros((6, 8)), G, 1, hp)[0][:, 0]
    got = np.concatenate([out[3][0], out[3][1]])
    np.testing.assert_allclose(got, want, rtol=1e-14, atol=1e-16)
    # the records take the Adam step of their straight-through gradient
    np.testing.assert_allclose(out[0], ref.adam_step(p, zeros, zeros, dp, 1)[0], rtol=1e-15)
    # the codebooks take the moving-average step, not a gradient step
    nb, ne = qat.ema_update(books, ema, idx, resids)
    np.testing.assert_array_equal(out[3][2], nb)
    np.testing.assert_array_equal(out[6], ne)
    # loss = image MSE + lambda L_c, L_c summed by brute force over stages and Gaussians
    lc = 0.0
    cb = books.astype(np.float32).astype(np.float64)
    for n in range(30):
        for m in range(2):
            lc += ((resids[m][n] - cb[m][idx[n, m]]) ** 2).sum()
    np.testing.assert_allclose(out[7], ref.mse(img, T) + 2.5 * lc / (30 * 8), rtol=1e-13)
