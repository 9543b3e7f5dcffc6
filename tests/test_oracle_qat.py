"""Pins of the quantisation-aware fine-tuning oracle (Sec. 3.3) against closed forms (binary16,
LSQ+ rounding and its gradients at representable points, K-means on separated clusters),
finite differences of the commitment loss, and the Adam oracle.  CPU only."""
import numpy as np

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
    q, x, code, idx, _ = qat.fake_quant(p, gamma, beta, books, 6)
    np.testing.assert_array_equal(q[:, 0], [0.5, 100.25, 1000.5, 2048.0])
    np.testing.assert_array_equal(code[:, 0], [0, 1, 0, 0])
    np.testing.assert_array_equal(q[:, 2], [1.0, 1.125, 1.0, 1.0])
    np.testing.assert_array_equal(code[:, 2], [8, 8, 8, 63])
    np.testing.assert_array_equal(q[:, 4], [2.0, 2.0, 2.0, 1.0 + 63 * 0.125])
    np.testing.assert_array_equal(idx[:, 0], [3, 3, 3, 3])
    np.testing.assert_array_equal(q[:, 5:8], np.float32([[0.2, 0.3, 0.4]] * 4))


def test_lsq_init_spans_the_range():
    p = synth.gaussians(500, 64, 64, seed=3)
    g, b = qat.lsq_init(p, 6)
    q, x, code, _, _ = qat.fake_quant(p, g, b, np.zeros((1, 1, 3)), 6)
    assert np.all((x >= -1e-12) & (x <= 63 + 1e-12))
    assert code.min() == 0 and code.max() == 63
    assert np.all(np.abs(q[:, 2:5] - p[:, 2:5].astype(np.float64)) <= g / 2 + 1e-12)


def test_kmeans_recovers_separated_cluster_means():
    rng = np.random.default_rng(4)
    centres = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0], [0, 0, 1], [1, 1, 0], [1, 0, 1],
                        [0, 1, 1], [1, 1, 1]], np.float64)
    # cluster j occupies indices [40 j, 40 j + 40): the seeds floor(j n / k) = 40 j are one per
    # cluster, so Lloyd's iterations reach the cluster means and stay there
    lab = np.repeat(np.arange(8), 40)
    pts = centres[lab] + rng.uniform(-0.05, 0.05, (320, 3))
    got = qat.kmeans(pts, 8, 5)
    want = np.array([pts[lab == j].mean(axis=0) for j in range(8)])
    np.testing.assert_allclose(got, want, rtol=0, atol=1e-12)


def test_commitment_gradient_matches_finite_differences():
    rng = np.random.default_rng(5)
    n, M, B = 60, 2, 4
    res0 = rng.uniform(0, 1, (n, 3)).astype(np.float32)
    books = rng.uniform(0, 1, (M, B, 3)).astype(np.float32).astype(np.float64)
    p = np.zeros((n, 8), np.float32)
    p[:, 5:8] = res0
    # the commitment part alone: the image loss does not depend on the codebooks' gradient path
    _, _, _, idx, resids = qat.fake_quant(p, np.ones(3), np.zeros(3), books, 6)

    def lc(bk):
        total = 0.0
        for m in range(M):
            total += ((bk[m][idx[:, m]] - resids[m]) ** 2).sum()
        return total / (n * B)

    g = np.zeros_like(books)
    for m in range(M):
        for k in range(B):
            sel = idx[:, m] == k
            g[m, k] = 2.0 / (n * B) * (books[m][idx[sel, m]] - resids[m][sel]).sum(axis=0)
    fd = np.zeros_like(books)
    for ind in np.ndindex(books.shape):
        a, b = books.copy(), books.copy()
        a[ind] += 1e-6
        b[ind] -= 1e-6
        fd[ind] = (lc(a) - lc(b)) / 2e-6
    np.testing.assert_allclose(g, fd, rtol=1e-6, atol=1e-9)
    # and qat_grads forms the same codebook gradient (lambda = 1)
    h, w = 16, 16
    pp = synth.gaussians(n, h, w, seed=6)
    pp[:, 5:8] = res0
    _, _, _, dbk, _, _ = qat.qat_grads(pp, np.ones(3), np.zeros(3), books, 6, h, w,
                                       np.zeros((h, w, 3)), 1.0)
    _, _, _, idx2, resids2 = qat.fake_quant(pp, np.ones(3), np.zeros(3), books, 6)
    np.testing.assert_array_equal(idx2, idx)
    np.testing.assert_allclose(dbk, g, rtol=1e-12, atol=1e-15)


def test_ste_gradients_are_the_image_gradient_at_the_quantised_record():
    h, w = 24, 24
    p = synth.gaussians(40, h, w, seed=7, l_lo=1.5, l_hi=5.0)
    g, b = qat.lsq_init(p, 6)
    books = qat.rvq_init(p, 2, 8)
    T = synth.target_sinusoids(h, w, 8)
    dp, dg, db, _, _, img = qat.qat_grads(p, g, b, books, 6, h, w, T)
    q, x, code, _, _ = qat.fake_quant(p, g, b, books, 6)
    want = ref.grads(q.astype(np.float32), h, w, ref.mse_grad(img, T))
    inside = (x >= 0) & (x <= 63)
    np.testing.assert_array_equal(dp[:, [0, 1, 5, 6, 7]], want[:, [0, 1, 5, 6, 7]])
    np.testing.assert_array_equal(dp[:, 2:5][inside], want[:, 2:5][inside])
    assert np.all(dp[:, 2:5][~inside] == 0)
    # LSQ+ at the bounds: the extreme Gaussians sit at code 0 and code 63 exactly (x = 0, 63)
    np.testing.assert_allclose(dg, (want[:, 2:5] * np.where(inside, code - x, 0)).sum(0),
                               rtol=1e-12, atol=1e-15)
    np.testing.assert_array_equal(db, np.zeros(3))


def test_quantiser_adam_is_the_adam_oracle():
    h, w = 20, 20
    p = synth.gaussians(30, h, w, seed=9)
    g, b = qat.lsq_init(p, 6)
    books = qat.rvq_init(p, 2, 8)
    T = synth.target_sinusoids(h, w, 10)
    zeros = np.zeros((30, 8))
    nq = 6 + 2 * 8 * 3
    out = qat.qat_step(p, zeros, zeros, (g, b, books), np.zeros(nq), np.zeros(nq), T, 1, h, w,
                       6, lr_q=0.01)
    _, dg, db, dbk, _, _ = qat.qat_grads(p, g, b, books, 6, h, w, T)
    flat = np.concatenate([g, b, books.ravel()])
    gflat = np.concatenate([dg, db, dbk.ravel()])
    hp = dict(ref.DEFAULT_ADAM, lr_mu=0.01, lr_l=0.01, lr_c=0.01, l_min=0.0)
    P = np.zeros((nq, 8))
    P[:, 0] = flat
    G = np.zeros((nq, 8))
    G[:, 0] = gflat
    want = ref.adam_step(P, np.zeros((nq, 8)), np.zeros((nq, 8)), G, 1, hp)[0][:, 0]
    got = np.concatenate([out[3][0], out[3][1], out[3][2].ravel()])
    np.testing.assert_allclose(got, want, rtol=1e-14, atol=1e-16)
