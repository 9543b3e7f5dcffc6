"""Plain FP64 oracle of the attribute quantisation-aware fine-tuning of Sec. 3.3 and Sec. 3.4.

TEST INFRASTRUCTURE.  Only the tests, the smoke check and the CPU-baseline leg of the benchmark
may import or call this module.  It shares no code with the GPU path and never imports it.

A fine-tuning step renders the fake-quantised records (Sec. 3.3):
  * positions rounded to IEEE binary16 and back;
  * covariance slot i as code * gamma_i + beta_i with code = round(clamp((l - beta_i) / gamma_i,
    0, 2^b - 1)), ties to even (the LSQ+ equation; gamma, beta learned, shared by all Gaussians);
  * colours by residual vector quantisation: stage m takes the codebook entry nearest (squared
    Euclidean distance, lowest index on ties) to the residual left by stages < m, and the colour
    is the sum of the chosen entries (the RVQ equation).
Loss (Sec. 3.4): the image L2 loss plus lambda L_c, L_c = 1/(N B) sum_m sum_n
|sg[r_n^{m-1}] - C^m[i_n^m]|^2 (the commitment loss of Sec. 3.3); lambda is unstated (1 here
unless given).
Gradients and updates (readings taken here, where the paper names the methods without their
formulas):
  * straight-through estimates: d(quantised)/d(float) = 1 for positions and colours, and for a
    covariance slot whose scaled value lies inside [0, 2^b - 1]; 0 where it is clamped;
  * LSQ+ gradients of the quantiser: inside the range d/dgamma = code - x and d/dbeta = 0; below
    it d/dgamma = 0, d/dbeta = 1; above it d/dgamma = 2^b - 1, d/dbeta = 1 (x the scaled value);
  * Gaussians take an Adam step (module ``ref``) with the fit step's rates, gamma and beta an
    Adam step with the rate ``lr_q``;
  * the codebooks are updated in exponential-moving-average mode (Sec. 3.4, Training), not by a
    gradient: every entry keeps a running count N and a running sum S of the residuals assigned
    to it, and after each step, with n_j Gaussians and their residual sum s_j at stage m,
        N <- d N + (1 - d) n_j,   S <- d S + (1 - d) s_j,   C^m[j] = S / N  (kept if N = 0).
    For fixed assignments the minimiser of L_c over an entry is the mean of its residuals,
    which is what S / N tracks, so this is how L_c steers the codebooks; the stop-gradient in
    L_c sends none of it to the Gaussians.  The decay d is unstated: 0.99 unless given.  Count,
    sum and codebook are float32 between steps (the arithmetic is float64, rounded once each).
Initialisation (readings): beta_i = min over Gaussians of slot i, gamma_i = the least float32 >=
(max - min) / (2^b - 1) (the whole range representable); codebooks by K-means (Sec. 3.4 and
Sec. 4.1: 5 iterations) on the colours, stage by stage on the residuals of the earlier stages,
seeded with the points at indices floor(j N / B), keeping a centroid whose cluster empties; the
running count of an entry starts at the number of points nearest to its final centroid and the
running sum at that count times the float32 centroid.
"""
from __future__ import annotations

import numpy as np

from . import ref

DEFAULT_DECAY = 0.99


def _p64(params):
    p = np.asarray(params)
    if p.dtype != np.float32:
        p = p.astype(np.float32)
    return p.astype(np.float64).reshape(-1, 8)


def _f32(x):
    return np.asarray(x, np.float64).astype(np.float32).astype(np.float64)


def lsq_init(params, bits: int):
    """(gamma [3], beta [3]) from the range of slots 2..4, as float32 values: beta = min and
    gamma = the least float32 >= (max - min) / (2^b - 1), so that the whole range maps into
    [0, 2^b - 1]."""
    p = _p64(params)
    lo, hi = p[:, 2:5].min(axis=0), p[:, 2:5].max(axis=0)
    top = (1 << bits) - 1
    exact = np.where(hi > lo, (hi - lo) / top, 1.0)
    gamma = exact.astype(np.float32)
    gamma = np.where(gamma.astype(np.float64) < exact, np.nextafter(gamma, np.float32(np.inf)),
                     gamma)
    return gamma.astype(np.float64), lo


def nearest(points, cent):
    """Index of the nearest centroid (squared distance, lowest index on ties) per point."""
    d = ((points[:, None, :] - cent[None, :, :]) ** 2).sum(-1)
    return np.argmin(d, axis=1)


def kmeans(points, k: int, iters: int):
    """Plain Lloyd iterations from the points at indices floor(j n / k); a centroid whose
    cluster is empty stays where it is.  Returns float64 centroids [k, d]."""
    x = np.asarray(points, np.float64)
    n = x.shape[0]
    cent = x[[(j * n) // k for j in range(k)]].copy()
    for _ in range(iters):
        a = nearest(x, cent)
        for j in range(k):
            sel = a == j
            if sel.any():
                cent[j] = x[sel].mean(axis=0)
    return cent


def rvq_init(params, stages: int, book: int, iters: int = 5):
    """(codebooks [M, B, 3], running state [M, B, 4] = (count, sum of 3 channels)), float64
    holding float32 values: K-means per stage on the residual colours; the state counts the
    points nearest to each final centroid and sums count x centroid."""
    c = _p64(params)[:, 5:8]
    books = np.zeros((stages, book, 3))
    ema = np.zeros((stages, book, 4))
    resid = c.copy()
    for m in range(stages):
        cent = kmeans(resid, book, iters)
        books[m] = _f32(cent)
        a = nearest(resid, cent)
        cnt = np.bincount(a, minlength=book).astype(np.float64)
        ema[m, :, 0] = cnt
        ema[m, :, 1:4] = _f32(cnt[:, None] * books[m])
        resid = resid - cent[a]
    return books, ema


def fake_quant(params, gamma, beta, books, bits: int):
    """Fake-quantised float64 records [N, 8] and the facts the gradients need:
    (scaled values x [N, 3], codes [N, 3], RVQ indices [N, M], residuals [M, N, 3])."""
    p = _p64(params)
    q = p.copy()
    q[:, 0:2] = p[:, 0:2].astype(np.float16).astype(np.float64)
    # the quantiser's state is float32 (as stored between steps); its arithmetic is float64
    g = np.asarray(gamma, np.float32).astype(np.float64)
    b = np.asarray(beta, np.float32).astype(np.float64)
    top = (1 << bits) - 1
    x = (p[:, 2:5] - b) / g
    code = np.rint(np.clip(x, 0, top))
    q[:, 2:5] = code * g + b
    cb = np.asarray(books, np.float32).astype(np.float64)
    resid = p[:, 5:8].copy()
    idx = np.zeros((p.shape[0], cb.shape[0]), np.int64)
    resids = np.zeros((cb.shape[0], p.shape[0], 3))
    col = np.zeros((p.shape[0], 3))
    for m in range(cb.shape[0]):
        resids[m] = resid
        idx[:, m] = nearest(resid, cb[m])
        col += cb[m][idx[:, m]]
        resid = resid - cb[m][idx[:, m]]
    q[:, 5:8] = col
    return q, x, code, idx, resids


def commitment_loss(books, idx, resids):
    """L_c of Sec. 3.3: 1/(N B) sum over stages and Gaussians of |r^{m-1} - C^m[i^m]|^2."""
    cb = np.asarray(books, np.float32).astype(np.float64)
    n, B = idx.shape[0], cb.shape[1]
    total = 0.0
    for m in range(cb.shape[0]):
        total += ((resids[m] - cb[m][idx[:, m]]) ** 2).sum()
    return total / (n * B)


def qat_grads(params, gamma, beta, books, bits, height, width, target, lam=1.0, cov="chol"):
    """(dparams [N, 8], dgamma [3], dbeta [3], loss, image, idx, resids) of
    L = mse(render(fake_quant(params)), target) + lam * L_c; L_c adds nothing to the gradients
    (its stop-gradient covers the residual, and the codebooks are not gradient-trained)."""
    q, x, code, idx, resids = fake_quant(params, gamma, beta, books, bits)
    q32 = q.astype(np.float32)
    img = ref.render_culled(q32, height, width, cov=cov)
    d = ref.grads(q32, height, width, ref.mse_grad(img, target), cov=cov)
    top = (1 << bits) - 1
    inside = (x >= 0) & (x <= top)
    dp = d.copy()
    dp[:, 2:5] = np.where(inside, d[:, 2:5], 0.0)
    dgam = (d[:, 2:5] * np.where(inside, code - x, np.where(x > top, float(top), 0.0))).sum(0)
    dbet = (d[:, 2:5] * np.where(inside, 0.0, 1.0)).sum(0)
    loss = ref.mse(img, target) + lam * commitment_loss(books, idx, resids)
    return dp, dgam, dbet, loss, img, idx, resids


def ema_update(books, ema, idx, resids, decay=DEFAULT_DECAY):
    """The codebooks' exponential-moving-average step (module header): new (books, ema), float64
    holding float32 values.  ``idx``, ``resids`` are the assignments and the residuals before
    each stage that the step's render used."""
    cb = _f32(books).copy()
    st = _f32(ema).copy()
    d = float(np.float32(decay))
    M, B = cb.shape[0], cb.shape[1]
    for m in range(M):
        for j in range(B):
            sel = idx[:, m] == j
            n_j = float(sel.sum())
            s_j = resids[m][sel].sum(axis=0)
            cnt = float(np.float32(d * st[m, j, 0] + (1.0 - d) * n_j))
            tot = _f32(d * st[m, j, 1:4] + (1.0 - d) * s_j)
            st[m, j, 0] = cnt
            st[m, j, 1:4] = tot
            if cnt > 0.0:
                cb[m, j] = _f32(tot / cnt)
    return cb, st


def qat_step(params, m, v, quant, quant_m, quant_v, ema, target, step, height, width, bits,
             hp=None, lr_q=1e-3, lam=1.0, decay=DEFAULT_DECAY, cov="chol"):
    """One fine-tuning step.  ``quant`` = (gamma, beta, books); ``quant_m``/``quant_v`` the Adam
    moments of (gamma, beta) as one vector of 6; ``ema`` the codebooks' running state
    [M, B, 4].  Returns (params, m, v, quant, quant_m, quant_v, ema, loss, image)."""
    gamma, beta, books = quant
    dp, dg, db, loss, img, idx, resids = qat_grads(params, gamma, beta, books, bits, height,
                                                   width, target, lam, cov)
    p, m, v = ref.adam_step(params, m, v, dp, step, hp, cov)
    flat = np.concatenate([np.asarray(gamma, np.float64), np.asarray(beta, np.float64)])
    gflat = np.concatenate([dg, db])
    h = dict(ref.DEFAULT_ADAM if hp is None else hp)
    b1, b2, eps = h["beta1"], h["beta2"], h["eps"]
    qm = b1 * np.asarray(quant_m, np.float64) + (1 - b1) * gflat
    qv = b2 * np.asarray(quant_v, np.float64) + (1 - b2) * gflat * gflat
    flat = flat - lr_q * (qm / (1 - b1 ** step)) / (np.sqrt(qv / (1 - b2 ** step)) + eps)
    nb, ne = ema_update(books, ema, idx, resids, decay)
    return p, m, v, (flat[0:3], flat[3:6], nb), qm, qv, ne, loss, img
