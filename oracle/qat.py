"""Plain FP64 oracle of the attribute quantisation-aware fine-tuning of Sec. 3.3.

TEST INFRASTRUCTURE.  Only the tests, the smoke check and the CPU-baseline leg of the benchmark
may import or call this module.  It shares no code with the GPU path and never imports it.

A fine-tuning step renders the fake-quantised records (Sec. 3.3):
  * positions rounded to IEEE binary16 and back;
  * covariance slot i as code * gamma_i + beta_i with code = round(clamp((l - beta_i) / gamma_i,
    0, 2^b - 1)), ties to even (the LSQ+ equation; gamma, beta learned, shared by all Gaussians);
  * colours by residual vector quantisation: stage m takes the codebook entry nearest (squared
    Euclidean distance, lowest index on ties) to the residual left by stages < m, and the colour
    is the sum of the chosen entries (the RVQ equation).
Gradients (readings taken here, where the paper names the methods without their formulas):
  * straight-through estimates: d(quantised)/d(float) = 1 for positions and colours, and for a
    covariance slot whose scaled value lies inside [0, 2^b - 1]; 0 where it is clamped;
  * LSQ+ gradients of the quantiser: inside the range d/dgamma = code - x and d/dbeta = 0; below
    it d/dgamma = 0, d/dbeta = 1; above it d/dgamma = 2^b - 1, d/dbeta = 1 (x the scaled value);
  * the codebooks learn from the commitment loss only (Sec. 3.3, with the stop-gradient on the
    residual): L_c = 1/(N B) sum_m sum_n |r_n^{m-1} - C^m[i_n^m]|^2, weighted by lambda
    (unstated in the paper; 1 here unless given), added to the image loss;
  * every learned tensor takes an Adam step (module ``ref``): Gaussians with the fit step's
    rates, gamma, beta and the codebooks with the rate ``lr_q``.
Initialisation (readings): beta_i = min over Gaussians of slot i, gamma_i = (max - min) / (2^b - 1)
(the whole range representable); codebooks by K-means (Sec. 4.1: 5 iterations) on the colours,
stage by stage on the residuals of the earlier stages, seeded with the points at indices
floor(j N / B) and keeping a centroid whose cluster empties.
"""
from __future__ import annotations

import numpy as np

from . import ref


def _p64(params):
    p = np.asarray(params)
    if p.dtype != np.float32:
        p = p.astype(np.float32)
    return p.astype(np.float64).reshape(-1, 8)


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


def kmeans(points, k: int, iters: int):
    """Plain Lloyd iterations from the points at indices floor(j n / k); a centroid whose
    cluster is empty stays where it is.  Returns float64 centroids [k, d]."""
    x = np.asarray(points, np.float64)
    n = x.shape[0]
    cent = x[[(j * n) // k for j in range(k)]].copy()
    for _ in range(iters):
        d = ((x[:, None, :] - cent[None, :, :]) ** 2).sum(-1)
        a = np.argmin(d, axis=1)
        for j in range(k):
            sel = a == j
            if sel.any():
                cent[j] = x[sel].mean(axis=0)
    return cent


def rvq_init(params, stages: int, book: int, iters: int = 5):
    """Codebooks [M, B, 3] float64: K-means per stage on the residual colours."""
    c = _p64(params)[:, 5:8]
    books = np.zeros((stages, book, 3))
    resid = c.copy()
    for m in range(stages):
        books[m] = kmeans(resid, book, iters)
        d = ((resid[:, None, :] - books[m][None, :, :]) ** 2).sum(-1)
        resid = resid - books[m][np.argmin(d, axis=1)]
    return books


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
        d = ((resid[:, None, :] - cb[m][None, :, :]) ** 2).sum(-1)
        idx[:, m] = np.argmin(d, axis=1)
        col += cb[m][idx[:, m]]
        resid = resid - cb[m][idx[:, m]]
    q[:, 5:8] = col
    return q, x, code, idx, resids


def qat_grads(params, gamma, beta, books, bits, height, width, target, lam=1.0, cov="chol"):
    """(dparams [N, 8], dgamma [3], dbeta [3], dbooks [M, B, 3], loss, image) of
    L = mse(render(fake_quant(params)), target) + lam * L_c."""
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
    cb = np.asarray(books, np.float32).astype(np.float64)
    M, B = cb.shape[0], cb.shape[1]
    n = q.shape[0]
    dbooks = np.zeros_like(cb)
    lc = 0.0
    for m in range(M):
        diff = cb[m][idx[:, m]] - resids[m]            # C[i] - r
        lc += (diff ** 2).sum()
        for k in range(B):
            sel = idx[:, m] == k
            dbooks[m, k] = 2.0 * lam / (n * B) * diff[sel].sum(axis=0)
    loss = ref.mse(img, target) + lam * lc / (n * B)
    return dp, dgam, dbet, dbooks, loss, img


def qat_step(params, m, v, quant, quant_m, quant_v, target, step, height, width, bits,
             hp=None, lr_q=1e-3, lam=1.0, cov="chol"):
    """One fine-tuning step.  ``quant`` = (gamma, beta, books); ``quant_m``/``quant_v`` its
    Adam moments as one flat vector of 6 + M B 3 numbers (gamma, beta, books).  Returns
    (params, m, v, quant, quant_m, quant_v, loss, image)."""
    gamma, beta, books = quant
    dp, dg, db, dbk, loss, img = qat_grads(params, gamma, beta, books, bits, height, width,
                                           target, lam, cov)
    p, m, v = ref.adam_step(params, m, v, dp, step, hp, cov)
    flat = np.concatenate([np.asarray(gamma, np.float64), np.asarray(beta, np.float64),
                           np.asarray(books, np.float64).ravel()])
    gflat = np.concatenate([dg, db, dbk.ravel()])
    h = dict(ref.DEFAULT_ADAM if hp is None else hp)
    b1, b2, eps = h["beta1"], h["beta2"], h["eps"]
    qm = b1 * np.asarray(quant_m, np.float64) + (1 - b1) * gflat
    qv = b2 * np.asarray(quant_v, np.float64) + (1 - b2) * gflat * gflat
    flat = flat - lr_q * (qm / (1 - b1 ** step)) / (np.sqrt(qv / (1 - b2 ** step)) + eps)
    M, B = np.asarray(books).shape[:2]
    new = (flat[0:3], flat[3:6], flat[6:].reshape(M, B, 3))
    return p, m, v, new, qm, qv, loss, img
