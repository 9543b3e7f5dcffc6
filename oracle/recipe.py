"""Plain FP64 oracle of the paper's fitting recipe around the rasteriser (Sec. 4.1 and App. C).

TEST INFRASTRUCTURE.  Only the tests, the smoke check and the CPU-baseline leg of the benchmark
may import or call this module.  It shares no code with the GPU path and never imports it.

Raw records (rho_x, rho_y, lam1, lam2, lam3, c0, c1, c2) are what the optimiser updates; the
renderer sees the effective record (App. C):
  * positions pass through tanh into (-1, 1), read here as the image extent:
        mu_x = W (tanh(rho_x) + 1) / 2,   mu_y = H (tanh(rho_y) + 1) / 2;
  * 0.5 is added to the diagonal of L (l1 = lam1 + 0.5, l2 = lam2, l3 = lam3 + 0.5), or to the
    scales of the rotation-scale form (s1 = lam1 + 0.5, s2 = lam2 + 0.5, theta = lam3), in
    pixel units;
  * colours are used as they are.
The optimiser is Adan (Xie et al., Adan: adaptive Nesterov momentum, 2022; Sec. 4.1 uses it with
a learning rate of 1e-3 halved every 20000 steps).  Its recursion, with g_0 = g_1 on the first
step and every moment starting at zero with bias correction (the reading taken here):
    m_k = b1 m + (1 - b1) g_k
    v_k = b2 v + (1 - b2) (g_k - g_{k-1})
    n_k = b3 n + (1 - b3) (g_k + b2 (g_k - g_{k-1}))^2
    theta <- (theta - lr_k (m_k / (1 - b1^k) + b2 v_k / (1 - b2^k))
                      / (sqrt(n_k / (1 - b3^k)) + eps)) / (1 + lr_k wd)
with lr_k = lr 0.5^floor((k - 1) / halve_every).  (b1, b2, b3) = (0.98, 0.92, 0.99) are the
published defaults written as decay rates.
"""
from __future__ import annotations

import math

import numpy as np

from . import ref

DEFAULT_ADAN = dict(lr=1e-3, beta1=0.98, beta2=0.92, beta3=0.99, eps=1e-8, weight_decay=0.0,
                    halve_every=20000)


def _raw64(raw):
    r = np.asarray(raw)
    if r.dtype != np.float32:
        r = r.astype(np.float32)
    return r.astype(np.float64).reshape(-1, 8)


def effective(raw, height: int, width: int, cov="chol") -> np.ndarray:
    """Effective float64 records from raw float32 ones (App. C)."""
    r = _raw64(raw)
    p = r.copy()
    p[:, 0] = width * (np.tanh(r[:, 0]) + 1.0) / 2.0
    p[:, 1] = height * (np.tanh(r[:, 1]) + 1.0) / 2.0
    if cov == "chol":
        p[:, 2] = r[:, 2] + 0.5
        p[:, 4] = r[:, 4] + 0.5
    else:
        p[:, 2] = r[:, 2] + 0.5
        p[:, 3] = r[:, 3] + 0.5
    return p


def raw_grads(raw, d_effective, height: int, width: int) -> np.ndarray:
    """dL/draw from dL/d(effective record): the positions pick up d mu / d rho =
    (extent / 2)(1 - tanh(rho)^2); the +0.5 shifts have unit derivative."""
    r = _raw64(raw)
    d = np.array(d_effective, np.float64).reshape(-1, 8)
    d[:, 0] *= width / 2.0 * (1.0 - np.tanh(r[:, 0]) ** 2)
    d[:, 1] *= height / 2.0 * (1.0 - np.tanh(r[:, 1]) ** 2)
    return d


def adan_step(raw, m, v, n, g_prev, grad, step: int, hp=None):
    """One Adan update of the raw records (module header).  ``step`` counts from 1; on step 1
    the previous gradient is taken equal to the current one.  Returns float64
    (raw, m, v, n, g)."""
    hp = dict(DEFAULT_ADAN if hp is None else hp)
    th = np.asarray(raw, np.float64)
    g = np.asarray(grad, np.float64)
    gp = g if step == 1 else np.asarray(g_prev, np.float64)
    b1, b2, b3 = hp["beta1"], hp["beta2"], hp["beta3"]
    diff = g - gp
    m = b1 * np.asarray(m, np.float64) + (1.0 - b1) * g
    v = b2 * np.asarray(v, np.float64) + (1.0 - b2) * diff
    n = b3 * np.asarray(n, np.float64) + (1.0 - b3) * (g + b2 * diff) ** 2
    lr = hp["lr"] * 0.5 ** ((step - 1) // hp["halve_every"]) if hp["halve_every"] else hp["lr"]
    upd = (m / (1.0 - b1 ** step) + b2 * v / (1.0 - b2 ** step)) / (
        np.sqrt(n / (1.0 - b3 ** step)) + hp["eps"])
    th = (th - lr * upd) / (1.0 + lr * hp["weight_decay"])
    return th, m, v, n, g


def fit_step(raw, state, target, step: int, height: int, width: int, hp=None, cov="chol"):
    """One recipe fit step: render the effective records (tile support, Eq. rasterization4),
    L2 loss (mean over H W 3, Sec. 3.4), gradients (App. A) chained to the raw records, Adan.
    ``state`` = (m, v, n, g_prev).  Returns (raw, state, image, loss)."""
    p = effective(raw, height, width, cov).astype(np.float32)
    img = ref.render_culled(p, height, width, cov=cov)
    loss = ref.mse(img, target)
    d = ref.grads(p, height, width, ref.mse_grad(img, target), cov=cov)
    g = raw_grads(raw, d, height, width)
    m, v, n, gp = state
    th, m, v, n, g = adan_step(raw, m, v, n, gp, g, step, hp)
    return th, (m, v, n, g), img, loss
