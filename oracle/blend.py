"""Plain FP64 oracle of the opacity variants of the rasteriser (Sec. 3.2).

TEST INFRASTRUCTURE.  Only the tests, the smoke check and the CPU-baseline leg of the benchmark
may import or call this module.  It shares no code with the GPU path and never imports it.

Each Gaussian has the 8-number record of ``ref`` (slots 5..7 now hold a colour c, not merged
with the opacity) and an opacity o.  Two renderings (the ablation rows of Table 3):
  * ``"sum"`` — accumulated summation with a separate opacity (Eq. rasterization3):
        C(p) = sum_n c_n o_n exp(-sigma_n(p));
  * ``"alpha"`` — alpha blending in a fixed order (Eq. rasterization1 with Eq. rasterization2):
        C(p) = sum_n c_n alpha_n T_n,  T_n = prod_{m<n} (1 - alpha_m),  alpha_n = o_n exp(-sigma_n).
Readings taken here:
  * the support is the tile support of ``ref`` (Gaussian n reaches every pixel of each tile its
    3-sigma box touches);
  * with no depth (Sec. 3.2 drops it) the blending order is ascending Gaussian index;
  * alpha is clamped from above at 0.99 as in the 3D-GS rasteriser that Eq. rasterization1 comes
    from, which keeps 1 - alpha >= 0.01; that rasteriser's skipping of alpha < 1/255 and its early
    stop at T < 1e-4 are speed heuristics, not part of the formula, and are not taken;
  * where the clamp is active, alpha does not depend on o or sigma (zero derivative there).

Gradients (the chain rule of App. A with dC/dalpha in place of dC/dsigma): with S_k the colour
blended behind Gaussian k, S_k = sum_{n>k} c_n alpha_n prod_{k<m<n} (1 - alpha_m),
    dC/dc_k = alpha_k T_k,   dC/dalpha_k = T_k (c_k - S_k),
then dalpha/do = exp(-sigma), dalpha/dsigma = -o exp(-sigma) where unclamped, and sigma's own
derivatives as in ``ref.grads``.
"""
from __future__ import annotations

import math

import numpy as np

from . import ref

ALPHA_MAX = 0.99


def _f64(a, cols):
    a = np.asarray(a)
    if a.dtype != np.float32:
        a = a.astype(np.float32)
    return a.astype(np.float64).reshape(-1, cols) if cols else a.astype(np.float64).reshape(-1)


def _tile_pixels(t, tw, height, width):
    tx, ty = t % tw, t // tw
    ys, xs = np.meshgrid(np.arange(ty * ref.TILE, min((ty + 1) * ref.TILE, height)),
                         np.arange(tx * ref.TILE, min((tx + 1) * ref.TILE, width)),
                         indexing="ij")
    return ys.ravel(), xs.ravel()


def _terms(p, inv, ids, ys, xs):
    """exp(-sigma) [L, P] and the offsets d of the tile's pixels from each listed Gaussian."""
    dx = (xs + 0.5)[None, :] - p[ids, 0][:, None]
    dy = (ys + 0.5)[None, :] - p[ids, 1][:, None]
    i00, i01, i11 = (v[ids][:, None] for v in inv)
    s = 0.5 * (i00 * dx * dx + 2.0 * i01 * dx * dy + i11 * dy * dy)
    return np.exp(-s), dx, dy


def _alpha(o, e):
    a = o[:, None] * e
    return np.minimum(a, ALPHA_MAX), a < ALPHA_MAX


def _render64(p, o, height, width, mode, cov, lists, inv, with_abs=False):
    img = np.zeros((height * width, 3))
    aimg = np.zeros((height * width, 3))
    tw, _ = ref.grid_tiles(height, width)
    ranges, ids_all = lists
    for t, (a, b) in enumerate(ranges):
        if a == b:
            continue
        ids = ids_all[a:b]
        ys, xs = _tile_pixels(t, tw, height, width)
        e, _, _ = _terms(p, inv, ids, ys, xs)
        c = p[ids, 5:8]
        if mode == "sum":
            w = o[ids][:, None] * e                       # [L, P]
        else:
            al, _ = _alpha(o[ids], e)
            T = np.cumprod(np.vstack([np.ones((1, al.shape[1])), 1.0 - al[:-1]]), axis=0)
            w = al * T
        pix = ys * width + xs
        img[pix] += w.T @ c
        aimg[pix] += np.abs(w).T @ np.abs(c)
    img = img.reshape(height, width, 3)
    if with_abs:
        return img, aimg.reshape(height, width, 3)
    return img


def render_blend(params, opacity, height: int, width: int, mode: str = "alpha", cov="chol",
                 with_abs: bool = False):
    """float64 image [H, W, 3] of the chosen opacity rendering; with ``with_abs`` also
    A(p) = sum |c_n| |w_n(p)| over the same terms (the scale for relative error)."""
    assert mode in ("sum", "alpha")
    p = _f64(params, 8)
    o = _f64(opacity, 0)
    return _render64(p, o, height, width, mode, cov, ref.tile_lists(params, height, width, cov),
                     ref.inverse_covariance(params, cov), with_abs)


def _sigma_chain(pn, inv_n, dx, dy, dsig, cov):
    """dL/dmu and dL/d(slots 2..4) per pixel from dL/dsigma per pixel (App. A)."""
    i00, i01, i11 = inv_n
    vx = i00 * dx + i01 * dy
    vy = i01 * dx + i11 * dy
    g1 = dsig * (-0.5 * vx * vx)
    g2 = dsig * (-0.5 * vx * vy)
    g3 = dsig * (-0.5 * vy * vy)
    if cov == "chol":
        l1, l2, l3 = pn[2], pn[3], pn[4]
        shape = [2 * g1 * l1 + 2 * g2 * l2, 2 * g2 * l1 + 2 * g3 * l2, 2 * g3 * l3]
    else:
        s1, s2, th = pn[2], pn[3], pn[4]
        c, sn = math.cos(th), math.sin(th)
        R = np.array([[c, -sn], [sn, c]])
        dR = np.array([[-sn, -c], [c, -sn]])
        SS = np.diag([s1 * s1, s2 * s2])
        mats = [R @ np.diag([2 * s1, 0.0]) @ R.T, R @ np.diag([0.0, 2 * s2]) @ R.T,
                dR @ SS @ R.T + R @ SS @ dR.T]
        shape = [g1 * M[0, 0] + g2 * (M[0, 1] + M[1, 0]) + g3 * M[1, 1] for M in mats]
    return [-dsig * vx, -dsig * vy, *shape]  # dsigma/dmu = -Sigma^{-1} d


def grads_blend(params, opacity, height: int, width: int, dl_dimage, mode: str = "alpha",
                cov="chol", with_abs: bool = False):
    """(dL/dparams [N, 8], dL/dopacity [N]) in float64; with ``with_abs`` also the sums of the
    absolute per-pixel contributions of each (same shapes)."""
    p = _f64(params, 8)
    o = _f64(opacity, 0)
    G = np.asarray(dl_dimage, np.float64).reshape(height * width, 3)
    n = p.shape[0]
    d = np.zeros((n, 9))
    ad = np.zeros((n, 9))
    inv = ref.inverse_covariance(params, cov)
    ranges, ids_all = ref.tile_lists(params, height, width, cov)
    tw, _ = ref.grid_tiles(height, width)
    for t, (a, b) in enumerate(ranges):
        if a == b:
            continue
        ids = ids_all[a:b]
        ys, xs = _tile_pixels(t, tw, height, width)
        e, dx, dy = _terms(p, inv, ids, ys, xs)
        g = G[ys * width + xs]                             # [P, 3]
        c = p[ids, 5:8]
        gc = c @ g.T                                       # [L, P]: <G, c_k>
        if mode == "sum":
            ok = np.ones_like(e, bool)
            w = o[ids][:, None] * e
            dc = w[:, :, None] * g[None, :, :]             # [L, P, 3]
            dalpha = gc                                    # dL/d(o e)
        else:
            al, ok = _alpha(o[ids], e)
            L = al.shape[0]
            T = np.cumprod(np.vstack([np.ones((1, al.shape[1])), 1.0 - al[:-1]]), axis=0)
            S = np.zeros_like(al[:, :, None].repeat(3, axis=2))   # [L, P, 3]
            for k in range(L - 2, -1, -1):
                S[k] = c[k + 1][None, :] * al[k + 1][:, None] + (1.0 - al[k + 1])[:, None] * S[k + 1]
            dc = (al * T)[:, :, None] * g[None, :, :]
            dalpha = T * (gc - np.einsum("lpc,pc->lp", S, g))
        do = np.where(ok, e * dalpha, 0.0)
        dsig = np.where(ok, -o[ids][:, None] * e * dalpha, 0.0)
        for j, nid in enumerate(ids):
            parts = _sigma_chain(p[nid], tuple(v[nid] for v in inv), dx[j], dy[j], dsig[j], cov)
            parts += [dc[j, :, 0], dc[j, :, 1], dc[j, :, 2], do[j]]
            for k, q in enumerate(parts):
                d[nid, k] += q.sum()
                ad[nid, k] += np.abs(q).sum()
    if with_abs:
        return d[:, :8], d[:, 8], ad[:, :8], ad[:, 8]
    return d[:, :8], d[:, 8]


def fd_grads_blend(params, opacity, height, width, dl_dimage, mode="alpha", cov="chol",
                   rel_step=1e-6):
    """Central differences of sum(dL/dC * C) in float64 with the tile lists held fixed (a
    parameter change that moves a Gaussian across a tile edge is outside the derivative)."""
    p0 = _f64(params, 8)
    o0 = _f64(opacity, 0)
    G = np.asarray(dl_dimage, np.float64)
    lists = ref.tile_lists(params, height, width, cov)
    out = np.zeros((p0.shape[0], 9))

    def loss(p, o):
        inv = ref._inv_from(p, cov)
        return float((_render64(p, o, height, width, mode, cov, lists, inv) * G).sum())

    for n in range(p0.shape[0]):
        for k in range(9):
            p, o = p0.copy(), o0.copy()
            base = o0[n] if k == 8 else p0[n, k]
            h = rel_step * max(abs(base), 1.0)
            if k == 8:
                o[n] = base + h
                up = loss(p, o)
                o[n] = base - h
                dn = loss(p, o)
            else:
                p[n, k] = base + h
                up = loss(p, o)
                p[n, k] = base - h
                dn = loss(p, o)
            out[n, k] = (up - dn) / (2 * h)
    return out[:, :8], out[:, 8]


def adam_opacity_step(opacity, m, v, grad, step: int, hp=None):
    """Adam with bias correction on the opacities (learning rate lr_c, no floor): the same
    update as ``ref.adam_step`` applies to the colour slots.  Returns float64 (o, m, v)."""
    hp = dict(ref.DEFAULT_ADAM if hp is None else hp)
    g = np.asarray(grad, np.float64)
    m = hp["beta1"] * np.asarray(m, np.float64) + (1.0 - hp["beta1"]) * g
    v = hp["beta2"] * np.asarray(v, np.float64) + (1.0 - hp["beta2"]) * g * g
    mhat = m / (1.0 - hp["beta1"] ** step)
    vhat = v / (1.0 - hp["beta2"] ** step)
    o = np.asarray(opacity, np.float64) - hp["lr_c"] * mhat / (np.sqrt(vhat) + hp["eps"])
    return o, m, v
