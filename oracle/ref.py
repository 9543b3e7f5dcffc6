"""Plain FP64 CPU oracle of the accumulated-summation 2-D Gaussian rasteriser.

TEST INFRASTRUCTURE.  Only the tests, the smoke check and the CPU-baseline leg of the benchmark
may import or call this module.  It shares no code with the GPU path and never imports it.

Everything is evaluated in float64 from float32 inputs cast exactly to float64.  Each function
cites the passage of the paper it restates.  Readings of points the paper leaves open are listed
next to the function that takes them.

Record layout (Sec. 3.2, Eq. rasterization4: position, covariance and weighted colour, 8 numbers):
``(mu_x, mu_y, l1, l2, l3, c0, c1, c2)``, pixel units, ``L = [[l1, 0], [l2, l3]]``, Sigma = L L^T
(Sec. 3.1, Eq. cholesky).

Readings taken here (the paper is silent on them):
  * the centre of pixel (x, y) is (x + 0.5, y + 0.5) and d = p - mu (Sec. 3.2 calls d the
    displacement between the pixel centre and the Gaussian centre, but fixes neither);
  * the rasteriser is tile based (Sec. 1 and Sec. 4.1 build on the tile-based rasteriser of
    3D-GS); a Gaussian reaches every pixel of each 16x16 tile that its 3-sigma box touches, and
    no other pixel.  The box half-width is r = ceil(3 sqrt(lambda_max)) in whole pixels,
    decided exactly (see ``radius``);
  * no clamp and no background: uncovered pixels are 0 and colours are unbounded (Sec. 3.2);
  * a Gaussian is inactive (no tiles, no contribution, zero gradient) when any of its numbers is
    not finite, when |l1| or |l3| < 2^-24, or when |l2|, |mu_x| or |mu_y| > 2^24.
"""
from __future__ import annotations

import math

import numpy as np

TILE = 16
R_MAX = 2 ** 25
L_MIN_ABS = 2.0 ** -24
BIG_ABS = 2.0 ** 24


def _f64(params) -> np.ndarray:
    p = np.asarray(params)
    if p.dtype != np.float32:
        p = p.astype(np.float32)
    return p.astype(np.float64).reshape(-1, 8)


# ---------------------------------------------------------------- Gaussian formation (Sec. 3.1)
#
# Two factorisations of the covariance (Sec. 3.1): ``cov="chol"`` reads the record as
# (mu_x, mu_y, l1, l2, l3, c0, c1, c2) with Sigma = L L^T, L = [[l1, 0], [l2, l3]]
# (Eq. cholesky); ``cov="rs"`` reads it as (mu_x, mu_y, s1, s2, theta, c0, c1, c2) with
# Sigma = (R S)(R S)^T, R the rotation by theta and S = diag(s1, s2) (Eq. RSSR, rot_scale).

def _cov_from(p, cov):
    """Sigma entries (s00, s01, s11) of float64 records (no float32 rounding)."""
    if cov == "chol":
        l1, l2, l3 = p[:, 2], p[:, 3], p[:, 4]
        return l1 * l1, l1 * l2, l2 * l2 + l3 * l3
    if cov == "rs":
        s1, s2, th = p[:, 2], p[:, 3], p[:, 4]
        c, s = np.cos(th), np.sin(th)
        a, b = s1 * s1, s2 * s2
        return c * c * a + s * s * b, c * s * (a - b), s * s * a + c * c * b
    raise ValueError(cov)


def _det_from(p, cov):
    """det Sigma in product form: (l1 l3)^2 or (s1 s2)^2."""
    if cov == "chol":
        return (p[:, 2] * p[:, 4]) ** 2
    return (p[:, 2] * p[:, 3]) ** 2


def _inv_from(p, cov):
    s00, s01, s11 = _cov_from(p, cov)
    det = _det_from(p, cov)
    with np.errstate(divide="ignore", invalid="ignore"):
        return s11 / det, -s01 / det, s00 / det


def covariance(params, cov="chol"):
    """Sigma entries ``(s00, s01, s11)`` of the records (Sec. 3.1, Eq. cholesky or Eq. RSSR):
    for the Cholesky vector (l1^2, l1 l2, l2^2 + l3^2)."""
    return _cov_from(_f64(params), cov)


def inverse_covariance(params, cov="chol"):
    """Sigma^{-1} = [[s11, -s01], [-s01, s00]] / det (Sec. 3.2, Eq. rasterization2 needs
    Sigma^{-1}), det in product form.  Returns ``(i00, i01, i11)``."""
    return _inv_from(_f64(params), cov)


def active(params, cov="chol") -> np.ndarray:
    """Which Gaussians take part (the domain reading in the module header; for the
    rotation-scale form |s1|, |s2| >= 2^-24 and |theta| <= 2^24)."""
    p = _f64(params)
    finite = np.all(np.isfinite(p), axis=1)
    with np.errstate(invalid="ignore"):
        if cov == "chol":
            dom = ((np.abs(p[:, 2]) >= L_MIN_ABS) & (np.abs(p[:, 4]) >= L_MIN_ABS)
                   & (np.abs(p[:, 3]) <= BIG_ABS))
        else:
            dom = ((np.abs(p[:, 2]) >= L_MIN_ABS) & (np.abs(p[:, 3]) >= L_MIN_ABS)
                   & (np.abs(p[:, 4]) <= BIG_ABS))
        dom &= (np.abs(p[:, 0]) <= BIG_ABS) & (np.abs(p[:, 1]) <= BIG_ABS)
    return finite & dom


# ---------------------------------------------------------------- tile binning

def _covers(r: np.ndarray, s00, s01, s11) -> np.ndarray:
    """True where the integer r satisfies r >= 3 sqrt(lambda_max(Sigma)).

    r^2 >= 9 lambda_max holds exactly when, with R = r^2, p = R - 9 s00 and q = R - 9 s11, both
    p + q >= 0 and p q >= 81 s01^2 (R/9 then lies at or above the larger root of the
    characteristic polynomial of Sigma).  Each step is one IEEE float64 operation in this fixed
    order, so any IEEE machine that follows the same order reaches the same decision.
    """
    rr = r.astype(np.float64)
    R = rr * rr
    p = R - 9.0 * s00
    q = R - 9.0 * s11
    return ((p + q) >= 0.0) & ((p * q) >= 81.0 * (s01 * s01))


def radius(params, cov="chol") -> np.ndarray:
    """Box half-width r = ceil(3 sqrt(lambda_max)) in pixels, capped at 2^25 (int64, 0 if
    inactive).  The cap covers any image once |mu| <= 2^24.

    Defined as the least integer r in [0, 2^25] for which ``_covers`` holds (2^25 if none).  The
    float64 square root only gives the starting guess; the search then moves to that least r.
    """
    act = active(params, cov)
    if cov == "rs":
        return _radius_rs(params, act)
    with np.errstate(invalid="ignore", over="ignore"):
        s00, s01, s11 = covariance(params, cov)
        lam = 0.5 * (s00 + s11) + np.sqrt(0.25 * (s00 - s11) ** 2 + s01 * s01)
        guess = np.ceil(3.0 * np.sqrt(lam))
    guess = np.where(act & np.isfinite(guess), guess, 0.0)
    r = np.clip(guess, 0, R_MAX).astype(np.int64)
    s00 = np.where(act, s00, 0.0)
    s01 = np.where(act, s01, 0.0)
    s11 = np.where(act, s11, 0.0)
    while True:  # step down while r - 1 still covers
        down = act & (r > 0) & _covers(r - 1, s00, s01, s11)
        if not down.any():
            break
        r = r - down
    while True:  # step up while r does not cover
        up = act & (r < R_MAX) & ~_covers(r, s00, s01, s11)
        if not up.any():
            break
        r = r + up
    return np.where(act, r, 0)


def _radius_rs(params, act) -> np.ndarray:
    """Box half-width of the rotation-scale form.  Sigma = R S S^T R^T has the eigenvalues s1^2
    and s2^2 (Eq. RSSR: R is orthogonal), so lambda_max = max(s1^2, s2^2) and r is the least
    integer in [0, 2^25] with r^2 >= 9 max(s1^2, s2^2).  For float32 s1, s2 every product below
    is exact in float64, so the decision involves no rounding and no trigonometry.
    """
    p = _f64(params)
    m = np.where(act, np.maximum(p[:, 2] * p[:, 2], p[:, 3] * p[:, 3]), 0.0)
    with np.errstate(invalid="ignore", over="ignore"):
        guess = np.ceil(3.0 * np.sqrt(m))
    r = np.clip(np.where(act & np.isfinite(guess), guess, 0.0), 0, R_MAX).astype(np.int64)
    while True:
        rr = (r - 1).astype(np.float64)
        down = act & (r > 0) & (rr * rr >= 9.0 * m)
        if not down.any():
            break
        r = r - down
    while True:
        rr = r.astype(np.float64)
        up = act & (r < R_MAX) & (rr * rr < 9.0 * m)
        if not up.any():
            break
        r = r + up
    return np.where(act, r, 0)


def grid_tiles(height: int, width: int):
    """Tile grid of an image: (tiles across, tiles down), ceil(W/16) by ceil(H/16)."""
    return -(-width // TILE), -(-height // TILE)


def tile_rects(params, height: int, width: int, cov="chol"):
    """Per Gaussian, the inclusive tile rectangle (tx0, ty0, tx1, ty1) its 3-sigma box touches,
    and the tile count.  Inactive or off-image Gaussians get count 0 and rect (0, 0, -1, -1).

    tx0 = max(floor((mu_x - r) / 16), 0), tx1 = min(floor((mu_x + r) / 16), TW - 1), and the same
    along y, all in float64 (mu_x - r and the division by 16 are exact for |mu| <= 2^24).
    """
    p = _f64(params)
    tw, th = grid_tiles(height, width)
    r = radius(params, cov).astype(np.float64)
    act = active(params, cov)
    mx = np.where(act, p[:, 0], 0.0)
    my = np.where(act, p[:, 1], 0.0)
    fx0 = np.maximum(np.floor((mx - r) / TILE), 0.0)
    fx1 = np.minimum(np.floor((mx + r) / TILE), tw - 1.0)
    fy0 = np.maximum(np.floor((my - r) / TILE), 0.0)
    fy1 = np.minimum(np.floor((my + r) / TILE), th - 1.0)
    ok = act & (fx0 <= fx1) & (fy0 <= fy1)
    rect = np.stack([fx0, fy0, fx1, fy1], axis=1)
    rect = np.where(ok[:, None], rect, np.array([0.0, 0.0, -1.0, -1.0])).astype(np.int64)
    count = np.where(ok, (rect[:, 2] - rect[:, 0] + 1) * (rect[:, 3] - rect[:, 1] + 1), 0)
    return rect, count.astype(np.int64)


def tile_lists(params, height: int, width: int, cov="chol"):
    """The per-tile Gaussian lists with depth order removed (Sec. 3.2: the sum does not depend on
    order, so only membership matters; ties are listed by ascending Gaussian index).

    Returns ``(ranges [T, 2], ids [K])`` where tile t (row-major, t = ty * TW + tx) owns
    ``ids[ranges[t, 0]:ranges[t, 1]]``, found by enumerating each rectangle.
    """
    tw, th = grid_tiles(height, width)
    rect, count = tile_rects(params, height, width, cov)
    tiles, owners = [], []
    for n in np.nonzero(count)[0]:
        tx0, ty0, tx1, ty1 = rect[n]
        ty, tx = np.meshgrid(np.arange(ty0, ty1 + 1), np.arange(tx0, tx1 + 1), indexing="ij")
        tiles.append((ty * tw + tx).ravel())
        owners.append(np.full(tiles[-1].size, n, dtype=np.int64))
    if tiles:
        t_all = np.concatenate(tiles)
        n_all = np.concatenate(owners)
    else:
        t_all = np.zeros(0, np.int64)
        n_all = np.zeros(0, np.int64)
    order = np.lexsort((n_all, t_all))
    t_sorted = t_all[order]
    ids = n_all[order]
    starts = np.searchsorted(t_sorted, np.arange(tw * th), side="left")
    ends = np.searchsorted(t_sorted, np.arange(tw * th), side="right")
    return np.stack([starts, ends], axis=1).astype(np.int64), ids


# ---------------------------------------------------------------- forward (Sec. 3.2)

def _gauss_box(rect_row, height, width):
    tx0, ty0, tx1, ty1 = rect_row
    x0, x1 = tx0 * TILE, min((tx1 + 1) * TILE, width)
    y0, y1 = ty0 * TILE, min((ty1 + 1) * TILE, height)
    return x0, x1, y0, y1


def _sigma(pn, inv, xs, ys):
    """sigma = 1/2 d^T Sigma^{-1} d with d = pixel centre - mu (Sec. 3.2, Eq. rasterization2)."""
    dx = (xs + 0.5)[None, :] - pn[0]
    dy = (ys + 0.5)[:, None] - pn[1]
    i00, i01, i11 = inv
    return 0.5 * (i00 * dx * dx + 2.0 * i01 * dx * dy + i11 * dy * dy), dx, dy


def render_full(params, height: int, width: int, cov="chol") -> np.ndarray:
    """C_i = sum over all Gaussians of c'_n exp(-sigma_n) at every pixel (Sec. 3.2,
    Eq. rasterization4), with no culling.  float64 ``[H, W, 3]``."""
    p = _f64(params)
    act = active(params, cov)
    i00, i01, i11 = inverse_covariance(params, cov)
    img = np.zeros((height, width, 3))
    xs = np.arange(width, dtype=np.float64)
    ys = np.arange(height, dtype=np.float64)
    for n in np.nonzero(act)[0]:
        s, _, _ = _sigma(p[n], (i00[n], i01[n], i11[n]), xs, ys)
        img += np.exp(-s)[:, :, None] * p[n, 5:8]
    return img


def render_culled(params, height: int, width: int, with_abs: bool = False, cov="chol"):
    """Eq. rasterization4 restricted to the tile support: Gaussian n reaches pixel p only when the
    tile of p lies in n's tile rectangle.  Returns the float64 image, and with ``with_abs`` also
    A(p) = sum |c'_n| exp(-sigma_n(p)) over the same support (the scale for relative error)."""
    p = _f64(params)
    rect, count = tile_rects(params, height, width, cov)
    i00, i01, i11 = inverse_covariance(params, cov)
    img = np.zeros((height, width, 3))
    aimg = np.zeros((height, width, 3)) if with_abs else None
    for n in np.nonzero(count)[0]:
        x0, x1, y0, y1 = _gauss_box(rect[n], height, width)
        xs = np.arange(x0, x1, dtype=np.float64)
        ys = np.arange(y0, y1, dtype=np.float64)
        s, _, _ = _sigma(p[n], (i00[n], i01[n], i11[n]), xs, ys)
        e = np.exp(-s)[:, :, None]
        img[y0:y1, x0:x1] += e * p[n, 5:8]
        if with_abs:
            aimg[y0:y1, x0:x1] += e * np.abs(p[n, 5:8])
    if with_abs:
        return img, aimg
    return img


# ---------------------------------------------------------------- backward (App. A)

def grads(params, height: int, width: int, dl_dimage, culled: bool = True, with_abs=False,
          cov="chol"):
    """dL/dparams from dL/dC (App. A), float64 ``[N, 8]`` in record order.

    Per pixel and Gaussian (App. A.1): dC^k/dc'^k = e with e = exp(-sigma); dC^k/dsigma =
    -c'^k e (the printed form drops the colour factor); dsigma/dmu = -Sigma^{-1} d (d = p - mu;
    the printed +Sigma^{-1} d holds for d = mu - p); dsigma/dSigma = -1/2 Sigma^{-1} d d^T
    Sigma^{-1}.  Per Gaussian (App. A.2), with G = dL/dSigma = [[g1, g2], [g2, g3]]:
    dL/dl1 = 2 g1 l1 + 2 g2 l2, dL/dl2 = 2 g2 l1 + 2 g3 l2 (the printed "+ g2 l2" is a slip:
    <G, dSigma/dl2> with dSigma/dl2 = [[0, l1], [l1, 2 l2]] gives 2 g3 l2), dL/dl3 = 2 g3 l3.
    For the rotation-scale form (App. A.2, second part), dL/dtheta = <G, R' S S^T R^T +
    R S S^T R'^T>, dL/ds1 = <G, R diag(2 s1, 0) R^T>, dL/ds2 = <G, R diag(0, 2 s2) R^T> (the
    printed lines drop the inner product with G and write s1 for s2 in the last one).

    With ``with_abs`` also returns, per parameter, the sum over pixels of the absolute value of
    each pixel's contribution (the scale for relative error).
    """
    p = _f64(params)
    G = np.asarray(dl_dimage, dtype=np.float64).reshape(height, width, 3)
    n_g = p.shape[0]
    out = np.zeros((n_g, 8))
    absd = np.zeros((n_g, 8))
    rect, count = tile_rects(params, height, width, cov)
    act = active(params, cov)
    i00, i01, i11 = inverse_covariance(params, cov)
    which = np.nonzero(count)[0] if culled else np.nonzero(act)[0]
    for n in which:
        if culled:
            x0, x1, y0, y1 = _gauss_box(rect[n], height, width)
        else:
            x0, x1, y0, y1 = 0, width, 0, height
        xs = np.arange(x0, x1, dtype=np.float64)
        ys = np.arange(y0, y1, dtype=np.float64)
        s, dx, dy = _sigma(p[n], (i00[n], i01[n], i11[n]), xs, ys)
        e = np.exp(-s)
        g = G[y0:y1, x0:x1]
        dc = g * e[:, :, None]                                   # dL/dc'^k per pixel
        dsig = -e * (g @ p[n, 5:8])                              # dL/dsigma per pixel
        vx = i00[n] * dx + i01[n] * dy                           # Sigma^{-1} d
        vy = i01[n] * dx + i11[n] * dy
        dmx = dsig * (-vx)
        dmy = dsig * (-vy)
        g1 = dsig * (-0.5 * vx * vx)                             # dL/dSigma per pixel
        g2 = dsig * (-0.5 * vx * vy)
        g3 = dsig * (-0.5 * vy * vy)
        if cov == "chol":
            l1, l2, l3 = p[n, 2], p[n, 3], p[n, 4]
            dl1 = 2.0 * g1 * l1 + 2.0 * g2 * l2
            dl2 = 2.0 * g2 * l1 + 2.0 * g3 * l2
            dl3 = 2.0 * g3 * l3
            shape = [dl1, dl2, dl3]
        else:
            s1, s2, th = p[n, 2], p[n, 3], p[n, 4]
            c, sn = math.cos(th), math.sin(th)
            R = np.array([[c, -sn], [sn, c]])
            dR = np.array([[-sn, -c], [c, -sn]])
            SS = np.diag([s1 * s1, s2 * s2])
            dS_th = dR @ SS @ R.T + R @ SS @ dR.T
            dS_s1 = R @ np.diag([2.0 * s1, 0.0]) @ R.T
            dS_s2 = R @ np.diag([0.0, 2.0 * s2]) @ R.T

            def inner(M):  # <G, M> with G = [[g1, g2], [g2, g3]] per pixel
                return g1 * M[0, 0] + g2 * (M[0, 1] + M[1, 0]) + g3 * M[1, 1]
            shape = [inner(dS_s1), inner(dS_s2), inner(dS_th)]
        parts = [dmx, dmy, *shape, dc[..., 0], dc[..., 1], dc[..., 2]]
        for k, q in enumerate(parts):
            out[n, k] = q.sum()
            if with_abs:
                absd[n, k] = np.abs(q).sum()
    if with_abs:
        return out, absd
    return out


def fd_grads(params, height: int, width: int, dl_dimage, which=None, rel_step=1e-6,
             culled: bool = True, cov="chol"):
    """Central finite differences of S = <dL/dC, C> in float64, h = rel_step * max(1, |theta|).

    For the culled sum the tile rectangles must not move under +-h; the perturbed Gaussian's
    rect is checked and a ValueError raised where it does.  ``which`` lists the Gaussians to
    differentiate (default: all).
    """
    base = _f64(params)
    G = np.asarray(dl_dimage, dtype=np.float64).reshape(height, width, 3)
    idx = range(base.shape[0]) if which is None else which
    out = np.zeros((base.shape[0], 8))
    rect0, _ = tile_rects(base.astype(np.float32), height, width, cov) if culled else (None, None)
    for n in idx:
        for k in range(8):
            h = rel_step * max(1.0, abs(base[n, k]))
            vals = []
            for sgn in (1.0, -1.0):
                q = base.copy()
                q[n, k] += sgn * h
                vals.append(np.sum(G * _render64(q, height, width, culled, rect0, n, cov)))
            out[n, k] = (vals[0] - vals[1]) / (2.0 * h)
    return out


def fd_local(params, height: int, width: int, dl_dimage, n: int, rel_step=1e-6, cov="chol"):
    """Central finite differences of S = <dL/dC, C> for Gaussian n alone, float64.

    Only Gaussian n's own term changes when its parameters move, so S(theta + h) - S(theta - h)
    is evaluated over n's tile support (held at the unperturbed rectangle, which the caller
    checks does not move) without touching the other Gaussians.  Returns the 8 derivatives.
    """
    p = _f64(params)[n].copy()
    G = np.asarray(dl_dimage, dtype=np.float64).reshape(height, width, 3)
    rect, count = tile_rects(np.asarray(params, np.float32)[n:n + 1], height, width, cov)
    out = np.zeros(8)
    if count[0] == 0:
        return out
    x0, x1, y0, y1 = _gauss_box(rect[0], height, width)
    xs = np.arange(x0, x1, dtype=np.float64)
    ys = np.arange(y0, y1, dtype=np.float64)
    g = G[y0:y1, x0:x1]

    def term(q):
        inv = tuple(v[0] for v in _inv_from(q[None, :], cov))
        s, _, _ = _sigma(q, inv, xs, ys)
        return np.sum(g * (np.exp(-s)[:, :, None] * q[5:8]))

    for k in range(8):
        h = rel_step * max(1.0, abs(p[k]))
        qp, qm = p.copy(), p.copy()
        qp[k] += h
        qm[k] -= h
        out[k] = (term(qp) - term(qm)) / (2.0 * h)
    return out


def _render64(p64, height, width, culled, rect0, moved, cov="chol"):
    """Render float64 parameters (no float32 rounding), used by finite differences only.  With
    ``culled`` the support is the unperturbed ``rect0``, after checking that the perturbed
    Gaussian's own float64 rect equals it."""
    img = np.zeros((height, width, 3))
    i00, i01, i11 = _inv_from(p64, cov)
    xs_all = np.arange(width, dtype=np.float64)
    ys_all = np.arange(height, dtype=np.float64)
    if culled:
        s00, s01, s11 = (v[0] for v in _cov_from(p64[moved:moved + 1], cov))
        lam = 0.5 * (s00 + s11) + math.sqrt(0.25 * (s00 - s11) ** 2 + s01 ** 2)
        r = math.ceil(3.0 * math.sqrt(lam))
        tw, th = grid_tiles(height, width)
        mx, my = p64[moved, 0], p64[moved, 1]
        new = [max(math.floor((mx - r) / TILE), 0), max(math.floor((my - r) / TILE), 0),
               min(math.floor((mx + r) / TILE), tw - 1), min(math.floor((my + r) / TILE), th - 1)]
        if list(rect0[moved]) != new and rect0[moved][2] >= 0:
            raise ValueError(f"tile rect of Gaussian {moved} moves under the FD step")
    for n in range(p64.shape[0]):
        if culled:
            if rect0[n][2] < 0:
                continue
            x0, x1, y0, y1 = _gauss_box(rect0[n], height, width)
            xs, ys = xs_all[x0:x1], ys_all[y0:y1]
        else:
            x0, x1, y0, y1 = 0, width, 0, height
            xs, ys = xs_all, ys_all
        s, _, _ = _sigma(p64[n], (i00[n], i01[n], i11[n]), xs, ys)
        img[y0:y1, x0:x1] += np.exp(-s)[:, :, None] * p64[n, 5:8]
    return img


# ---------------------------------------------------------------- loss and update

def mse(image, target) -> float:
    """L2 reconstruction loss (Sec. 3.4): mean over H*W*3 of (C - T)^2."""
    d = np.asarray(image, np.float64) - np.asarray(target, np.float64)
    return float(np.mean(d * d))


def mse_grad(image, target) -> np.ndarray:
    """dL/dC of ``mse``: 2 (C - T) / (3 H W)."""
    d = np.asarray(image, np.float64) - np.asarray(target, np.float64)
    return 2.0 * d / d.size


DEFAULT_ADAM = dict(lr_mu=0.05, lr_l=0.01, lr_c=0.005, beta1=0.9, beta2=0.999, eps=1e-8,
                    l_min=0.5)


def adam_step(params, m, v, grad, step: int, hp=None, cov="chol"):
    """One Adam update with bias correction (Kingma and Ba), per-group learning rates for
    position, covariance factors and colour, then |l1|, |l3| (or |s1|, |s2|) held at >= l_min
    (the paper keeps them away from zero by adding 0.5, App. C; outside the record, so here a
    floor).

    Returns new float64 ``(params, m, v)``; ``step`` counts from 1.
    """
    hp = dict(DEFAULT_ADAM if hp is None else hp)
    p = np.array(params, np.float64).reshape(-1, 8)
    g = np.asarray(grad, np.float64).reshape(-1, 8)
    m = hp["beta1"] * np.asarray(m, np.float64).reshape(-1, 8) + (1.0 - hp["beta1"]) * g
    v = hp["beta2"] * np.asarray(v, np.float64).reshape(-1, 8) + (1.0 - hp["beta2"]) * g * g
    mhat = m / (1.0 - hp["beta1"] ** step)
    vhat = v / (1.0 - hp["beta2"] ** step)
    lr = np.array([hp["lr_mu"]] * 2 + [hp["lr_l"]] * 3 + [hp["lr_c"]] * 3)
    p = p - lr * mhat / (np.sqrt(vhat) + hp["eps"])
    if hp["l_min"] > 0:
        for k in ((2, 4) if cov == "chol" else (2, 3)):
            small = np.abs(p[:, k]) < hp["l_min"]
            p[small, k] = np.copysign(hp["l_min"], p[small, k])
    return p, m, v
