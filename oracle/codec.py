"""Plain FP64 oracle of the codec's decode side (Sec. 3.3, attribute quantisation).

TEST INFRASTRUCTURE.  Only the tests, the smoke check and the CPU-baseline leg of the benchmark
may import or call this module.  It shares no code with the GPU path and never imports it.

A compressed Gaussian set holds, per Gaussian n:
  * the position as two IEEE binary16 numbers (Sec. 3.3: 16-bit floats for positions);
  * three b-bit codes of the covariance vector, dequantised with a scale gamma_i and an offset
    beta_i shared by all Gaussians (Sec. 3.3, the LSQ+ equation: l_bar = l_hat * gamma + beta);
  * M residual vector quantisation indices, one per stage, into codebooks C^m of B colours
    (Sec. 3.3, the RVQ equation: the colour is the sum over stages of C^m[i^m]).
Decoding gives the 8-number record (mu_x, mu_y, l1, l2, l3, c0, c1, c2) that the renderer takes
(Sec. 3.2).  Readings taken here: codes outside [0, 2^b - 1] and indices outside [0, B - 1] are
invalid, and such a Gaussian takes no part (it decodes to NaN here, which ``ref`` treats as
inactive); the stages are summed in stage order.

The encoding side (``quantise``) restates the same equations the other way round: the code is
round(clamp((l - beta) / gamma, 0, 2^b - 1)) with ties to even, and each RVQ stage takes the
codebook entry nearest to the residual left by the previous stages (squared Euclidean distance,
lowest index on ties).  It produces test inputs and checks the decode; it is not on the
rendering path.
"""
from __future__ import annotations

import numpy as np


def decode_mu(mu_half_bits) -> np.ndarray:
    """binary16 bit patterns [N, 2] (uint16) -> float64 positions (exact)."""
    return np.asarray(mu_half_bits, np.uint16).view(np.float16).astype(np.float64)


def dequantise_l(codes, gamma, beta) -> np.ndarray:
    """LSQ+ dequantisation l_bar = l_hat * gamma_i + beta_i per component (Sec. 3.3), float64.
    ``gamma``, ``beta`` are float32 values; the product and sum are formed in float64."""
    c = np.asarray(codes, np.float64)
    g = np.asarray(gamma, np.float32).astype(np.float64)
    b = np.asarray(beta, np.float32).astype(np.float64)
    return c * g[None, :] + b[None, :]


def rvq_colour(indices, codebooks) -> np.ndarray:
    """RVQ colour: sum over the M stages of C^m[i^m] (Sec. 3.3), float64.  ``indices`` [N, M],
    ``codebooks`` [M, B, 3] float32."""
    cb = np.asarray(codebooks, np.float32).astype(np.float64)
    idx = np.asarray(indices, np.int64)
    out = np.zeros((idx.shape[0], 3))
    for m in range(cb.shape[0]):
        out += cb[m][idx[:, m]]
    return out


def valid(l_codes, indices, bits: int, book_size: int) -> np.ndarray:
    lc = np.asarray(l_codes, np.int64)
    ix = np.asarray(indices, np.int64)
    ok = np.all((lc >= 0) & (lc <= (1 << bits) - 1), axis=1)
    return ok & np.all((ix >= 0) & (ix < book_size), axis=1)


def decode(mu_half_bits, l_codes, indices, gamma, beta, codebooks, bits: int) -> np.ndarray:
    """Full decode to float64 records [N, 8]; invalid Gaussians are all NaN."""
    cb = np.asarray(codebooks, np.float32)
    n = np.asarray(l_codes).shape[0]
    out = np.empty((n, 8))
    out[:, 0:2] = decode_mu(mu_half_bits)
    ok = valid(l_codes, indices, bits, cb.shape[1])
    lc = np.where(ok[:, None], np.asarray(l_codes, np.int64), 0)
    ix = np.where(ok[:, None], np.asarray(indices, np.int64), 0)
    out[:, 2:5] = dequantise_l(lc, gamma, beta)
    out[:, 5:8] = rvq_colour(ix, cb)
    out[~ok] = np.nan
    return out


def quantise(params, gamma, beta, codebooks, bits: int):
    """Encode float records: (mu binary16 bits [N, 2], l codes [N, 3], RVQ indices [N, M])."""
    p = np.asarray(params, np.float64).reshape(-1, 8)
    mu = p[:, 0:2].astype(np.float16).view(np.uint16)
    g = np.asarray(gamma, np.float32).astype(np.float64)
    b = np.asarray(beta, np.float32).astype(np.float64)
    lhat = np.rint(np.clip((p[:, 2:5] - b) / g, 0, (1 << bits) - 1)).astype(np.uint8)
    cb = np.asarray(codebooks, np.float32).astype(np.float64)
    resid = p[:, 5:8].copy()
    idx = np.empty((p.shape[0], cb.shape[0]), np.uint8)
    for m in range(cb.shape[0]):
        d = ((resid[:, None, :] - cb[m][None, :, :]) ** 2).sum(-1)
        idx[:, m] = np.argmin(d, axis=1)  # first minimum: lowest index on ties
        resid -= cb[m][idx[:, m]]
    return mu, lhat, idx
