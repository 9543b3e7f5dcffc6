"""Pins of the codec decode oracle (Sec. 3.3) against definitions that do not go through it:
the IEEE binary16 bit layout, the closed forms of the LSQ+ dequantisation, the quantisation
error bound, and brute-force residual vector quantisation.  CPU only."""
import math

import numpy as np

import synth
from oracle import codec, ref


def test_binary16_decode_matches_the_bit_layout():
    bits = np.arange(1 << 16, dtype=np.uint32)
    sign = np.where(bits >> 15, -1.0, 1.0)
    e = (bits >> 10) & 0x1F
    f = (bits & 0x3FF).astype(np.float64)
    want = np.where(e == 0, sign * f * 2.0 ** -24,                 # subnormals and zeros
                    sign * (1.0 + f / 1024.0) * 2.0 ** (e.astype(np.float64) - 15.0))
    got = codec.decode_mu(bits.astype(np.uint16).reshape(-1, 2)).reshape(-1)
    fin = e != 31
    np.testing.assert_array_equal(got[fin], want[fin])
    assert np.all(np.isinf(got[(e == 31) & (f == 0)])) and np.all(np.isnan(got[(e == 31) & (f > 0)]))
    assert got[0x7BFF] == 65504.0 and got[0x3C00] == 1.0 and got[0x0001] == 2.0 ** -24


def test_dequantisation_closed_forms():
    gamma = np.array([0.125, 0.046875, 3.0], np.float32)
    beta = np.array([1.0, -1.5, -96.0], np.float32)
    codes = np.array([[0, 0, 0], [63, 63, 63], [1, 32, 17]])
    got = codec.dequantise_l(codes, gamma, beta)
    np.testing.assert_array_equal(got[0], [1.0, -1.5, -96.0])
    np.testing.assert_array_equal(got[1], [1.0 + 63 * 0.125, -1.5 + 63 * 0.046875, 93.0])
    np.testing.assert_array_equal(got[2], [1.125, 0.0, -45.0])


def test_quantisation_error_is_at_most_half_a_step():
    rng = np.random.default_rng(3)
    cs = synth.codec_set(4000, 64, 64, seed=4)
    lo = cs.beta.astype(np.float64)
    hi = lo + 63 * cs.gamma.astype(np.float64)
    p = np.zeros((4000, 8))
    p[:, 2:5] = rng.uniform(lo - 1.0, hi + 1.0, (4000, 3))
    _, lhat, _ = codec.quantise(p, cs.gamma, cs.beta, cs.codebooks, 6)
    back = codec.dequantise_l(lhat, cs.gamma, cs.beta)
    inside = (p[:, 2:5] >= lo) & (p[:, 2:5] <= hi)
    step = cs.gamma.astype(np.float64)
    err = np.abs(back - p[:, 2:5])
    assert np.all(err[inside] <= (0.5 + 1e-9) * np.broadcast_to(step, err.shape)[inside])
    # outside the range the code saturates at 0 or 2^b - 1
    assert np.all(lhat[p[:, 2:5] < lo] == 0) and np.all(lhat[p[:, 2:5] > hi] == 63)


def test_rvq_stages_pick_the_nearest_entry_by_brute_force():
    rng = np.random.default_rng(5)
    cs = synth.codec_set(300, 32, 32, seed=6, stages=3, book=8)
    p = np.zeros((300, 8))
    p[:, 5:8] = rng.uniform(-0.3, 1.3, (300, 3))
    _, _, idx = codec.quantise(p, cs.gamma, cs.beta, cs.codebooks, 6)
    cb = cs.codebooks.astype(np.float64)
    for n in range(300):
        resid = p[n, 5:8].copy()
        for m in range(3):
            dists = [sum((resid[k] - cb[m, j, k]) ** 2 for k in range(3)) for j in range(8)]
            best = min(dists)
            assert dists[idx[n, m]] == best and idx[n, m] == dists.index(best)
            resid = resid - cb[m, idx[n, m]]
    # decoded colour = sum of the chosen entries
    col = codec.rvq_colour(idx, cs.codebooks)
    want = cb[0][idx[:, 0]] + cb[1][idx[:, 1]] + cb[2][idx[:, 2]]
    np.testing.assert_allclose(col, want, rtol=0, atol=1e-15)


def test_rvq_is_exact_when_the_first_codebook_holds_the_colours():
    cs = synth.codec_set(50, 16, 16, seed=7)
    books = np.zeros((2, 8, 3), np.float32)
    books[0] = cs.codebooks[0]
    p = np.zeros((50, 8))
    p[:, 5:8] = books[0][np.arange(50) % 8]
    _, _, idx = codec.quantise(p, cs.gamma, cs.beta, books, 6)
    np.testing.assert_array_equal(idx[:, 0], np.arange(50) % 8)
    np.testing.assert_array_equal(codec.rvq_colour(idx, books), p[:, 5:8])


def test_invalid_codes_and_indices_take_no_part():
    cs = synth.codec_set(6, 40, 40, seed=8)
    codes = cs.codes.copy()
    index = cs.index.copy()
    codes[1, 2] = 64        # above 2^6 - 1
    index[3, 1] = 8         # outside a codebook of 8
    dec = codec.decode(cs.mu_bits, codes, index, cs.gamma, cs.beta, cs.codebooks, 6)
    bad = np.isnan(dec).all(axis=1)
    np.testing.assert_array_equal(bad, [False, True, False, True, False, False])
    act = ref.active(dec.astype(np.float32))
    assert not act[1] and not act[3] and act[[0, 2, 4, 5]].all()


def test_decode_of_quantised_records_reproduces_them_within_the_codec_steps():
    rng = np.random.default_rng(9)
    n = 500
    p = np.zeros((n, 8))
    p[:, 0] = rng.uniform(0, 700, n)
    p[:, 1] = rng.uniform(0, 500, n)
    cs = synth.codec_set(n, 512, 768, seed=10)
    lo = cs.beta.astype(np.float64)
    p[:, 2:5] = rng.uniform(lo, lo + 63 * cs.gamma.astype(np.float64), (n, 3))
    p[:, 5:8] = rng.uniform(0, 1, (n, 3))
    mu, lhat, idx = codec.quantise(p, cs.gamma, cs.beta, cs.codebooks, 6)
    dec = codec.decode(mu, lhat, idx, cs.gamma, cs.beta, cs.codebooks, 6)
    # binary16 keeps 11 significant bits: |mu| < 1024 is within 2^-2 after rounding
    assert np.all(np.abs(dec[:, :2] - p[:, :2]) <= 0.25)
    assert np.all(np.abs(dec[:, 2:5] - p[:, 2:5]) <= 0.5 * cs.gamma.astype(np.float64) + 1e-12)
    assert math.isfinite(dec.sum())
