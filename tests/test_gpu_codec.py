"""Parity of the codec decode path (Sec. 3.3) on the HIP side with the FP64 oracle.

Bars: decoded records bit-exact (both sides form code * gamma + beta and the stage sum of the
colours in float64 in the same order and round once to float32, so the results are the same
numbers); the fused decode-and-render equal bit for bit to rendering the decoded records, and
within 1e-5 A(p) of the oracle's render of the oracle's decode.
"""
import numpy as np
import pytest

import synth
from oracle import codec as ocodec
from oracle import ref

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

FWD_RTOL = 1e-5


def dev(a, dtype=None):
    t = torch.as_tensor(np.ascontiguousarray(a))
    return t.to(device="cuda", dtype=dtype) if dtype is not None else t.to("cuda")


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def to_codec(P, cs, codes=None, index=None):
    return P.Codec(mu=dev(cs.mu_bits.view(np.int16)), codes=dev(cs.codes if codes is None else codes),
                   index=dev(cs.index if index is None else index), codebooks=dev(cs.codebooks),
                   gamma=tuple(float(x) for x in cs.gamma), beta=tuple(float(x) for x in cs.beta),
                   bits=cs.bits)


def oracle_decode(cs, codes=None, index=None):
    return ocodec.decode(cs.mu_bits, cs.codes if codes is None else codes,
                         cs.index if index is None else index, cs.gamma, cs.beta, cs.codebooks,
                         cs.bits)


@pytest.fixture(scope="module")
def gi():
    import paper_2403_08551_amd as P
    ctx = P.Context(0)
    yield ctx
    ctx.close()


@pytest.fixture(params=[1, 2, 3], ids=["radix", "one-pass", "rows"])
def mode(request, gi):
    import paper_2403_08551_amd as P
    gi.set_option(P._lib.GI_OPT_BINNING, request.param)
    yield request.param
    gi.set_option(P._lib.GI_OPT_BINNING, 0)


CASES = {
    # the paper's settings: 6-bit codes, 2 stages of 8 colours
    "paper-200x300": dict(n=3000, h=200, w=300, seed=70),
    "wide-codes-8bit-4x16": dict(n=800, h=64, w=96, seed=71, bits=8, stages=4, book=16),
    "one-bit-1x1": dict(n=300, h=37, w=53, seed=72, bits=1, stages=1, book=1),
    "max-book-256": dict(n=2000, h=128, w=128, seed=73, stages=3, book=256),
}


def make(name):
    c = dict(CASES[name])
    n, h, w, seed = c.pop("n"), c.pop("h"), c.pop("w"), c.pop("seed")
    return synth.codec_set(n, h, w, seed, **c), h, w


@pytest.mark.parametrize("name", list(CASES))
def test_decode_bit_exact(gi, name):
    import paper_2403_08551_amd as P
    cs, h, w = make(name)
    got = host(gi.codec_decode(to_codec(P, cs)))
    want = oracle_decode(cs).astype(np.float32)
    np.testing.assert_array_equal(got, want)


@pytest.mark.parametrize("name", list(CASES))
def test_fused_decode_render_matches_oracle(gi, name, mode):
    import paper_2403_08551_amd as P
    cs, h, w = make(name)
    c = to_codec(P, cs)
    img = host(gi.render_codec(c, h, w))
    np.testing.assert_array_equal(img, host(gi.render(gi.codec_decode(c), h, w)))
    o, A = ref.render_culled(oracle_decode(cs).astype(np.float32), h, w, with_abs=True)
    bad = np.abs(img - o) > FWD_RTOL * A + 1e-30
    assert not bad.any(), (bad.sum(), np.abs(img - o).max())


def test_invalid_codes_take_no_part_and_raise_the_flag(gi):
    import paper_2403_08551_amd as P
    cs, h, w = make("paper-200x300")
    codes, index = cs.codes.copy(), cs.index.copy()
    codes[5, 1] = 64
    index[9, 0] = 8
    c = to_codec(P, cs, codes, index)
    gi.query(clear=True)
    dec = host(gi.codec_decode(c))
    assert np.isnan(dec[[5, 9]]).all() and np.isfinite(np.delete(dec, [5, 9], axis=0)).all()
    _, flags = gi.query(clear=True)
    assert flags & P._lib.GI_FLAG_BAD_CODE
    img = host(gi.render_codec(c, h, w))
    _, flags = gi.query(clear=True)
    assert flags & P._lib.GI_FLAG_BAD_CODE and not flags & P._lib.GI_FLAG_NONFINITE
    o = ref.render_culled(oracle_decode(cs, codes, index).astype(np.float32), h, w)
    _, A = ref.render_culled(oracle_decode(cs, codes, index).astype(np.float32), h, w,
                             with_abs=True)
    assert np.all(np.abs(img - o) <= FWD_RTOL * A + 1e-30)


def test_rotation_scale_codec(gi):
    import paper_2403_08551_amd as P
    cs = synth.codec_set(1500, 150, 170, seed=74, rotation_scale=True)
    ctx = P.Context(0, covariance="rotation_scale")
    try:
        c = to_codec(P, cs)
        img = host(ctx.render_codec(c, 150, 170))
        dec = oracle_decode(cs).astype(np.float32)
        np.testing.assert_array_equal(host(ctx.codec_decode(c)), dec)
        o, A = ref.render_culled(dec, 150, 170, with_abs=True, cov="rs")
        assert np.all(np.abs(img - o) <= FWD_RTOL * A + 1e-30)
    finally:
        ctx.close()


def test_empty_set_and_argument_checks(gi):
    import paper_2403_08551_amd as P
    cs = synth.codec_set(0, 20, 20, seed=75)
    img = host(gi.render_codec(to_codec(P, cs), 20, 20))
    assert img.shape == (20, 20, 3) and not img.any()
    cs, h, w = make("paper-200x300")
    c = to_codec(P, cs)
    for field, value in (("bits", 9), ("bits", 0)):
        bad = P.Codec(**{**c.__dict__, field: value})
        with pytest.raises(P.GiError):
            gi.render_codec(bad, h, w)
    # positions not 4-byte aligned are refused before anything is enqueued
    buf = torch.empty(cs.mu_bits.size + 1, dtype=torch.int16, device="cuda")
    mis = buf[1:].view(-1, 2)
    mis.copy_(c.mu)
    g = P.Codec(**{**c.__dict__, "mu": mis}).c(gi.device)
    import ctypes
    out = torch.empty(h, w, 3, device="cuda")
    rc = P._lib.lib().gi_render_codec(gi._h, ctypes.byref(g), cs.codes.shape[0], h, w,
                                      ctypes.c_void_p(out.data_ptr()), None)
    assert rc == P._lib.GI_ERR_INVALID_ARG


def test_kodak_size_decode_render(gi):
    import paper_2403_08551_amd as P
    cs = synth.codec_set(70_000, 512, 768, seed=76)
    c = to_codec(P, cs)
    dec = host(gi.codec_decode(c))
    np.testing.assert_array_equal(dec, oracle_decode(cs).astype(np.float32))
    img = host(gi.render_codec(c, 512, 768))
    np.testing.assert_array_equal(img, host(gi.render(dev(dec), 512, 768)))
    # sampled pixels against the oracle's per-pixel sum over every Gaussian whose box covers
    # the pixel's tile
    rng = np.random.default_rng(77)
    pix = np.stack([rng.integers(0, 512, 64), rng.integers(0, 768, 64)], axis=1)
    rect, _ = ref.tile_rects(dec, 512, 768)
    pf = dec.astype(np.float64)
    inv = ref.inverse_covariance(dec)
    for y, x in pix:
        ty, tx = y // 16, x // 16
        sel = (rect[:, 0] <= tx) & (tx <= rect[:, 2]) & (rect[:, 1] <= ty) & (ty <= rect[:, 3])
        dx = x + 0.5 - pf[sel, 0]
        dy = y + 0.5 - pf[sel, 1]
        s = 0.5 * (inv[0][sel] * dx * dx + 2 * inv[1][sel] * dx * dy + inv[2][sel] * dy * dy)
        e = np.exp(-s)
        want = (e[:, None] * pf[sel, 5:8]).sum(0)
        A = (e[:, None] * np.abs(pf[sel, 5:8])).sum(0)
        assert np.all(np.abs(img[y, x] - want) <= FWD_RTOL * A + 1e-30), (y, x)
