"""Parity of the quantisation-aware fine-tuning (Sec. 3.3, Sec. 3.4) on the HIP path with the
FP64 oracle: quantiser initialisation (gamma, beta exactly; codebooks from K-means on separated
colour clusters within float64 rounding; the moving average's running counts exactly and its
sums within float32 rounding), fine-tuning steps (images within 1e-5 A(p), the loss within 1e-5,
records as for the Adam fit steps, gamma and beta within a step's bound; the codebooks' moving
average from the same state within float32 rounding, counts exactly), the fused kernel's
gradients element by element through the first Adam moment at beta1 = 0 (records, gamma,
beta), and the encoding (codes and indices bit-exact against the oracle's fake quantiser;
rendering the encoded set with the codec equals rendering the fake-quantised records)."""
import numpy as np
import pytest

import parity_util as pu
import synth
from oracle import qat, ref

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

def dev(a):
    return torch.as_tensor(np.ascontiguousarray(a)).to(dtype=torch.float32, device="cuda")


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def clustered(n, h, w, seed):
    """Records whose colours form 8 separated clusters laid out so that the K-means seeds
    floor(j n / 8) fall one per cluster (the stage-1 codebook is then the cluster means)."""
    p = synth.gaussians(n, h, w, seed=seed, l_lo=0.8, l_hi=6.0)
    rng = np.random.default_rng(seed + 1)
    centres = rng.uniform(0.05, 0.95, (8, 3))
    lab = (np.arange(n) * 8) // n
    p[:, 5:8] = centres[lab] + rng.uniform(-0.01, 0.01, (n, 3))
    return p


@pytest.fixture(scope="module")
def gi():
    import paper_2403_08551_amd as P
    ctx = P.Context(0)
    yield ctx
    ctx.close()


def test_init_matches_oracle(gi):
    import paper_2403_08551_amd as P
    p = clustered(4000, 128, 160, 80)
    qz = P.Quantiser.zeros("cuda")
    gi.qat_init(dev(p), qz, 5)
    g, b = qat.lsq_init(p, 6)
    np.testing.assert_array_equal(host(qz.gamma), g.astype(np.float32))
    np.testing.assert_array_equal(host(qz.beta), b.astype(np.float32))
    books, ema = qat.rvq_init(p, 2, 8, 5)
    np.testing.assert_allclose(host(qz.codebooks), books.astype(np.float32), rtol=1e-6,
                               atol=1e-7)
    got = host(qz.ema)
    np.testing.assert_array_equal(got[..., 0], ema[..., 0])
    np.testing.assert_allclose(got[..., 1:], ema[..., 1:], rtol=1e-6, atol=1e-7)
    assert got[0, :, 0].sum() == 4000 and got[1, :, 0].sum() == 4000


def _check_codebooks(qz, books_in, ema_in, idx, resids, decay, what):
    # the moving average from the step's own start state: counts exactly, sums and entries
    # within float32 rounding (the float64 residual sums are added in another order)
    want_b, want_e = qat.ema_update(books_in, ema_in, idx, resids, decay)
    got_e = host(qz.ema)
    np.testing.assert_array_equal(got_e[..., 0], want_e[..., 0], err_msg=what)
    np.testing.assert_allclose(got_e[..., 1:], want_e[..., 1:], rtol=2.5e-7, atol=1e-12,
                               err_msg=what)
    np.testing.assert_allclose(host(qz.codebooks), want_b, rtol=2.5e-7, atol=1e-12,
                               err_msg=what)
    # and the entries moved: the test would see a codebook left alone
    assert np.abs(want_b - np.asarray(books_in, np.float64)).max() > 1e-6


def test_fine_tuning_steps_match_oracle(gi):
    import paper_2403_08551_amd as P
    h, w = 96, 112
    p0 = clustered(900, h, w, 81)
    T = synth.target_noise_rects(h, w, seed=82)
    qz = P.Quantiser.zeros("cuda", lam=1.0, lr_q=1e-3, decay=0.9)
    pd = dev(p0)
    gi.qat_init(pd, qz, 5)
    hp = dict(ref.DEFAULT_ADAM)
    hp32 = {k: float(np.float32(v)) for k, v in hp.items()}
    lr = np.array([hp32["lr_mu"]] * 2 + [hp32["lr_l"]] * 3 + [hp32["lr_c"]] * 3)
    lr_q = float(np.float32(1e-3))
    md, vd = torch.zeros_like(pd), torch.zeros_like(pd)
    step = torch.ones(1, dtype=torch.int32, device="cuda")
    img = torch.empty(h, w, 3, device="cuda")
    loss = torch.empty(1, device="cuda")
    Mo, Vo = np.zeros((900, 8)), np.zeros((900, 8))
    for t in range(1, 4):
        pin = host(pd).copy()
        quant = host(qz.quant).copy()
        qm, qv = host(qz.quant_m).copy(), host(qz.quant_v).copy()
        ema_in = host(qz.ema).copy()
        gi.fit_step_qat(pd, md, vd, dev(T), step, qz, P.AdamConfig(**hp), image_out=img,
                        loss_out=loss)
        g, b, books = quant[0:3], quant[3:6], quant[6:].reshape(2, 8, 3)
        dp, dg, db, want_loss, want_img, idx, resids = qat.qat_grads(pin, g, b, books, 6, h, w, T)
        q, *_ = qat.fake_quant(pin, g, b, books, 6)
        _, A = ref.render_culled(q.astype(np.float32), h, w, with_abs=True)
        assert np.all(np.abs(host(img) - want_img) <= pu.FWD_RTOL * A + 1e-30), t
        np.testing.assert_allclose(host(loss)[0], want_loss, rtol=1e-5)
        out = qat.qat_step(pin, Mo, Vo, (g, b, books), qm, qv, ema_in, T, t, h, w, 6, hp32,
                           lr_q=lr_q, lam=1.0, decay=float(np.float32(0.9)))
        po, Mo, Vo = out[0], out[1], out[2]
        got = host(pd)
        _, Ad = ref.grads(q.astype(np.float32), h, w, ref.mse_grad(want_img, T), with_abs=True)
        firm = np.abs(dp) > 10 * pu.GRAD_RTOL * Ad + 1e-20
        tol = 1e-4 * lr + 1e-6 * np.abs(po)
        assert np.all(np.abs(got - po)[firm] <= np.broadcast_to(tol, po.shape)[firm]), t
        assert np.all(np.abs(got - po) <= 2.0 * lr + 1e-6 * np.abs(po))
        assert firm.mean() > 0.8
        # gamma and beta: one Adam step of at most lr_q each, in the oracle's direction where
        # the gradient is well above the float32 noise of the sums (their gradients are
        # compared element by element in the next test)
        want_q = np.concatenate([out[3][0], out[3][1]])
        got_q = host(qz.quant)[0:6]
        assert np.all(np.abs(got_q - want_q) <= 2 * lr_q + 1e-6 * np.abs(want_q)), t
        gflat = np.concatenate([dg, db])
        strong = np.abs(gflat) > 1e-3 * np.abs(gflat).max()
        assert np.all(np.abs(got_q - want_q)[strong] <= 1e-4 * lr_q + 1e-6 * np.abs(want_q)[strong]), t
        _check_codebooks(qz, books, ema_in, idx, resids, float(np.float32(0.9)), f"step {t}")
    assert int(host(step)[0]) == 4


@pytest.mark.parametrize("stages,size", [(1, 64), (8, 8), (4, 4)])
def test_fine_tuning_codebook_shapes(gi, stages, size):
    """Codebook shapes away from the paper's 2 x 8: the most entries (64, one stage), the most
    stages (8), and a small square case.  Two steps: the fake-quantised image within the
    forward bar, and the moving average of every entry against the oracle's from the same
    state (the search, the per-entry sums and the quantiser update at these sizes)."""
    import paper_2403_08551_amd as P
    h, w = 96, 112
    p0 = clustered(900, h, w, 83 + stages)
    T = synth.target_noise_rects(h, w, seed=84)
    qz = P.Quantiser.zeros("cuda", stages=stages, size=size, lam=1.0, lr_q=1e-3, decay=0.9)
    pd = dev(p0)
    gi.qat_init(pd, qz, 5)
    hp = dict(ref.DEFAULT_ADAM)
    md, vd = torch.zeros_like(pd), torch.zeros_like(pd)
    step = torch.ones(1, dtype=torch.int32, device="cuda")
    img = torch.empty(h, w, 3, device="cuda")
    for t in range(1, 3):
        pin = host(pd).copy()
        quant = host(qz.quant).copy()
        ema_in = host(qz.ema).copy()
        gi.fit_step_qat(pd, md, vd, dev(T), step, qz, P.AdamConfig(**hp), image_out=img)
        g, b, books = quant[0:3], quant[3:6], quant[6:].reshape(stages, size, 3)
        _, _, _, _, want_img, idx, resids = qat.qat_grads(pin, g, b, books, 6, h, w, T)
        q, *_ = qat.fake_quant(pin, g, b, books, 6)
        _, A = ref.render_culled(q.astype(np.float32), h, w, with_abs=True)
        assert np.all(np.abs(host(img) - want_img) <= pu.FWD_RTOL * A + 1e-30), t
        assert idx.shape[1] == stages and idx.max() < size
        _check_codebooks(qz, books, ema_in, idx, resids, float(np.float32(0.9)),
                         f"{stages} x {size}, step {t}")
    _, flags = gi.query(clear=True)
    assert flags == 0


def test_fine_tuning_gradients_element_by_element(gi):
    # beta1 = beta2 = 0, eps = 1: the first moments are the gradients of the records (through
    # the straight-through estimates) and of gamma and beta (LSQ+), compared with the oracle at
    # the gradient bar; the records' step is lr g / (|g| + 1).  Gamma and beta are set so that
    # codes fall below, inside and above the range
    import paper_2403_08551_amd as P
    h, w = 96, 112
    p0 = clustered(900, h, w, 85)
    T = synth.target_noise_rects(h, w, seed=86)
    qz = P.Quantiser.zeros("cuda", lam=1.0, lr_q=1.0, decay=0.99)
    pd = dev(p0)
    gi.qat_init(pd, qz, 5)
    qz.quant[0:3] *= 0.6            # a narrower code range: the extremes now clamp
    qz.quant[3:6] += 0.2 * qz.quant[0:3] * 63
    quant = host(qz.quant).copy()
    g, b, books = quant[0:3], quant[3:6], quant[6:].reshape(2, 8, 3)
    q, x, code, idx, resids = qat.fake_quant(p0, g, b, books, 6)
    assert (x < 0).any() and (x > 63).any()
    dp, dg, db, _, want_img, _, _ = qat.qat_grads(p0, g, b, books, 6, h, w, T)
    _, A = ref.render_culled(q.astype(np.float32), h, w, with_abs=True)
    q32 = q.astype(np.float32)
    up, bound = pu.grad_bound(ref.grads, q32, h, w, ref.mse_grad(want_img, T), A)
    inside = (x >= 0) & (x <= 63)
    bound_p = bound.copy()
    bound_p[:, 2:5] = np.where(inside, bound[:, 2:5], 1e-30)
    wgt = np.where(inside, np.abs(code - x), np.where(x > 63, 63.0, 0.0))
    bound_g = (bound[:, 2:5] * wgt).sum(0) + 1e-5 * np.abs(up[:, 2:5] * wgt).sum(0) + 1e-30
    bound_b = (bound[:, 2:5] * ~inside).sum(0) + 1e-5 * np.abs(up[:, 2:5] * ~inside).sum(0) + 1e-30
    hp = pu.linear_hp(pu.lr_for(p0, bound_p, [0, 1]), pu.lr_for(p0, bound_p, [2, 3, 4]),
                      pu.lr_for(p0, bound_p, [5, 6, 7]))
    md, vd = torch.zeros_like(pd), torch.zeros_like(pd)
    step = torch.ones(1, dtype=torch.int32, device="cuda")
    ema_in = host(qz.ema).copy()
    gi.fit_step_qat(pd, md, vd, dev(T), step, qz, P.AdamConfig(**hp))
    pu.assert_gradient(host(md), dp, bound_p, "record gradients")
    pu.assert_gradient(host(qz.quant_m)[0:3], dg, bound_g, "dL/dgamma")
    pu.assert_gradient(host(qz.quant_m)[3:6], db, bound_b, "dL/dbeta")
    lr = np.array([hp["lr_mu"]] * 2 + [hp["lr_l"]] * 3 + [hp["lr_c"]] * 3)
    pu.assert_linear_step(p0, host(pd), dp, bound_p, lr, "records after the linear step")
    want_q = np.concatenate([g, b]) - np.concatenate([dg, db]) / (np.abs(np.concatenate([dg, db])) + 1)
    tol_q = np.concatenate([bound_g, bound_b]) + 2.0 ** -21 * (np.abs(want_q) + 1)
    assert np.all(np.abs(host(qz.quant)[0:6] - want_q) <= tol_q)
    _check_codebooks(qz, books, ema_in, idx, resids, float(np.float32(0.99)), "linear step")


def test_encode_matches_oracle_and_renders_the_fine_tuned_image(gi):
    import paper_2403_08551_amd as P
    h, w = 80, 90
    p = clustered(1200, h, w, 83)
    qz = P.Quantiser.zeros("cuda")
    pd = dev(p)
    gi.qat_init(pd, qz, 5)
    codec = gi.qat_encode(pd, qz)
    quant = host(qz.quant)
    q, x, code, idx, _ = qat.fake_quant(p, quant[0:3], quant[3:6], quant[6:].reshape(2, 8, 3), 6)
    np.testing.assert_array_equal(host(codec.codes), code.astype(np.uint8))
    np.testing.assert_array_equal(host(codec.index), idx.astype(np.uint8))
    np.testing.assert_array_equal(host(codec.mu).view(np.float16).astype(np.float64), q[:, :2])
    # decoding the encoded set gives the fake-quantised records bit for bit
    np.testing.assert_array_equal(host(gi.codec_decode(codec)), q.astype(np.float32))
    np.testing.assert_array_equal(host(gi.render_codec(codec, h, w)),
                                  host(gi.render(dev(q.astype(np.float32)), h, w)))


def test_argument_checks(gi):
    import paper_2403_08551_amd as P
    p = dev(clustered(100, 32, 32, 84))
    with pytest.raises(P.GiError):
        gi.qat_init(p, P.Quantiser.zeros("cuda", stages=3, size=32))  # 96 entries > 64
    with pytest.raises(P.GiError):
        gi.qat_init(p, P.Quantiser.zeros("cuda", bits=9))


def test_fine_tuning_graph_replay_equals_eager_steps(gi):
    # a captured fine-tuning step replayed gives the eager steps' records, moments and
    # quantiser state bit for bit
    import paper_2403_08551_amd as P
    h, w = 96, 112
    p0 = clustered(900, h, w, 83)
    T = dev(synth.target_noise_rects(h, w, seed=84))
    hp = P.AdamConfig(**dict(ref.DEFAULT_ADAM))
    out = []
    for use_graph in (False, True):
        qz = P.Quantiser.zeros("cuda", lam=1.0, lr_q=1e-3)
        pd = dev(p0)
        gi.qat_init(pd, qz, 5)
        md, vd = torch.zeros_like(pd), torch.zeros_like(pd)
        step = torch.ones(1, dtype=torch.int32, device="cuda")
        if use_graph:
            graph = gi.fit_graph_qat(pd, md, vd, T, step, qz, hp)
            try:
                for _ in range(2):
                    graph.launch(2)
                    torch.cuda.synchronize()
                    _ = torch.zeros(10, device="cuda").sum().item()
                assert graph.query()[1] == 0
            finally:
                graph.close()
        else:
            for _ in range(4):
                gi.fit_step_qat(pd, md, vd, T, step, qz, hp)
        out.append([host(t).copy() for t in (pd, md, vd, qz.quant, qz.quant_m, qz.quant_v,
                                              step)])
    for a, b in zip(*out):
        np.testing.assert_array_equal(a, b)
