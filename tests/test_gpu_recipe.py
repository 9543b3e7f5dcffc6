"""Parity of the paper's fitting recipe on the HIP path (App. C parametrisation on raw records,
Adan of Sec. 4.1) with the FP64 oracle: images within 1e-5 A(p), the loss within 1e-5, the raw
records after each step within 1e-4 of a step of the oracle (and never more than four steps
apart where a gradient is too small to fix the direction), as for the Adam fit steps; and the
fused kernel's raw-record gradients element by element, read from Adan's state with all rates
0 (first moment and previous gradient are then the gradient)."""
import numpy as np
import pytest

import parity_util as pu
import synth
from oracle import recipe, ref

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

FWD_RTOL = 1e-5
GRAD_RTOL = 1e-4


def dev(a):
    return torch.as_tensor(np.ascontiguousarray(a)).to(dtype=torch.float32, device="cuda")


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def raw_set(n, seed, cov):
    rng = np.random.default_rng(seed)
    raw = np.zeros((n, 8), np.float32)
    raw[:, 0:2] = np.arctanh(rng.uniform(-0.98, 0.98, (n, 2)))  # App. C initialisation
    raw[:, 2:5] = rng.uniform(0.5, 4.0, (n, 3))
    if cov == "chol":
        raw[:, 3] = rng.uniform(-0.5, 0.5, n)
    else:
        raw[:, 4] = rng.uniform(-3.0, 3.0, n)
    raw[:, 5:8] = rng.uniform(0.0, 0.4, (n, 3))
    return raw


@pytest.mark.parametrize("cov", ["chol", "rs"])
def test_recipe_steps_match_oracle(cov):
    import paper_2403_08551_amd as P
    h, w = 80, 112
    raw0 = raw_set(500, 70 if cov == "chol" else 71, cov)
    T = synth.target_noise_rects(h, w, seed=72)
    hp = dict(recipe.DEFAULT_ADAN, lr=0.01, halve_every=2)
    hp32 = {k: (float(np.float32(v)) if k != "halve_every" else v) for k, v in hp.items()}
    ctx = P.Context(0, covariance="cholesky" if cov == "chol" else "rotation_scale")
    try:
        rd = dev(raw0)
        state = torch.zeros(4, 500, 8, device="cuda")
        step = torch.ones(1, dtype=torch.int32, device="cuda")
        img = torch.empty(h, w, 3, device="cuda")
        loss = torch.empty(1, device="cuda")
        np.testing.assert_array_equal(host(ctx.recipe_params(rd, h, w)),
                                      recipe.effective(raw0, h, w, cov).astype(np.float32))
        st = tuple(np.zeros((500, 8)) for _ in range(4))
        for k in range(1, 5):
            rin = host(rd).copy()
            ctx.fit_step_recipe(rd, state, dev(T), step, P.AdanConfig(**hp), image_out=img,
                                loss_out=loss)
            p = recipe.effective(rin, h, w, cov).astype(np.float32)
            o, A = ref.render_culled(p, h, w, with_abs=True, cov=cov)
            assert np.all(np.abs(host(img) - o) <= FWD_RTOL * A + 1e-30), k
            np.testing.assert_allclose(host(loss)[0], ref.mse(o, T), rtol=1e-5)
            d, Ad = ref.grads(p, h, w, ref.mse_grad(o, T), with_abs=True, cov=cov)
            g = recipe.raw_grads(rin, d, h, w)
            Ag = recipe.raw_grads(rin, Ad, h, w)
            want, *st = recipe.adan_step(rin, *st, g, k, hp32)
            got = host(rd)
            lr = hp32["lr"] * 0.5 ** ((k - 1) // 2)
            firm = np.abs(g) > 10 * GRAD_RTOL * np.abs(Ag) + 1e-20
            tol = 1e-4 * lr + 1e-6 * np.abs(want)
            assert np.all(np.abs(got - want)[firm] <= tol[firm]), (k, np.abs(got - want)[firm].max())
            assert np.all(np.abs(got - want) <= 4.0 * lr + 1e-6 * np.abs(want)), k
            assert firm.mean() > 0.9
        assert int(host(step)[0]) == 5
    finally:
        ctx.close()


@pytest.mark.parametrize("cov", ["chol", "rs"])
def test_recipe_gradients_element_by_element(cov):
    # Adan with all three rates 0 and eps = 1: m = g, n = g^2 and the previous-gradient slot
    # holds g, so the state exposes the fused kernel's gradient of the raw records (through
    # tanh and the +0.5 shifts), compared element by element with the oracle at the gradient
    # bar; the step is lr g / (|g| + 1)
    import paper_2403_08551_amd as P
    h, w = 80, 112
    raw0 = raw_set(500, 75 if cov == "chol" else 76, cov)
    T = synth.target_noise_rects(h, w, seed=77)
    p = recipe.effective(raw0, h, w, cov).astype(np.float32)
    o, A = ref.render_culled(p, h, w, with_abs=True, cov=cov)

    def grads_fn(pp, hh, ww, G, with_abs):
        return ref.grads(pp, hh, ww, G, with_abs=with_abs, cov=cov)

    d, bound = pu.grad_bound(grads_fn, p, h, w, ref.mse_grad(o, T), A)
    g = recipe.raw_grads(raw0, d, h, w)
    gb = recipe.raw_grads(raw0, bound, h, w)
    lr = pu.lr_for(raw0, gb, list(range(8)))
    hp = dict(recipe.DEFAULT_ADAN, lr=lr, beta1=0.0, beta2=0.0, beta3=0.0, eps=1.0,
              weight_decay=0.0, halve_every=0)
    ctx = P.Context(0, covariance="cholesky" if cov == "chol" else "rotation_scale")
    try:
        rd = dev(raw0)
        state = torch.zeros(4, 500, 8, device="cuda")
        step = torch.ones(1, dtype=torch.int32, device="cuda")
        ctx.fit_step_recipe(rd, state, dev(T), step, P.AdanConfig(**hp))
        st = host(state)
        pu.assert_gradient(st[0], g, gb, f"{cov} recipe gradient (first moment)")
        np.testing.assert_array_equal(st[3], st[0])
        pu.assert_linear_step(raw0, host(rd), g, gb, np.full(8, lr), f"{cov} recipe linear step")
    finally:
        ctx.close()


def test_recipe_graph_replay_equals_eager_steps():
    # a captured recipe step replayed (with eager work and synchronisation between replays)
    # gives the eager steps' records and Adan state bit for bit
    import paper_2403_08551_amd as P
    h, w = 80, 112
    raw0 = raw_set(500, 73, "chol")
    T = dev(synth.target_noise_rects(h, w, seed=74))
    hp = P.AdanConfig(**dict(recipe.DEFAULT_ADAN, lr=0.01, halve_every=2))
    ea, gr = P.Context(0), P.Context(0)
    try:
        ra, rb = dev(raw0), dev(raw0)
        sa, sb = torch.zeros(4, 500, 8, device="cuda"), torch.zeros(4, 500, 8, device="cuda")
        ka = torch.ones(1, dtype=torch.int32, device="cuda")
        kb = torch.ones(1, dtype=torch.int32, device="cuda")
        for _ in range(4):
            ea.fit_step_recipe(ra, sa, T, ka, hp)
        graph = gr.fit_graph_recipe(rb, sb, T, kb, hp)
        try:
            for _ in range(2):
                graph.launch(2)
                torch.cuda.synchronize()
                _ = torch.zeros(10, device="cuda").sum().item()
            assert graph.query()[1] == 0
        finally:
            graph.close()
        np.testing.assert_array_equal(host(rb), host(ra))
        np.testing.assert_array_equal(host(sb), host(sa))
        assert int(host(kb)[0]) == 5
    finally:
        ea.close()
        gr.close()
