"""Checkpoint and resume: the library keeps no fitting state of its own (parameters, moments,
the step counter and the quantiser's buffers are the caller's tensors), and its kernels are
deterministic, so a fit whose state is written to disk, read back into fresh tensors and
continued with a new context and a new captured step ends bit for bit where the uninterrupted
fit ends.  Covered: the Adam fit (graph-replayed), the fitting recipe (Adan state) and the
fine-tuning (quantiser, its moments and the moving-average codebook state)."""
import numpy as np
import pytest

import synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def dev(a):
    return torch.as_tensor(np.ascontiguousarray(a)).to(dtype=torch.float32, device="cuda")


def _save(path, tensors):
    torch.save({k: v.detach().cpu().clone() for k, v in tensors.items()}, path)


def _load(path):
    return {k: v.to("cuda") for k, v in torch.load(path, weights_only=True).items()}


def test_adam_fit_resumes_bit_exact(tmp_path):
    import paper_2403_08551_amd as P
    w = synth.kodak_like(10_000)
    T = dev(w.target())
    state = {"params": dev(w.params())}
    state["m"] = torch.zeros_like(state["params"])
    state["v"] = torch.zeros_like(state["params"])
    state["step"] = torch.ones(1, dtype=torch.int32, device="cuda")

    def run(st, steps):
        ctx = P.Context(0)
        g = ctx.fit_graph(st["params"], st["m"], st["v"], T, st["step"])
        try:
            g.launch(steps)
            torch.cuda.synchronize()
            assert g.query()[1] == 0
        finally:
            g.close()
            ctx.close()

    run(state, 20)
    ck = str(tmp_path / "fit.pt")
    _save(ck, state)
    run(state, 20)  # the uninterrupted fit: 40 steps
    resumed = _load(ck)
    run(resumed, 20)
    for k in state:
        assert torch.equal(resumed[k], state[k]), k
    assert int(state["step"].item()) == 41


def test_recipe_fit_resumes_bit_exact(tmp_path):
    import paper_2403_08551_amd as P
    h, w = 128, 160
    rng = np.random.default_rng(11)
    n = 1500
    raw = np.zeros((n, 8), np.float32)
    raw[:, 0:2] = np.arctanh(rng.uniform(-0.95, 0.95, (n, 2)))
    raw[:, 2] = rng.uniform(0.5, 3.0, n)
    raw[:, 3] = rng.normal(0.0, 0.3, n)
    raw[:, 4] = rng.uniform(0.5, 3.0, n)
    raw[:, 5:8] = rng.uniform(0.0, 1.0, (n, 3))
    T = dev(synth.target_noise_rects(h, w, seed=12))
    state = {"raw": dev(raw), "state": torch.zeros(4, n, 8, device="cuda"),
             "step": torch.ones(1, dtype=torch.int32, device="cuda")}

    def run(st, steps):
        ctx = P.Context(0)
        try:
            for _ in range(steps):
                ctx.fit_step_recipe(st["raw"], st["state"], T, st["step"])
            torch.cuda.synchronize()
            assert ctx.query()[1] == 0
        finally:
            ctx.close()

    run(state, 6)
    ck = str(tmp_path / "recipe.pt")
    _save(ck, state)
    run(state, 6)
    resumed = _load(ck)
    run(resumed, 6)
    for k in state:
        assert torch.equal(resumed[k], state[k]), k


def test_fine_tuning_resumes_bit_exact(tmp_path):
    import paper_2403_08551_amd as P
    w = synth.plain_256(1500)
    T = dev(w.target())
    hp = P.AdamConfig()
    ctx0 = P.Context(0)
    q = P.Quantiser.zeros("cuda")
    params = dev(w.params())
    ctx0.qat_init(params, q, 5)
    ctx0.close()
    state = {"params": params, "m": torch.zeros_like(params), "v": torch.zeros_like(params),
             "step": torch.ones(1, dtype=torch.int32, device="cuda"), "quant": q.quant,
             "quant_m": q.quant_m, "quant_v": q.quant_v, "ema": q.ema}

    def run(st, steps):
        qq = P.Quantiser(st["quant"], st["quant_m"], st["quant_v"], st["ema"])
        ctx = P.Context(0)
        g = ctx.fit_graph_qat(st["params"], st["m"], st["v"], T, st["step"], qq, hp)
        try:
            g.launch(steps)
            torch.cuda.synchronize()
            assert g.query()[1] == 0
        finally:
            g.close()
            ctx.close()

    run(state, 5)
    ck = str(tmp_path / "qat.pt")
    _save(ck, state)
    run(state, 5)
    resumed = _load(ck)
    run(resumed, 5)
    for k in state:
        assert torch.equal(resumed[k], state[k]), k
