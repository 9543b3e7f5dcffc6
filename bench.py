#!/usr/bin/env python3
"""Throughput of the accumulated-summation 2-D Gaussian rasteriser on one MI355X.

Workload: one 768x512 RGB image (Kodak's size) with 70 000 Gaussians (Table 1 of the paper uses
560K parameters = 70 000 x 8), synthetic seeded inputs (synth.kodak_like).  A step is one fit
step of the whole path: projection and culling, scan, key duplication, radix sort, tile ranges
and gather, fused forward + L2 loss gradient + adjoint, per-Gaussian gradient reduction with the
Adam update.  Steps are replayed from a captured HIP graph with the inputs resident in HBM.

Prints one JSON line: value = fit iterations per second; also render FPS, the roofline of the
dominant kernel (the fused raster kernel, VALU bound) timed with HIP events on its stream, and
the FP64 CPU oracle timed on a bounded sample on the host.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# Algorithmic work per pixel-Gaussian pair (the unit) of the fused fit kernel, counting each
# pair's own arithmetic and sharing what a pixel column or a Gaussian shares:
#   forward (Eq. rasterization4): u2 (1 FMA), the exponent |u|^2 (1 FMA), exp2, colour (3 FMA)
#   adjoint (App. A): u2, |u|^2, exp2, dL/dc sums (3 FMA), <dL/dC, c'> (a multiply and 2 FMA),
#   its product with exp and u2 (2 multiplies), the sums of w u2 and w u2^2 (an add and an FMA)
# = 16 FP32 VALU operations (30 flops, an FMA counted as two) and 2 exp2 per pair.
VALU_PER_PAIR_FIT = 5 + 11
EXP_PER_PAIR_FIT = 2
FLOPS_PER_PAIR_FIT = 10 + 20
VALU_PER_PAIR_FWD = 5
EXP_PER_PAIR_FWD = 1
FLOPS_PER_PAIR_FWD = 10
# MI355X published dense FP32 vector rate (an FMA as two flops), and the same as FP32 lane
# operations per second from unit counts and clock: 256 CUs x 128 FP32 lanes x 2.4 GHz.
PUBLISHED_FP32_TFLOPS = 157.3
DERIVED_FP32_LANE_OPS = 256 * 128 * 2.4e9


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=500)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", default="kodak", choices=["kodak", "div2k"],
                    help="kodak: 768x512 (the metric's workload); div2k: 2040x1356")
    ap.add_argument("--n", type=int, default=0,
                    help="Gaussians (default 70k for kodak, 100k for div2k)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-steps", type=int, default=0, help="oracle fit steps (0: auto ~15 s)")
    ap.add_argument("--batch-images", type=int, default=64,
                    help="images of the batched-vs-plain comparison (0 skips it)")
    ap.add_argument("--batch-set", default="small", choices=["small", "large"],
                    help="small: sides 128-1024, 1k-50k Gaussians; large: sides 512-2048, "
                         "20k-200k Gaussians")
    ap.add_argument("--batch-steps", type=int, default=1000)
    ap.add_argument("--no-tune", action="store_true", help="skip the autotuner")
    ap.add_argument("--no-codec", action="store_true",
                    help="skip the codec decode leg (Sec. 3.3, Table 2)")
    ap.add_argument("--no-ablation", action="store_true",
                    help="skip the rasterisation ablation leg (Table 3 rows, 768x512 / 30k)")
    ap.add_argument("--no-recipe", action="store_true",
                    help="skip the fitting-recipe and fine-tuning leg (Sec. 4.1, Sec. 3.3)")
    ap.add_argument("--no-rs", action="store_true",
                    help="skip the rotation-scale leg (Sec. 3.1, Eq. RSSR)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only copy 256 MiB device-to-device 10 times (scales rocprof FETCH_SIZE "
                         "and WRITE_SIZE to bytes)")
    ap.add_argument("--binning", type=int, default=0,
                    help="0 auto, 1 duplication + radix sort, 2 one-pass counting sort")
    ap.add_argument("--peaks", action="store_true",
                    help="only run the roofline microbenchmarks and print their rates")
    ap.add_argument("--profile", type=int, default=0, metavar="K",
                    help="only run K eager fit steps with zero learning rates (every step the "
                         "same work: the initial parameters) and K renders of the workload, for "
                         "kernel traces and counters")
    ap.add_argument("--long-steps", type=int, default=1000,
                    help="fit steps of the long-fit leg (keys at step 0 and at its end; 0 skips)")
    return ap.parse_args()


def pairs_from_ranges(ranges, height, width):
    """Exact pixel-Gaussian pair count: tile list lengths times in-image pixels of each tile."""
    import numpy as np
    tw = (width + 15) // 16
    t = np.arange(ranges.shape[0])
    tx, ty = t % tw, t // tw
    pw = np.minimum(16, width - tx * 16)
    ph = np.minimum(16, height - ty * 16)
    return int(((ranges[:, 1] - ranges[:, 0]).astype(np.int64) * pw * ph).sum())


def cpu_baseline(w, steps):
    import numpy as np
    from oracle import cref, ref
    p = w.params()
    T = w.target()
    n = p.shape[0]
    zeros = np.zeros((n, 8))
    hp = dict(ref.DEFAULT_ADAM)
    t0 = time.perf_counter()
    cref.fit_step(p, zeros, zeros, T, 1, hp)  # one step to size the sample
    one = time.perf_counter() - t0
    k = steps if steps > 0 else max(1, min(20, int(15.0 / max(one, 1e-3))))
    t0 = time.perf_counter()
    for i in range(k):
        cref.fit_step(p, zeros, zeros, T, i + 1, hp)
    dt = time.perf_counter() - t0
    return {"value": k / dt, "unit": "it/s", "cores": cref.num_threads(), "kind": "oracle",
            "sample": f"{k} FP64 fit steps (culled render, L2 loss, gradients, Adam) of the "
                      f"same {w.width}x{w.height} / {n} Gaussian workload, after one untimed step"}


def peaks():
    """Roofline denominators measured on this GPU (libgi_peaks.so): the FP32 FMA lane rate of the
    v_fmac_f32 form, the exp2 rate alone and its marginal rate among other VALU work, the device
    copy bandwidth, and the pixel-Gaussian pair rates of the kernels' smallest per-pair
    instruction sequences."""
    import ctypes
    lib = ctypes.CDLL(os.path.join(ROOT, "paper_2403_08551_amd", "libgi_peaks.so"))
    lib.peaks_run.argtypes = [ctypes.c_int, ctypes.c_int64, ctypes.POINTER(ctypes.c_double),
                              ctypes.POINTER(ctypes.c_double)]
    out = {}
    # about 20 ms of FMAs first, so that the clocks have risen before anything is timed
    r, r2 = ctypes.c_double(), ctypes.c_double()
    if lib.peaks_run(0, 20000, ctypes.byref(r), ctypes.byref(r2)) != 0:
        raise RuntimeError("peaks_run warm-up failed")
    for kind, name, size in ((0, "fma", 20000), (1, "exp2", 5000), (2, "exp2_marginal", 4000),
                             (3, "copy", 1 << 30), (4, "fwd_pairs", 4000),
                             (5, "bwd_pairs", 2000)):
        r, r2 = ctypes.c_double(), ctypes.c_double()
        st = lib.peaks_run(kind, size, ctypes.byref(r), ctypes.byref(r2))
        if st != 0 or r.value <= 0:
            raise RuntimeError(f"peaks_run({kind}) failed: {st}")
        out[name] = r.value
        if kind == 2:
            out["add_steps"] = r2.value
    return {"fp32_fma_per_s": out["fma"], "exp2_alone_per_s": out["exp2"],
            "exp2_marginal_per_s": out["exp2_marginal"],
            "exp2_cost_in_fma": out["fma"] / out["exp2_marginal"],
            "fp32_add_per_s": 2.0 * out["add_steps"],
            "copy_bytes_per_s": out["copy"],
            "fwd_pairs_per_s": out["fwd_pairs"], "bwd_pairs_per_s": out["bwd_pairs"],
            "derived_fp32_lane_ops_per_s": DERIVED_FP32_LANE_OPS,
            "fma_frac_of_derived": out["fma"] / DERIVED_FP32_LANE_OPS}


def valu_roofline(pairs, seconds, valu_per_pair, exp_per_pair, flops_per_pair, pk):
    """Roofline object of the ALU-bound raster kernel: pairs x (FP32 VALU operations + exp2)
    per launch over the launch time, against the rate the measured FP32 FMA and (marginal) exp2
    rates give that mix, t = pairs (VALU / R_fma + exp2 / R_exp2); beside it the fraction of the
    pair rate of the kernels' smallest per-pair sequences and the flop rate against the
    published FP32 peak."""
    r_fma, r_exp = pk["fp32_fma_per_s"], pk["exp2_marginal_per_s"]
    t_floor = pairs * (valu_per_pair / r_fma + exp_per_pair / r_exp)
    ops = pairs * (valu_per_pair + exp_per_pair)
    if exp_per_pair == EXP_PER_PAIR_FIT:
        t_pairs = pairs * (1.0 / pk["fwd_pairs_per_s"] + 1.0 / pk["bwd_pairs_per_s"])
    else:
        t_pairs = pairs / pk["fwd_pairs_per_s"]
    tflops = pairs * flops_per_pair / seconds / 1e12
    return {"bound": "alu", "achieved": ops / seconds / 1e12, "peak": ops / t_floor / 1e12,
            "unit": "T op/s (FP32 VALU + exp2)", "frac": t_floor / seconds,
            "valu_per_pair": valu_per_pair, "exp2_per_pair": exp_per_pair,
            "frac_of_pair_sequences": t_pairs / seconds,
            "tflops": tflops, "frac_of_published_fp32": tflops / PUBLISHED_FP32_TFLOPS}


def issued_fraction(executed, pairs, seconds, pk):
    """The executed instructions (SQ counters) priced at the measured rates, over the launch
    time: how close the kernel issues what it runs to the measured peak rates (frac above prices
    the algorithmic count instead, so frac / frac_issued is the share of executed work that is
    algorithmic)."""
    if executed is None:
        return {"frac_issued": None}
    valu, exp2 = executed
    t = pairs * (valu / pk["fp32_fma_per_s"] + exp2 / pk["exp2_marginal_per_s"])
    return {"frac_issued": t / seconds, "executed_valu_per_pair": valu,
            "executed_exp2_per_pair": exp2}


def render_graph_leg(P, torch, params, H, W, renders):
    """Render FPS from a captured graph: 16 no-allocation renders (gi_render_noalloc) recorded
    into one HIP graph on a side stream (a graph launch leaves the device idle for a few
    microseconds at its boundary, so one render per launch would time that gap), replayed;
    the last replay's image equals the eager one."""
    dev = params.device
    tiles = ((H + 15) // 16) * ((W + 15) // 16)
    if tiles > P._lib.GI_NOALLOC_MAX_TILES or params.shape[0] > P._lib.GI_NOALLOC_MAX_GAUSSIANS:
        return None  # beyond the no-allocation render's limits
    per = 16
    img = torch.empty(H, W, 3, device=dev)
    flags = torch.zeros(1, dtype=torch.int32, device=dev)
    P.render_noalloc(params, H, W, img, flags)  # eager: sets up the device's scratch
    torch.cuda.synchronize()
    eager = img.clone()
    g = torch.cuda.CUDAGraph()
    side = torch.cuda.Stream(dev)
    side.wait_stream(torch.cuda.current_stream(dev))
    with torch.cuda.stream(side):
        with torch.cuda.graph(g, stream=side):
            for _ in range(per):
                P.render_noalloc(params, H, W, img, flags)
    torch.cuda.current_stream(dev).wait_stream(side)
    for _ in range(2):
        g.replay()
    torch.cuda.synchronize()
    replays = max(1, renders // per)
    t0 = time.perf_counter()
    for _ in range(replays):
        g.replay()
    torch.cuda.synchronize()
    fps = replays * per / (time.perf_counter() - t0)
    if int(flags.item()) != 0 or not torch.equal(img, eager):
        raise RuntimeError("graph-replayed render differs from the eager one")
    del g
    return fps


def long_fit_leg(P, torch, w, steps):
    """The cfg2 run: `steps` graph-replayed fit steps from the initial parameters; keys, loss
    and pairs at step 0 and at the end, and the it/s over the whole run."""
    dev = torch.device("cuda", 0)
    ctx = P.Context(0)
    params = torch.tensor(w.params(), device=dev)
    target = torch.tensor(w.target(), device=dev)
    b0 = ctx.binning(params, w.height, w.width)
    pairs0 = pairs_from_ranges(b0["ranges"].cpu().numpy(), w.height, w.width)
    m, v = torch.zeros_like(params), torch.zeros_like(params)
    step = torch.ones(1, dtype=torch.int32, device=dev)
    loss = torch.empty(1, device=dev)
    graph = ctx.fit_graph(params, m, v, target, step, loss_out=loss)
    graph.launch(1)
    torch.cuda.synchronize()
    loss0 = float(loss.item())
    t0 = time.perf_counter()
    graph.launch(steps - 1)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    loss_end = float(loss.item())
    _, flags = graph.query(clear=True)
    graph.close()
    if flags & (P._lib.GI_FLAG_KEY_OVERFLOW | P._lib.GI_FLAG_SCAN_STALL):
        raise RuntimeError(f"flags {flags} raised during the long fit")
    b1 = ctx.binning(params, w.height, w.width)
    pairs1 = pairs_from_ranges(b1["ranges"].cpu().numpy(), w.height, w.width)
    ctx.close()
    return {"steps": steps, "fit_its": (steps - 1) / dt, "keys_step0": b0["keys"],
            "keys_end": b1["keys"], "pairs_step0": pairs0, "pairs_end": pairs1,
            "loss_step0": loss0, "loss_end": loss_end}


def profile_run(P, torch, ctx, params0, target, H, W, k):
    """k eager fit steps at zero learning rates (the parameters stay the initial ones, so every
    step does the same work) and k renders; prints the stage times."""
    hp = P.AdamConfig(lr_mu=0.0, lr_l=0.0, lr_c=0.0)
    params = params0.clone()
    m, v = torch.zeros_like(params), torch.zeros_like(params)
    step = torch.ones(1, dtype=torch.int32, device=params.device)
    img = torch.empty(H, W, 3, device=params.device)
    ctx.fit_step(params, m, v, target, step, hp)  # sizes the buffers
    ctx.render(params, H, W, out=img)
    ctx.set_option(P._lib.GI_OPT_SYNC, 0)
    ctx.set_option(P._lib.GI_OPT_TIMING, 1)
    ctx.timing(0, reset=True)
    for _ in range(k):
        ctx.fit_step(params, m, v, target, step, hp)
    for _ in range(k):
        ctx.render(params, H, W, out=img)
    torch.cuda.synchronize()
    out = {name: ctx.timing(st)[0] / max(ctx.timing(st)[1], 1) for name, st in
           (("binning", P._lib.GI_STAGE_BINNING), ("raster_fit", P._lib.GI_STAGE_RASTER_FIT),
            ("update", P._lib.GI_STAGE_UPDATE), ("raster_fwd", P._lib.GI_STAGE_RASTER_FWD))}
    _, flags = ctx.query(clear=True)
    if flags:
        raise RuntimeError(f"flags {flags} raised during the profiled steps")
    if not torch.equal(params, params0):
        raise RuntimeError("zero learning rates changed the parameters")
    print(json.dumps({"profile_steps": k, "stage_ms": out}), flush=True)


def batch_inputs(images, which):
    """Workloads, parameters and targets of the batch (targets made in worker processes; call
    this before the process touches the GPU)."""
    import synth
    ws = synth.batch_small(images) if which == "small" else synth.batch_large(images)
    ps = [w.params() for w in ws]
    ts = synth.targets(ws, processes=min(8, os.cpu_count() or 1))
    return ws, ps, ts


def batched_vs_plain(ctx, inputs, steps, P, torch, np, tune_plain=True):
    """Fit uneven images for `steps` steps as one batch (one launch per stage) and as sequential
    single-image fits, each side with the schedule the autotuner picks for it (the batch's, and
    every image's own, unless tune_plain is off: then the default schedule); both
    graph-replayed after one untimed replay each.  The batched fit is
    bit-identical to the plain one, so every image's final loss is equal."""
    ws, ps, ts = inputs
    images = len(ws)
    dev = ctx.device
    bad = P._lib.GI_FLAG_KEY_OVERFLOW | P._lib.GI_FLAG_SCAN_STALL
    off = np.concatenate([[0], np.cumsum([p.shape[0] for p in ps])])
    batch = P.Batch([w.height for w in ws], [w.width for w in ws], off)
    allp = torch.tensor(np.concatenate(ps), device=dev)
    allt = torch.tensor(np.concatenate([t.reshape(-1, 3) for t in ts]), device=dev)
    m, v = torch.zeros_like(allp), torch.zeros_like(allp)
    step = torch.ones(1, dtype=torch.int32, device=dev)
    loss_b = torch.empty(images, device=dev)
    # the batch's own schedule (its size class); the plain fits keep the default schedule
    tuned = ctx.autotune(allp, allt, batch=batch, reps=3)
    g = ctx.fit_graph(allp, m, v, allt, step, batch=batch, loss_out=loss_b)
    g.launch(1)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    g.launch(steps)
    torch.cuda.synchronize()
    t_batched = time.perf_counter() - t0
    _, flags = g.query(clear=True)
    g.close()
    if flags & bad:
        raise RuntimeError(f"flags {flags} raised during the batched fit")
    # plain: one graph per image, replayed in turn, each image with its own tuned schedule
    singles = []
    plain_tuned = {}
    for w, p, t in zip(ws, ps, ts):
        pd = torch.tensor(p, device=dev)
        td = torch.tensor(t, device=dev)
        md, vd = torch.zeros_like(pd), torch.zeros_like(pd)
        sd = torch.ones(1, dtype=torch.int32, device=dev)
        ld = torch.empty(1, device=dev)
        if tune_plain:
            sc = ctx.autotune(pd, td, reps=2)
            key = f"waves {sc['fit_waves']}, binning {sc['binning']}"
            plain_tuned[key] = plain_tuned.get(key, 0) + 1
        gr = ctx.fit_graph(pd, md, vd, td, sd, loss_out=ld)
        gr.launch(1)
        singles.append((gr, pd, ld))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for gr, _, _ in singles:
        gr.launch(steps)
    torch.cuda.synchronize()
    t_plain = time.perf_counter() - t0
    lb = loss_b.cpu().numpy()
    lp = np.array([float(ld.item()) for _, _, ld in singles])
    same_params = all(torch.equal(allp[off[i]:off[i + 1]], pd) for i, (_, pd, _) in
                      enumerate(singles))
    for gr, _, _ in singles:
        _, f = gr.query(clear=True)
        gr.close()
        if f & bad:
            raise RuntimeError(f"flags {f} raised during a plain fit")
    rel = np.abs(lb - lp) / np.abs(lp)
    return {"images": images, "steps": steps, "gaussians": int(off[-1]),
            "pixels": int(batch.n_pix), "batched_s": t_batched, "plain_s": t_plain,
            "speedup": t_plain / t_batched,
            "batched_image_steps_per_s": images * steps / t_batched,
            "final_mse_max_rel_diff": float(rel.max()), "batch_schedule": tuned,
            "plain_schedules": plain_tuned,
            "images_within_1e-3": int((rel <= 1e-3).sum()),
            "params_bit_identical": bool(same_params)}


TRAFFIC_RECORD = os.path.join(ROOT, "profiles", "traffic-k_raster_fit-kodak-768x512-70k.json")


def raster_fit_digest():
    """sha256 of the source of the fused fit kernel and the device functions it calls (the
    marked region of k_raster.hip)."""
    import hashlib
    src = open(os.path.join(ROOT, "paper_2403_08551_amd", "csrc", "k_raster.hip")).read()
    a = src.index("// ---- begin: the fused fit kernel")
    b = src.index("// ---- end: the fused fit kernel")
    return hashlib.sha256(src[a:b].encode()).hexdigest()


def measured_traffic(kernel, workload):
    """HBM bytes per launch of the fused raster kernel instance `kernel` on `workload` from the
    committed counter record, if it was taken on the current source of the kernel (else None)."""
    try:
        rec = json.load(open(TRAFFIC_RECORD))
    except (OSError, ValueError):
        return None
    if rec.get("kernel") != kernel or rec.get("workload") != workload:
        return None
    return _traffic_if_current(rec)


def _traffic_if_current(rec):
    if rec.get("kernel_source_sha256") != raster_fit_digest():
        return None
    return rec.get("bytes_per_launch")


def executed_per_pair(kernel, workload):
    """(FP32 VALU lane instructions, exp2) per pair that the kernel executed by the SQ counters
    of the committed record (exp2 not among the first), if taken on the current source and the
    same workload (else None)."""
    try:
        rec = json.load(open(TRAFFIC_RECORD))
    except (OSError, ValueError):
        return None
    if (rec.get("kernel") != kernel or rec.get("workload") != workload
            or rec.get("kernel_source_sha256") != raster_fit_digest()
            or "executed_valu_per_pair" not in rec):
        return None
    return rec["executed_valu_per_pair"], rec["executed_exp2_per_pair"]


def copy_calibration():
    import torch
    n = 256 << 20
    a = torch.ones(n // 4, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    for _ in range(10):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_read": n, "copy_bytes_written": n, "copies": 10}), flush=True)


def apply_schedule(P, ctx, sched):
    """Set a tuned schedule's knobs as explicit options of another context."""
    if not sched:
        return
    ctx.set_option(P._lib.GI_OPT_BINNING, sched["binning"])
    ctx.set_option(P._lib.GI_OPT_FWD_PIXELS, sched["fwd_pixels"])
    ctx.set_option(P._lib.GI_OPT_SORT_BITS, sched["sort_bits"])
    ctx.set_option(P._lib.GI_OPT_TILE_ORDER, sched["tile_order"])
    ctx.set_option(P._lib.GI_OPT_FIT_WAVES, sched["fit_waves"])


def rotation_scale_leg(P, torch, w, steps, tuned):
    """Fit it/s (graph replay) and render FPS of the same workload with rotation-scale records
    (s1, s2 with the Cholesky diagonals' distribution, theta uniform)."""
    import synth
    dev = torch.device("cuda", 0)
    ctx = P.Context(0, covariance="rotation_scale")
    apply_schedule(P, ctx, tuned)
    p0 = torch.tensor(synth.gaussians_rs(w.n, w.height, w.width, w.param_seed, s_lo=w.l_lo,
                                         s_hi=w.l_hi, c_lo=0.0, c_hi=1.0), device=dev)
    target = torch.tensor(w.target(), device=dev)
    b = ctx.binning(p0, w.height, w.width)
    pairs = pairs_from_ranges(b["ranges"].cpu().numpy(), w.height, w.width)
    params = p0.clone()
    m, v = torch.zeros_like(params), torch.zeros_like(params)
    step = torch.ones(1, dtype=torch.int32, device=dev)
    graph = ctx.fit_graph(params, m, v, target, step)
    graph.launch(10)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    graph.launch(steps)
    torch.cuda.synchronize()
    its = steps / (time.perf_counter() - t0)
    _, flags = graph.query(clear=True)
    graph.close()
    if flags & (P._lib.GI_FLAG_KEY_OVERFLOW | P._lib.GI_FLAG_SCAN_STALL):
        raise RuntimeError(f"flags {flags} raised during the rotation-scale steps")
    ctx.set_option(P._lib.GI_OPT_SYNC, 0)
    img = torch.empty(w.height, w.width, 3, device=dev)
    for _ in range(10):
        ctx.render(p0, w.height, w.width, out=img)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        ctx.render(p0, w.height, w.width, out=img)
    torch.cuda.synchronize()
    fps = steps / (time.perf_counter() - t0)
    ctx.close()
    return {"fit_its": its, "render_fps": fps, "keys": b["keys"], "pairs": pairs,
            "steps": steps, "paper_context_render_fps_ours_rs": 2321.0}


def codec_leg(P, torch, w, steps):
    """Decode FPS: fused dequantisation + render of a compressed set of the workload's size (the
    paper's codec settings: binary16 positions, 6-bit covariance codes, 2 x 8 RVQ colours)."""
    import numpy as np
    import synth
    dev = torch.device("cuda", 0)
    cs = synth.codec_set(w.n, w.height, w.width, seed=w.param_seed)
    c = P.Codec(mu=torch.tensor(cs.mu_bits.view(np.int16), device=dev),
                codes=torch.tensor(cs.codes, device=dev), index=torch.tensor(cs.index, device=dev),
                codebooks=torch.tensor(cs.codebooks, device=dev),
                gamma=tuple(float(x) for x in cs.gamma), beta=tuple(float(x) for x in cs.beta),
                bits=cs.bits)
    ctx = P.Context(0)
    img = torch.empty(w.height, w.width, 3, device=dev)
    ctx.render_codec(c, w.height, w.width, out=img)  # grows the workspace
    ctx.set_option(P._lib.GI_OPT_SYNC, 0)
    for _ in range(10):
        ctx.render_codec(c, w.height, w.width, out=img)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        ctx.render_codec(c, w.height, w.width, out=img)
    torch.cuda.synchronize()
    fps = steps / (time.perf_counter() - t0)
    _, flags = ctx.query(clear=True)
    ctx.close()
    if flags & (P._lib.GI_FLAG_KEY_OVERFLOW | P._lib.GI_FLAG_SCAN_STALL | P._lib.GI_FLAG_BAD_CODE):
        raise RuntimeError(f"flags {flags} raised during the codec renders")
    bits = 2 * 16 + 3 * cs.bits + cs.index.shape[1] * int(np.log2(cs.codebooks.shape[1]))
    return {"decode_fps": fps, "steps": steps, "bits_per_gaussian": bits,
            "paper_context_decode_fps_v100_div2k": [1970.76, 1980.54]}


def ablation_leg(P, torch, steps):
    """Table 3's speed ablation on this GPU (768x512, 30k Gaussians): fit it/s and render FPS of
    accumulated summation with merged colours, with a separate opacity, and alpha blending.
    Eager non-waiting calls on one context."""
    import numpy as np
    import synth
    dev = torch.device("cuda", 0)
    w = synth.kodak_like(30_000)
    H, W = w.height, w.width
    p0 = torch.tensor(w.params(), device=dev)
    o0 = torch.tensor(np.random.default_rng(7).uniform(0.05, 0.95, w.n).astype(np.float32),
                      device=dev)
    target = torch.tensor(w.target(), device=dev)
    p_rs = torch.tensor(synth.gaussians_rs(w.n, H, W, w.param_seed, s_lo=w.l_lo, s_hi=w.l_hi,
                                           c_lo=0.0, c_hi=1.0), device=dev)
    ctx = P.Context(0)
    ctx_rs = P.Context(0, covariance="rotation_scale")
    out = {}
    for name in ("merged", "sum", "alpha", "rotation_scale"):
        params, opac = (p_rs if name == "rotation_scale" else p0).clone(), o0.clone()
        m, v = torch.zeros_like(params), torch.zeros_like(params)
        mo, vo = torch.zeros_like(opac), torch.zeros_like(opac)
        step = torch.ones(1, dtype=torch.int32, device=dev)
        img = torch.empty(H, W, 3, device=dev)

        c = ctx_rs if name == "rotation_scale" else ctx

        def fit():
            if name in ("merged", "rotation_scale"):
                c.fit_step(params, m, v, target, step)
            else:
                c.fit_step_opacity(params, opac, m, v, mo, vo, target, step, name)

        def render():
            if name == "merged":
                c.render(p0, H, W, out=img)
            elif name == "rotation_scale":
                c.render(p_rs, H, W, out=img)
            else:
                c.render_opacity(p0, o0, H, W, name, out=img)

        c.set_option(P._lib.GI_OPT_SYNC, 1)
        fit()
        render()
        c.set_option(P._lib.GI_OPT_SYNC, 0)
        res = {}
        for label, fn in (("fit_its", fit), ("render_fps", render)):
            for _ in range(5):
                fn()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for _ in range(steps):
                fn()
            torch.cuda.synchronize()
            res[label] = steps / (time.perf_counter() - t0)
        out[name] = res
    flags = ctx.query(clear=True)[1] | ctx_rs.query(clear=True)[1]
    ctx.close()
    ctx_rs.close()
    if flags & (P._lib.GI_FLAG_KEY_OVERFLOW | P._lib.GI_FLAG_SCAN_STALL):
        raise RuntimeError(f"flags {flags} raised during the ablation leg")
    out["workload"] = w.name
    out["steps"] = steps
    # Table 3 (V100, 50k steps): FPS and training seconds per variant
    out["paper_context_table3"] = {"merged": [2565, 91.06], "sum": [2555, 98.54],
                                   "alpha": [2340, 104.76], "rotation_scale": [2321, 98.55]}
    return out


def recipe_leg(P, torch, w, steps):
    """Fit it/s of the paper's recipe (raw records, App. C parametrisation, Adan) and of the
    quantisation-aware fine-tuning (b = 6, M = 2, B = 8) on the workload's size, graph-replayed
    steps (and eager non-waiting steps beside them); also the quantiser set-up and encoding
    times."""
    import numpy as np
    dev = torch.device("cuda", 0)
    H, W = w.height, w.width
    rng = np.random.default_rng(w.param_seed)
    raw = np.zeros((w.n, 8), np.float32)
    raw[:, 0:2] = np.arctanh(rng.uniform(-0.999, 0.999, (w.n, 2)))
    raw[:, 2] = rng.uniform(0.5, 7.5, w.n)
    raw[:, 3] = rng.normal(0.0, 0.5, w.n)
    raw[:, 4] = rng.uniform(0.5, 7.5, w.n)
    raw[:, 5:8] = rng.uniform(0.0, 1.0, (w.n, 3))
    target = torch.tensor(w.target(), device=dev)
    ctx = P.Context(0)
    out = {}
    rd = torch.tensor(raw, device=dev)
    state = torch.zeros(4, w.n, 8, device=dev)
    step = torch.ones(1, dtype=torch.int32, device=dev)
    ctx.fit_step_recipe(rd, state, target, step)
    ctx.set_option(P._lib.GI_OPT_SYNC, 0)
    for _ in range(5):
        ctx.fit_step_recipe(rd, state, target, step)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        ctx.fit_step_recipe(rd, state, target, step)
    torch.cuda.synchronize()
    out["recipe_fit_its_eager"] = steps / (time.perf_counter() - t0)
    g = ctx.fit_graph_recipe(rd, state, target, step)
    g.launch(5)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    g.launch(steps)
    torch.cuda.synchronize()
    out["recipe_fit_its"] = steps / (time.perf_counter() - t0)
    g.close()
    ctx.set_option(P._lib.GI_OPT_SYNC, 1)
    params = ctx.recipe_params(rd, H, W)
    q = P.Quantiser.zeros(dev)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ctx.qat_init(params, q, 5)
    torch.cuda.synchronize()
    out["quantiser_init_ms"] = 1e3 * (time.perf_counter() - t0)
    m, v = torch.zeros_like(params), torch.zeros_like(params)
    step.fill_(1)
    ctx.fit_step_qat(params, m, v, target, step, q)
    ctx.set_option(P._lib.GI_OPT_SYNC, 0)
    for _ in range(5):
        ctx.fit_step_qat(params, m, v, target, step, q)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        ctx.fit_step_qat(params, m, v, target, step, q)
    torch.cuda.synchronize()
    out["qat_fit_its_eager"] = steps / (time.perf_counter() - t0)
    g = ctx.fit_graph_qat(params, m, v, target, step, q)
    g.launch(5)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    g.launch(steps)
    torch.cuda.synchronize()
    out["qat_fit_its"] = steps / (time.perf_counter() - t0)
    g.close()
    t0 = time.perf_counter()
    codec = ctx.qat_encode(params, q)
    torch.cuda.synchronize()
    out["encode_ms"] = 1e3 * (time.perf_counter() - t0)
    _, flags = ctx.query(clear=True)
    ctx.close()
    if flags & (P._lib.GI_FLAG_KEY_OVERFLOW | P._lib.GI_FLAG_SCAN_STALL):
        raise RuntimeError(f"flags {flags} raised during the recipe leg")
    out["steps"] = steps
    out["bits_per_gaussian"] = 2 * 16 + 3 * q.bits + q.stages * int(np.log2(q.size))
    out["paper_context"] = {"training_s_50k_steps_v100_kodak_70k": 106.59}
    del codec
    return out


def main():
    args = parse()
    if args.copy_calibration:
        copy_calibration()
        return
    if args.peaks:
        print(json.dumps(peaks()), flush=True)
        return
    if args.gpus != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path (work shards as "
              "one image, or one batch of images, per GPU)", file=sys.stderr)
        sys.exit(2)
    import numpy as np

    binputs = (batch_inputs(args.batch_images, args.batch_set)
               if args.batch_images > 0 and not args.profile else None)

    import torch

    import paper_2403_08551_amd as P
    import synth

    if args.workload == "kodak":
        w = synth.kodak_like(args.n or 70_000)
    else:
        w = synth.div2k_full(args.n or 100_000)
    n_gauss = w.n
    H, W = w.height, w.width
    dev = torch.device("cuda", 0)
    params0 = torch.tensor(w.params(), device=dev)
    target = torch.tensor(w.target(), device=dev)
    ctx = P.Context(0)
    ctx.set_option(P._lib.GI_OPT_BINNING, args.binning)
    if args.profile > 0:
        profile_run(P, torch, ctx, params0, target, H, W, args.profile)
        ctx.close()
        return
    pk = peaks()

    # exact work of this workload
    b = ctx.binning(params0, H, W)
    ranges = b["ranges"].cpu().numpy()
    P_pairs = pairs_from_ranges(ranges, H, W)
    K = b["keys"]

    # ---- tune the kernel settings for this size class, then capture and replay fit steps
    tuned = ctx.autotune(params0, target, reps=5) if not args.no_tune else None
    px_used = (tuned or {}).get("fwd_pixels") or 4
    waves_used = (tuned or {}).get("fit_waves") or 4
    fit_kernel = f"k_raster_fit<{px_used}, {waves_used}>"
    params = params0.clone()
    m = torch.zeros_like(params)
    v = torch.zeros_like(params)
    step = torch.ones(1, dtype=torch.int32, device=dev)
    loss = torch.empty(1, device=dev)
    graph = ctx.fit_graph(params, m, v, target, step, loss_out=loss)
    graph.launch(args.warmup)
    torch.cuda.synchronize()
    loss_start = float(loss.item())
    # the K timed steps in launches of up to 16 (the library replays runs of 16 steps as one
    # graph launch), each launch bracketed by HIP events on the launch stream so that a one-off
    # cost shows up as an outlier (per-step times of each launch)
    st = torch.cuda.current_stream(dev)
    runs = [16] * (args.steps // 16) + ([args.steps % 16] if args.steps % 16 else [])
    evs = [torch.cuda.Event(enable_timing=True) for _ in range(len(runs) + 1)]
    t0 = time.perf_counter()
    evs[0].record(st)
    for i, k in enumerate(runs):
        graph.launch(k)
        evs[i + 1].record(st)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    rep = np.array([evs[i].elapsed_time(evs[i + 1]) / k for i, k in enumerate(runs)])
    its = args.steps / dt
    loss_end = float(loss.item())
    keys_now, flags = graph.query(clear=True)
    if flags & (P._lib.GI_FLAG_KEY_OVERFLOW | P._lib.GI_FLAG_SCAN_STALL):
        raise RuntimeError(f"flags {flags} raised during the timed steps")
    graph.close()

    # ---- dominant kernel: the fused raster kernel, timed with events on its stream over eager
    # steps without host waits at zero learning rates on the initial parameters (every step the
    # same work, the state `--profile` runs and the committed counters were taken on)
    n_prof = min(max(args.steps, 20), 100)
    hp0 = P.AdamConfig(lr_mu=0.0, lr_l=0.0, lr_c=0.0)
    pz = params0.clone()
    mz, vz = torch.zeros_like(pz), torch.zeros_like(pz)
    sz = torch.ones(1, dtype=torch.int32, device=dev)
    for _ in range(3):  # waiting calls: the key buffers fit this state
        ctx.fit_step(pz, mz, vz, target, sz, hp0)
    torch.cuda.synchronize()
    ctx.query(clear=True)
    ctx.set_option(P._lib.GI_OPT_SYNC, 0)
    ctx.set_option(P._lib.GI_OPT_TIMING, 1)
    ctx.timing(0, reset=True)
    for _ in range(n_prof):
        ctx.fit_step(pz, mz, vz, target, sz, hp0)
    torch.cuda.synchronize()
    fit_ms, fit_n = ctx.timing(P._lib.GI_STAGE_RASTER_FIT)
    bin_ms, bin_n = ctx.timing(P._lib.GI_STAGE_BINNING)
    upd_ms, upd_n = ctx.timing(P._lib.GI_STAGE_UPDATE, reset=True)
    _, flags = ctx.query(clear=True)
    if flags & (P._lib.GI_FLAG_KEY_OVERFLOW | P._lib.GI_FLAG_SCAN_STALL):
        raise RuntimeError(f"flags {flags} raised during the profiled steps")
    if not torch.equal(pz, params0):
        raise RuntimeError("zero learning rates changed the parameters")
    P_prof = P_pairs  # the initial parameters' pairs
    ctx.set_option(P._lib.GI_OPT_SYNC, 0)
    fit_avg_s = fit_ms / fit_n / 1e3
    roof = valu_roofline(P_prof, fit_avg_s, VALU_PER_PAIR_FIT, EXP_PER_PAIR_FIT,
                         FLOPS_PER_PAIR_FIT, pk)

    # ---- render FPS: eager non-waiting renders of the initial parameters, no stage timing
    ctx.set_option(P._lib.GI_OPT_TIMING, 0)
    img = torch.empty(H, W, 3, device=dev)
    for _ in range(10):
        ctx.render(params0, H, W, out=img)
    torch.cuda.synchronize()
    n_render = max(args.steps, 100)
    t0 = time.perf_counter()
    for _ in range(n_render):
        ctx.render(params0, H, W, out=img)
    torch.cuda.synchronize()
    fps = n_render / (time.perf_counter() - t0)
    ctx.set_option(P._lib.GI_OPT_TIMING, 1)
    ctx.timing(0, reset=True)
    for _ in range(100):
        ctx.render(params0, H, W, out=img)
    torch.cuda.synchronize()
    fwd_ms, fwd_n = ctx.timing(P._lib.GI_STAGE_RASTER_FWD)
    rbin_ms, rbin_n = ctx.timing(P._lib.GI_STAGE_BINNING, reset=True)
    ctx.set_option(P._lib.GI_OPT_TIMING, 0)
    fwd_roof = valu_roofline(P_pairs, fwd_ms / fwd_n / 1e3, VALU_PER_PAIR_FWD, EXP_PER_PAIR_FWD,
                             FLOPS_PER_PAIR_FWD, pk)
    fps_graph = render_graph_leg(P, torch, params0, H, W, n_render)
    ctx.set_option(P._lib.GI_OPT_SYNC, 1)
    rs = None if args.no_rs else rotation_scale_leg(P, torch, w, min(max(args.steps, 100), 300),
                                                     tuned)
    cod = None if args.no_codec else codec_leg(P, torch, w, max(args.steps, 100))
    abl = None if args.no_ablation else ablation_leg(P, torch, 100)
    rcp = None if args.no_recipe else recipe_leg(P, torch, w, 100)
    lng = long_fit_leg(P, torch, w, args.long_steps) if args.long_steps > 1 else None
    bvp = None
    if args.batch_images > 0:
        # every plain image tuned for the 64-image set; the 256 large images keep the default
        # schedule (tuning each would take minutes)
        bvp = batched_vs_plain(ctx, binputs, args.batch_steps, P, torch, np,
                               tune_plain=args.batch_set == "small")
    ctx.close()

    out = {
        "metric": "fit iters/s (fwd+bwd) + render FPS, 768x512 @70k Gaussians; batched vs plain",
        "value": its,
        "unit": "it/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * dt / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic (seeded value noise + rectangles target, random Gaussians)",
        "config": {"workload": w.name, "height": H, "width": W, "gaussians": n_gauss,
                   "keys": K, "pairs": P_pairs, "fit_steps": "hip graph replay"},
        "render_fps": fps,
        "render_fps_graph": fps_graph,
        "replay_ms_per_step": {"first": float(rep[0]), "min": float(rep.min()),
                      "median": float(np.median(rep)), "max": float(rep.max())},
        "tuned": tuned,
        "stage_ms": {"binning": bin_ms / max(bin_n, 1), "raster_fit": fit_ms / max(fit_n, 1),
                     "update": upd_ms / max(upd_n, 1),
                     "render_binning": rbin_ms / max(rbin_n, 1),
                     "raster_fwd": fwd_ms / max(fwd_n, 1)},
        "loss": {"after_warmup": loss_start, "after_timed": loss_end},
        "roofline": dict(roof, traffic=measured_traffic(fit_kernel, w.name),
                         **issued_fraction(executed_per_pair(fit_kernel, w.name),
                                           P_prof, fit_ms / fit_n / 1e3, pk),
                         kernel=fit_kernel, pairs_per_launch=P_prof,
                         avg_launch_ms=fit_ms / fit_n),
        "render_roofline": dict(fwd_roof, kernel=f"k_raster_fwd<{px_used}>",
                                pairs_per_launch=P_pairs,
                                avg_launch_ms=fwd_ms / fwd_n),
        "peaks": pk,
        "long_fit": lng,
        "batched_vs_plain": bvp,
        "rotation_scale": rs,
        "codec": cod,
        "ablation": abl,
        "recipe_and_fine_tuning": rcp,
        "paper_context": {"render_fps_v100_kodak_70k": 2092.17,
                          "fit_its_v100_kodak_70k_derived": 50000 / 106.59},
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(w, args.cpu_steps)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
