#!/usr/bin/env python3
"""Throughput benchmark of the hot path on one MI355X.

Workload (default): the fetal-scale head phantom -- 500,000 Gaussians, four
stacks (axial, coronal, sagittal, oblique) of 32 slices of 256x256 pixels at
0.8 x 0.8 x 3.5 mm, PSF FWHM (0.8, 0.8, 3.5) mm, per-slice motion ~N(0, 4 deg),
~N(0, 2 mm).  Observations are the library's own forward of the ground-truth
Gaussians at the true poses plus Rician noise at SNR 20 (synthetic data; no
dataset).  One step = svr_project_bin + svr_forward (masked MSE) +
svr_backward + svr_step (AdamW) from identity pose initialisation, i.e. one
full fitting iteration; inputs are resident in HBM before timing starts.

value = Gaussian-pixel pairs inside the 3-sigma footprint per step (counted
by the forward kernel) / seconds per step.

Prints ONE JSON line.  --gpus N with N > 1 exits: the hot path runs on one GPU.
"""
from __future__ import annotations

import argparse
import glob
import hashlib
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "Gaussian-pixel pair evals/s fwd+bwd; s to PSNR target learned vs plain"
PEAK_FP32 = 157.3e12      # MI355X FP32 vector, FLOP/s
PEAK_HBM = 8.0e12         # MI355X HBM3E, B/s
LR = [2.5e-2, 2.5e-2, 1e-2, 1e-2, 2.5e-3, 1e-1]   # mean, scale, quat, amp, rotation, translation

# Algorithmic work per unit: FLOP count a multiply-add as 2 and an exp2 as 1.
FLOP_FWD_PAIR = 13.0      # 12 FLOP + 1 exp per in-cut pixel-Gaussian pair
FLOP_BWD_PAIR = 32.0      # 31 FLOP + 1 exp per in-cut pair (recomputation included)
FLOP_CULL_CAND = 25.0     # plane test per (slice, Gaussian) candidate
FLOP_CULL_REC = 150.0     # projection per kept record
FLOP_PROJ_BWD_REC = 400.0
BYTES_SORT_INST_PASS = 20.0   # upsweep key read 4 + downsweep key/value read 8 + write 8
# adjoint tile kernel, per instance: key, record id and emission slot read (12),
# record payload read (28: centre, beta', amplitude, conic), seven sums
# written (28); per slice pixel: its upstream gradient read once (4)
BYTES_BWD_INST = 68.0
BYTES_BWD_PIXEL = 4.0
BYTES_EMIT = (32.0, 8.0)      # per record, per instance
# Normalised Top-K model (Eqs. 2 and 5), per (pixel, neighbour) pair: forward
# 57 FLOP + 1 exp (Sigma_obs, cofactor inverse, quadratic form, sums); adjoint
# 77 (pixel pass: recompute + pose terms) + 82 (Gaussian pass: recompute +
# parameter terms) FLOP + 2 exp.
FLOP_TOPK_FWD_PAIR = 58.0
FLOP_TOPK_BWD_PAIR = 161.0


# kernel source of each timed stage: a committed counter record is used only
# while these files are unchanged
STAGE_SOURCES = {"forward_tile": "render.hip", "backward_tile": "render.hip", "sort": "sort.hip",
                 "emit": "project.hip", "cull_count": "project.hip", "project_backward": "project.hip"}


# what the fitted observations are, per workload (the product benchmark may
# not run the CPU oracle, so the ground truth is rendered by the library)
OBSERVATIONS = {
    "head": "library forward (3-sigma window) of the ground-truth Gaussians at the true poses + Rician noise, SNR 20",
    "head-stress": "library forward (3-sigma window) of the ground-truth Gaussians at the true poses + Rician noise, "
                   "SNR 20",
    "batched": "library forward (3-sigma window) of the ground-truth Gaussians at the true poses + Rician noise, SNR 20",
    "cube": "library forward (3-sigma window) of the ground-truth Gaussians at the true poses + Rician noise, SNR 20",
}


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def source_digest(stage):
    h = hashlib.sha256()
    for f in (STAGE_SOURCES[stage], "svr_internal.h"):
        with open(os.path.join(ROOT, "paper_2512_11624_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(stage, tile, workload):
    """HBM bytes per launch of the stage's kernel, from the rocprofv3
    FETCH_SIZE / WRITE_SIZE summaries committed under profiles/ (lines
    "traffic-record: key=value ..."), or None when no record matches this
    stage, tile and workload or the kernel source changed since it was taken."""
    if stage not in STAGE_SOURCES:
        return None
    digest = source_digest(stage)
    for fn in sorted(glob.glob(os.path.join(ROOT, "profiles", "*.txt"))):
        with open(fn) as fh:
            for line in fh:
                if not line.startswith("traffic-record:"):
                    continue
                kv = dict(t.split("=", 1) for t in line.split()[1:] if "=" in t)
                if (kv.get("stage") == stage and kv.get("tile") == str(tile) and kv.get("workload") == workload
                        and kv.get("source") == digest):
                    return float(kv["bytes_per_launch"])
    return None


def make_workload(name, seed=0):
    from paper_2512_11624_amd import synth
    if name == "head":
        prob = synth.config2(seed)
        desc = ("head phantom, 500k Gaussians, 4 stacks x 32 slices of 256x256 px at 0.8x0.8x3.5 mm, "
                "motion N(0,4deg)/N(0,2mm), Rician SNR 20")
    elif name == "head-stress":
        prob = synth.config3(seed)
        desc = "head phantom, 1.2M Gaussians, 6 stacks x 40 slices of 320x320 px at 0.7x0.7x3 mm"
    elif name == "batched":
        prob = synth.config4(seed)
        desc = ("16 cube subjects, Gaussians log-uniform 1.5e5-1.5e6 (8.2M total), 3-9 stacks of 20-48 slices, "
                "192-320 px, thickness 2.5-4.5 mm, all subjects in one launch per stage")
    elif name == "cube":
        prob = synth.config1(seed)
        desc = "cube phantom, 2,000 Gaussians, 3 stacks x 16 slices of 32x32 px at 1x1x3 mm"
    else:
        raise SystemExit(f"unknown workload {name}")
    return prob, desc


def stage_roofline(stage, ms, st, n_incut):
    """(bound, achieved, peak, unit, algorithmic amount per launch) of one stage."""
    sec = ms / 1e3
    if stage == "forward_tile":
        w = FLOP_FWD_PAIR * n_incut
        return "alu", w / sec / 1e12, PEAK_FP32 / 1e12, "TFLOP/s", w
    if stage == "backward_tile":
        # bound by its memory accesses, not by its arithmetic: with the pixel
        # walk (all of its FP32 work) removed the kernel keeps 91 % of its
        # time on the head workload; the FP32 figure is stage_alu's
        w = BYTES_BWD_INST * st["n_instances"] + BYTES_BWD_PIXEL * st["n_pixels"]
        return "hbm", w / sec / 1e9, PEAK_HBM / 1e9, "GB/s", w
    if stage == "cull_count":
        w = FLOP_CULL_CAND * st["n_candidates"] + FLOP_CULL_REC * st["n_records"]
        return "alu", w / sec / 1e12, PEAK_FP32 / 1e12, "TFLOP/s", w
    if stage == "project_backward":
        w = FLOP_PROJ_BWD_REC * st["n_records"]
        return "alu", w / sec / 1e12, PEAK_FP32 / 1e12, "TFLOP/s", w
    if stage == "sort":
        w = BYTES_SORT_INST_PASS * st["n_instances"] * st["sort_passes"]
        return "hbm", w / sec / 1e9, PEAK_HBM / 1e9, "GB/s", w
    if stage == "emit":
        w = BYTES_EMIT[0] * st["n_records"] + BYTES_EMIT[1] * st["n_instances"]
        return "hbm", w / sec / 1e9, PEAK_HBM / 1e9, "GB/s", w
    if stage == "topk_forward":
        w = FLOP_TOPK_FWD_PAIR * n_incut
        return "alu", w / sec / 1e12, PEAK_FP32 / 1e12, "TFLOP/s", w
    if stage == "topk_backward":
        w = FLOP_TOPK_BWD_PAIR * n_incut
        return "alu", w / sec / 1e12, PEAK_FP32 / 1e12, "TFLOP/s", w
    return None


def stage_alu(stage, ms, n_incut):
    """FP32 rate of a tile kernel's algorithmic arithmetic (TFLOP/s, fraction
    of the FP32 vector peak), whatever bounds it; None for other stages."""
    per = {"forward_tile": FLOP_FWD_PAIR, "backward_tile": FLOP_BWD_PAIR}.get(stage)
    if per is None:
        return None
    achieved = per * n_incut / (ms / 1e3) / 1e12
    return dict(achieved=round(achieved, 4), peak=PEAK_FP32 / 1e12, unit="TFLOP/s",
                frac=round(achieved / (PEAK_FP32 / 1e12), 6), work_per_launch=per * n_incut)


def cpu_baseline(prob, params, pose, target, budget_s=15.0):
    """The FP64 oracle, as it stands, on a bounded sample of the same workload:
    every Gaussian against a subset of slices spread over the stacks."""
    import oracle
    from paper_2512_11624_amd import synth
    oracle.build(force=False)

    def run(sel):
        po = prob.pix_offset
        pix = np.concatenate([np.arange(po[i], po[i + 1]) for i in sel])
        sub = synth.Problem(prob.mean, prob.log_scale, prob.quat, prob.amp, prob.gauss_offsets,
                            prob.slice_subject[sel], prob.height[sel], prob.width[sel], prob.spacing[sel],
                            prob.psf_fwhm[sel], prob.rot0[sel], prob.trans0[sel], prob.pose[sel], prob.mask[pix])
        t0 = time.perf_counter()
        y, n_in, _ = oracle.forward(sub, 3.0, params=params, pose=pose[sel], counts=True)
        _, g, _ = oracle.masked_mse(y, target[pix], sub.mask, sub.pix_offset)
        oracle.backward(sub, g, 3.0, params=params, pose=pose[sel])
        return time.perf_counter() - t0, n_in

    M = prob.n_slices
    k = min(4, M)
    sel = np.linspace(0, M - 1, k).round().astype(int)
    dt, n_in = run(sel)
    if dt < budget_s / 3 and k < M:
        k = int(min(M, max(k + 1, k * budget_s / max(dt, 1e-3))))
        sel = np.unique(np.linspace(0, M - 1, k).round().astype(int))
        dt, n_in = run(sel)
    return dict(value=n_in / dt, unit="pair-evals/s", cores=oracle.num_threads(), kind="oracle",
                sample=f"FP64 oracle fwd+masked-MSE+bwd, all {prob.n_gauss} Gaussians x {len(sel)} of {M} "
                       f"slices ({n_in} in-cut pairs, {dt:.1f} s)")


def sequential_subjects(prob, par, target, mask, cfg, steps, warmup):
    """The same iteration run subject by subject (one context per subject, the
    configuration tuned for the batch), as 16 independent reconstructions
    would: returns the time of one round over all subjects."""
    import torch
    from paper_2512_11624_amd import svr, synth
    N0 = par.N
    po = prob.pix_offset
    runs = []
    for k in range(prob.n_subjects):
        sub = synth.subject(prob, k)
        g0, g1 = int(prob.gauss_offsets[k]), int(prob.gauss_offsets[k + 1])
        sl = np.nonzero(prob.slice_subject == k)[0]
        p0, p1 = int(po[sl[0]]), int(po[sl[-1] + 1])
        c = svr.Context(0)
        c.svr_set_config(**cfg)
        c.svr_set_geometry(sub)
        v = par.views()
        sp = svr.Params.from_arrays(v[0][g0:g1].cpu().numpy(), v[1][g0:g1].cpu().numpy(),
                                    v[2][g0:g1].cpu().numpy(), v[3][g0:g1].cpu().numpy(),
                                    v[4][sl[0]:sl[-1] + 1].cpu().numpy())
        P = p1 - p0
        runs.append(dict(ctx=c, par=sp, grad=svr.Params(sp.N, sp.M), m=torch.zeros_like(sp.flat),
                         v=torch.zeros_like(sp.flat), t=target[p0:p1], mk=mask[p0:p1],
                         pred=torch.empty(P, device="cuda"), g=torch.empty(P, device="cuda"),
                         loss=torch.empty(1, device="cuda"), it=0))

    def one_round():
        for r in runs:
            r["it"] += 1
            c = r["ctx"]
            c.svr_project_bin(*r["par"].views())
            c.svr_forward(r["pred"], r["t"], r["mk"], loss=r["loss"], grad_pred=r["g"])
            c.svr_backward(r["g"], *r["grad"].views())
            c.svr_step(r["par"].views(), r["grad"].views(), r["m"], r["v"], LR, r["it"])

    for _ in range(warmup):
        one_round()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        one_round()
    torch.cuda.synchronize()
    ms = (time.perf_counter() - t0) * 1e3 / steps
    for r in runs:
        r["ctx"].close()
    return dict(ms_per_round=ms, subjects=len(runs))


def stage_breakdown(ctx, run, n):
    """Per-stage GPU times over `run` called n times, with every stage
    bracketed by HIP events.  Event records leave the GPU idle for a few
    microseconds between kernels, so this runs outside the timed region."""
    ctx.svr_set_timing_stages(None)
    ctx.svr_set_timing(True)
    for _ in range(n):
        run()
    t = ctx.svr_get_timing()
    ctx.svr_set_timing(False)
    return {k: dict(calls=c, avg_ms=(tt / c if c else 0.0)) for k, (c, tt) in t.items() if c}


def build_parser():
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="head", choices=["head", "head-stress", "cube", "batched"])
    # tile 32 measured fastest on the head workload (fewer instances: a
    # cheaper sort and adjoint, against a slower forward)
    ap.add_argument("--tile", type=int, default=32)
    ap.add_argument("--batch", type=int, default=128)
    ap.add_argument("--persistent", type=int, default=0)
    ap.add_argument("--forward-mode", type=int, default=1,
                    help="0: pixel per lane, 1: record per lane, 2: record on lanes")
    ap.add_argument("--autotune", action="store_true", help="pick tile/batch/persistent with svr_autotune")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--model", default="windowed", choices=["windowed", "topk"],
                    help="windowed: the exact-amplitude model with 3-sigma footprints (the hot path); "
                         "topk: the paper's normalised Top-K model (Eqs. 2 and 5)")
    ap.add_argument("--topk-k", type=int, default=50, help="neighbours per pixel (the paper's K)")
    ap.add_argument("--topk-refresh", type=int, default=50, help="iterations between neighbour searches")
    ap.add_argument("--no-learned", action="store_true",
                    help="skip the learned-pose leg (train the pose network, then batched fits of 16 cube "
                         "subjects from identity and from accepted proposals)")
    ap.add_argument("--copy-probe", action="store_true",
                    help="only copy 256 MiB device to device three times (calibrates the HBM traffic counters)")
    return ap


def main():
    ap = build_parser()
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py: the hot path runs on one GPU only; multi-GPU runs are not supported "
              "(a slice-parallel split with an all-reduce of the parameter gradients is how it would shard).",
              file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2512_11624_amd import svr, synth

    if not torch.cuda.is_available():
        raise SystemExit("bench.py needs a GPU")
    if args.copy_probe:
        a = torch.ones(64 * 1024 * 1024, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        log(f"copied {a.numel() * 4} bytes x3")
        return
    dev = torch.device("cuda:0")
    prob, desc = make_workload(args.workload)
    log(f"workload: {desc}; N={prob.n_gauss} M={prob.n_slices} P={prob.n_pixels}")

    ctx = svr.Context(0)
    ctx.svr_set_config(tile=args.tile, batch=args.batch, persistent=args.persistent, cutoff=3.0,
                       forward_mode=args.forward_mode)
    ctx.svr_set_geometry(prob)
    N, M, P = prob.n_gauss, prob.n_slices, prob.n_pixels

    # observations: forward of the ground truth at the true poses + Rician noise (SNR 20)
    gt = svr.Params.from_arrays(*prob.params(), prob.pose)
    ctx.svr_project_bin(*gt.views())
    clean = torch.empty(P, device=dev)
    ctx.svr_forward(clean)
    clean_np = clean.cpu().numpy()
    mask_np = prob.mask
    sigma = float(clean_np[mask_np > 0].mean()) / 20.0 if (mask_np > 0).any() else 0.05
    target_np = synth.rician(clean_np, 1234, sigma)
    target = torch.as_tensor(target_np, device=dev)
    mask = torch.as_tensor(mask_np, device=dev)
    del gt

    # initial iterate: perturbed Gaussians, identity (zero) pose deltas
    init = synth.perturb_params(prob, 7, d_mu=0.2, d_ls=0.05, d_q=0.05, d_c=0.02)
    if args.model == "topk":
        run_topk(args, ctx, prob, desc, init, target, mask, target_np)
        return
    par = svr.Params.from_arrays(*init, np.zeros((M, 6), np.float32))
    grad = svr.Params(N, M)
    m_state = torch.zeros_like(par.flat)
    v_state = torch.zeros_like(par.flat)
    pred = torch.empty(P, device=dev)
    gpred = torch.empty(P, device=dev)
    loss = torch.empty(1, device=dev)
    sse = torch.empty(M, device=dev)
    it = [0]

    def step():
        it[0] += 1
        ctx.svr_project_bin(*par.views())
        ctx.svr_forward(pred, target, mask, loss=loss, slice_sse=sse, grad_pred=gpred)
        ctx.svr_backward(gpred, *grad.views())
        ctx.svr_step(par.views(), grad.views(), m_state, v_state, LR, it[0])

    tuned = None
    if args.autotune:
        ctx.svr_project_bin(*par.views())
        ctx.svr_forward(pred, target, mask, loss=loss, grad_pred=gpred)
        tuned, times = ctx.svr_autotune(*par.views(), gpred)
        log(f"autotune: {tuned} ({len(times)} trials, best {min(times):.3f} ms)")

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()

    # per-stage breakdown over steps of its own, then the timed region with
    # events around the dominant stage only
    n_bk = max(1, min(10, args.steps))
    stages = stage_breakdown(ctx, step, n_bk)
    per_step = {k: v["avg_ms"] * v["calls"] / n_bk for k, v in stages.items()}
    for k, v in sorted(stages.items(), key=lambda kv: -kv[1]["avg_ms"] * kv[1]["calls"]):
        log(f"  {k:18s} {v['calls']:5d} calls  {v['avg_ms']:.4f} ms avg")
    dominant = max(per_step, key=per_step.get)

    # the state the timed steps start from, to count their in-cut pairs by
    # replaying them afterwards (counting inside the timed region would add
    # its own work)
    snap = (par.flat.clone(), m_state.clone(), v_state.clone(), it[0])
    ctx.svr_set_timing_stages([dominant])
    ctx.svr_set_timing(True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    timing = ctx.svr_get_timing()
    ctx.svr_set_timing(False)
    ctx.svr_set_timing_stages(None)
    ms_per_step = (t1 - t0) * 1e3 / args.steps
    final_loss = float(loss.item())

    # replay of the timed steps from the same state, counting each step's
    # in-cut pairs (the algorithmic work of a step) in its forward
    par.flat.copy_(snap[0])
    m_state.copy_(snap[1])
    v_state.copy_(snap[2])
    it[0] = snap[3]
    counts = []
    ctx.svr_set_count_pairs(True)
    for _ in range(args.steps):
        it[0] += 1
        ctx.svr_project_bin(*par.views())
        ctx.svr_forward(pred, target, mask, loss=loss, slice_sse=sse, grad_pred=gpred)
        st = ctx.svr_get_stats(sync=True)
        counts.append(int(st["n_incut"]))
        ctx.svr_backward(gpred, *grad.views())
        ctx.svr_step(par.views(), grad.views(), m_state, v_state, LR, it[0])
    ctx.svr_set_count_pairs(False)
    del snap
    n_incut = int(round(float(np.mean(counts))))
    log(f"stats: {st}")
    value = float(np.sum(counts)) / ((t1 - t0))
    dom_calls, dom_total = timing[dominant]
    dom_ms = dom_total / dom_calls
    log(f"{ms_per_step:.3f} ms/step, {value:.4g} pair-evals/s, loss {final_loss:.5g}; "
        f"{dominant} {dom_ms:.4f} ms avg in the timed region")

    rl = stage_roofline(dominant, dom_ms, st, n_incut)
    roofline = None
    if rl:
        bound, achieved, peak, unit, work = rl
        traffic = measured_traffic(dominant, ctx.svr_get_config()["tile"], args.workload)
        roofline = dict(bound=bound, achieved=round(achieved, 4), peak=peak, unit=unit,
                        frac=round(achieved / peak, 6), traffic=traffic, kernel=dominant,
                        avg_ms=round(dom_ms, 5), work_per_launch=work)
        alu = stage_alu(dominant, dom_ms, n_incut)
        if alu and bound != "alu":
            roofline["alu"] = alu

    sequential = None
    if args.workload == "batched":
        sequential = sequential_subjects(prob, par, target, mask, ctx.svr_get_config(), args.steps, args.warmup)
        sequential["batched_speedup"] = sequential["ms_per_round"] / ms_per_step
        log(f"sequential: {sequential}")

    cfg = ctx.svr_get_config()
    learned = None
    if not args.no_learned and args.workload == "head":
        ctx.close()
        ctx = None
        from paper_2512_11624_amd import pose
        learned = pose.run_learned_vs_plain(log=log)
        log(f"learned vs plain: median {learned['median_t_learned']:.4f} s vs {learned['median_t_plain']:.4f} s, "
            f"learned faster on {learned['learned_faster']} of {learned['subjects']}")

    cpu = None
    if not args.no_cpu_baseline and args.workload != "batched":
        try:
            cpu = cpu_baseline(prob, init, np.zeros((M, 6), np.float32), target_np)
            log(f"cpu baseline: {cpu}")
        except Exception as e:  # reported, never silently replaced
            cpu = dict(error=str(e))

    out = {
        "metric": METRIC,
        "value": value,
        "unit": "pair-evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": desc, "gaussians": N, "slices": M, "pixels": P,
                   "tile": cfg["tile"], "batch": cfg["batch"],
                   "persistent": cfg["persistent"], "cutoff_sigma": 3.0,
                   "forward_mode": cfg["forward_mode"],
                   "step": "project_bin+forward(masked MSE)+backward+AdamW", "autotuned": tuned is not None,
                   "observations": OBSERVATIONS[args.workload],
                   "pair_count": "in-cut pairs of every timed step, counted by replaying the timed steps "
                                 "from their starting state"},
        "pairs": {"in_cut_per_step": n_incut, "in_cut_min": min(counts), "in_cut_max": max(counts),
                  "records": st["n_records"], "instances": st["n_instances"],
                  "candidates": st["n_candidates"], "evaluated_upper_bound": st["n_evaluated"]},
        "stages_ms_per_step": {k: round(v, 5) for k, v in per_step.items()},
        "final_loss": final_loss,
        "roofline": roofline,
        "cpu_baseline": cpu,
    }
    if sequential is not None:
        out["sequential_16_runs"] = sequential
    if learned is not None:
        out["learned_vs_plain"] = learned
    print(json.dumps(out), flush=True)
    if ctx is not None:
        ctx.close()


def run_topk(args, ctx, prob, desc, init, target, mask, target_np):
    """One step = svr_topk_forward (masked MSE) + svr_topk_backward + AdamW,
    with the neighbour lists rebuilt every --topk-refresh steps (the paper
    refreshes its index every 50 epochs); the search is timed separately and
    its cost is spread over the refresh interval.  value = pixel-neighbour
    pairs per step (K per pixel inside the mask, the pixels that have lists)
    / amortised seconds per step."""
    import torch
    from paper_2512_11624_amd import svr
    N, M, P = prob.n_gauss, prob.n_slices, prob.n_pixels
    K, delta = args.topk_k, 1e-6
    dev = target.device
    par = svr.Params.from_arrays(*init, np.zeros((M, 6), np.float32))
    grad = svr.Params(N, M)
    m_state = torch.zeros_like(par.flat)
    v_state = torch.zeros_like(par.flat)
    pred = torch.empty(P, device=dev)
    gpred = torch.empty(P, device=dev)
    loss = torch.empty(1, device=dev)
    nbr = torch.empty(P, K, dtype=torch.int32, device=dev)
    it = [0]

    def build():
        v = par.views()
        ctx.svr_topk_build(v[0], v[4], K, nbr, mask=mask)

    def step():
        it[0] += 1
        ctx.svr_topk_forward(*par.views(), nbr, K, delta, pred, target, mask, loss=loss, grad_pred=gpred)
        ctx.svr_topk_backward(*par.views(), nbr, K, gpred, *grad.views())
        ctx.svr_step(par.views(), grad.views(), m_state, v_state, LR, it[0])

    build()
    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    # per-stage breakdown (list build and iterations) over runs of their own,
    # then the timed region with events around the dominant iteration stage only
    n_bk = max(1, min(10, args.steps))

    def build_and_steps():
        build()
        for _ in range(n_bk):
            step()

    stages = stage_breakdown(ctx, build_and_steps, 1)
    for k, v in sorted(stages.items(), key=lambda kv: -kv[1]["avg_ms"] * kv[1]["calls"]):
        log(f"  {k:18s} {v['calls']:5d} calls  {v['avg_ms']:.4f} ms avg")
    per_step = {k: v["avg_ms"] * v["calls"] / n_bk for k, v in stages.items()
                if k not in ("topk_knn", "topk_inverse")}
    dominant = max(per_step, key=per_step.get)
    nb = max(1, min(3, args.steps))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(nb):
        build()
    torch.cuda.synchronize()
    ms_build = (time.perf_counter() - t0) * 1e3 / nb
    ctx.svr_set_timing_stages([dominant])
    ctx.svr_set_timing(True)
    t0 = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    ms_iter = (time.perf_counter() - t0) * 1e3 / args.steps
    timing = ctx.svr_get_timing()
    ctx.svr_set_timing(False)
    ctx.svr_set_timing_stages(None)
    dom_calls, dom_total = timing[dominant]
    dom_ms = dom_total / dom_calls
    ms_per_step = ms_iter + ms_build / args.topk_refresh
    # lists exist for the pixels inside the mask only; the others predict 0
    pairs = int((prob.mask > 0).sum()) * K
    value = pairs / (ms_per_step / 1e3)
    log(f"topk: build {ms_build:.3f} ms, iteration {ms_iter:.3f} ms, amortised {ms_per_step:.3f} ms/step, "
        f"{value:.4g} pair-evals/s; {dominant} {dom_ms:.4f} ms avg in the timed region")
    rl = stage_roofline(dominant, dom_ms, {}, pairs)
    roofline = None
    if rl:
        bound, achieved, peak, unit, work = rl
        roofline = dict(bound=bound, achieved=round(achieved, 4), peak=peak, unit=unit,
                        frac=round(achieved / peak, 6), traffic=None, kernel=dominant,
                        avg_ms=round(dom_ms, 5), work_per_launch=work)
    cpu = None
    if not args.no_cpu_baseline:
        cpu = topk_cpu_baseline(prob, init, target_np, K, delta)
        log(f"cpu baseline: {cpu}")
    out = {
        "metric": "pixel-neighbour pair evals/s fwd+bwd (normalised Top-K model)",
        "value": value, "unit": "pair-evals/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": ms_per_step, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": desc, "model": "normalised Top-K (Eqs. 2 and 5)", "K": K, "delta": delta,
                   "refresh_every": args.topk_refresh, "gaussians": N, "slices": M, "pixels": P,
                   "pixels_with_lists": int((prob.mask > 0).sum()), "pairs_per_step": pairs,
                   "step": "topk_forward(masked MSE)+topk_backward+AdamW, neighbour search amortised"},
        "ms_build": ms_build, "ms_iteration": ms_iter,
        "stages_ms_per_step": {k: round(v, 5) for k, v in per_step.items()},
        "final_loss": float(loss.item()), "roofline": roofline, "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)
    ctx.close()


def topk_cpu_baseline(prob, params, target, K, delta, n_pix=20000):
    """The FP64 Top-K oracle on a bounded sample: neighbour search, forward
    and autograd adjoint for n_pix masked pixels."""
    import torch
    from oracle import topk
    rng = np.random.default_rng(5)
    pix = np.sort(rng.choice(np.nonzero(prob.mask > 0)[0], n_pix, replace=False))
    pose = np.zeros((prob.n_slices, 6))
    t0 = time.perf_counter()
    nbr, _ = topk.knn(prob, params[0], pose, K, pixels=pix)
    y, _, _ = topk.forward_np(prob, params, pose, nbr, delta, pixels=pix)
    topk.gradients(prob, params, pose, nbr, delta, 2.0 * (y - target[pix]) / n_pix, pixels=pix)
    sec = time.perf_counter() - t0
    return dict(value=n_pix * K / sec, unit="pair-evals/s", cores=torch.get_num_threads(), kind="oracle",
                sample=f"{n_pix} masked pixels x K={K}: neighbour search, forward, autograd adjoint")


if __name__ == "__main__":
    main()
