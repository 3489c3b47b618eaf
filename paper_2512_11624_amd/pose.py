"""Learned pose proposal: training data, training and the proposal /
acceptance step.  Control flow and marshalling only; the slices are rendered
by the library's own forward kernels, the network runs on its BF16-MFMA
kernels, and the acceptance test uses the forward model's per-slice error.

* Template volumes: a fixed cloud of 2,000 cube Gaussians (seed 1234) and
  per-subject perturbations (mu += N(0, 0.5^2) mm, log-scale += N(0, 0.1^2),
  c *= U[0.9, 1.1]) so that slice content carries information about pose.
* Training slices: each volume is rendered at the cube geometry (three
  orthogonal stacks of 16 slices of 32x32 px at 1x1x3 mm) under random motion
  (angle U[0, 15 deg] about a uniform axis, translation U[-8, 8]^3 mm) plus
  N(0, 0.01^2) noise; the label is that motion.
* Network input: the slice's centre 32x32 window upsampled x4 to 128x128,
  and its nominal placement (stack rotation R0, nominal centre t0 / 16 mm);
  output: the 6-DoF motion in scaled units (omega / 0.25 rad, tau / 8 mm).
* Acceptance: a proposed pose is kept for a slice only where it lowers that
  slice's forward-model error (masked SSE) against the current volume; the
  plain pose optimisation has the last word.
"""
from __future__ import annotations

import math
import time

import numpy as np

from . import svr, synth

OMEGA_SCALE = 0.25   # rad
TAU_SCALE = 8.0      # mm
T0_SCALE = 16.0      # mm


def template(seed=1234):
    return synth.config1(seed)


def subject_params(tmpl: synth.Problem, seed: int):
    r1, r2, r3 = [np.random.default_rng(s) for s in np.random.SeedSequence(seed).spawn(3)]
    n = tmpl.n_gauss
    mu = tmpl.mean + r1.normal(0.0, 0.5, (n, 3))
    ls = tmpl.log_scale + r2.normal(0.0, 0.1, (n, 3))
    c = tmpl.amp * r3.uniform(0.9, 1.1, n)
    return [np.ascontiguousarray(a, np.float32) for a in (mu, ls, tmpl.quat, c)]


def random_motion(rng, m, max_deg, max_mm):
    axis = rng.standard_normal((m, 3))
    axis /= np.linalg.norm(axis, axis=1, keepdims=True)
    ang = rng.uniform(0.0, math.radians(max_deg), (m, 1))
    tau = rng.uniform(-max_mm, max_mm, (m, 3))
    return np.concatenate([axis * ang, tau], 1).astype(np.float32)


def placement(prob: synth.Problem):
    """[M, 12]: R0 (row-major) and t0 / 16 mm."""
    return np.concatenate([prob.rot0.reshape(-1, 9), prob.trans0 / T0_SCALE], 1).astype(np.float32)


def to_scaled(pose):
    out = np.array(pose, np.float32, copy=True)
    out[..., :3] /= OMEGA_SCALE
    out[..., 3:] /= TAU_SCALE
    return out


def from_scaled(y):
    out = np.array(y, np.float32, copy=True)
    out[..., :3] *= OMEGA_SCALE
    out[..., 3:] *= TAU_SCALE
    return out


def simulate(n_volumes, renders_per_volume, seed=0, max_deg=15.0, max_mm=8.0, noise=0.01, device=0):
    """Training set on the GPU: slices [n, 32, 32], placement [n, 12], labels
    [n, 6] (scaled).  n = n_volumes * renders_per_volume * 48."""
    import torch
    geo = template()
    ctx = svr.Context(device)
    ctx.svr_set_config(tile=16, batch=128, persistent=0, cutoff=3.0, forward_mode=1)
    ctx.svr_set_geometry(geo)
    M, P = geo.n_slices, geo.n_pixels
    pl = torch.as_tensor(placement(geo), device="cuda")
    total = n_volumes * renders_per_volume * M
    slices = torch.empty(total, 32, 32, device="cuda")
    plac = torch.empty(total, 12, device="cuda")
    labels = torch.empty(total, 6, device="cuda")
    rng = np.random.default_rng(seed)
    gen = torch.Generator(device="cuda").manual_seed(seed)
    pred = torch.empty(P, device="cuda")
    k = 0
    for v in range(n_volumes):
        prm = [torch.as_tensor(a, device="cuda") for a in subject_params(geo, 1000 + v)]
        for _ in range(renders_per_volume):
            mot = random_motion(rng, M, max_deg, max_mm)
            ctx.svr_project_bin(*prm, torch.as_tensor(mot, device="cuda"))
            ctx.svr_forward(pred)
            slices[k:k + M] = pred.view(M, 32, 32) + noise * torch.randn(M, 32, 32, device="cuda", generator=gen)
            plac[k:k + M] = pl
            labels[k:k + M] = torch.as_tensor(to_scaled(mot), device="cuda")
            k += M
    ctx.close()
    return slices, plac, labels


def train(net: svr.PoseNet, slices, plac, labels, epochs=8, batch=256, lr=1e-3, seed=0, log=None):
    """Mini-batch Adam over the simulated set; the learning rate halves every
    two epochs.  Returns per-epoch mean losses and the wall time."""
    import torch
    n = slices.shape[0]
    g = torch.Generator(device="cuda").manual_seed(seed)
    crops = torch.empty(batch, 128, 128, device="cuda")
    loss = torch.empty(1, device="cuda")
    hist = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for ep in range(epochs):
        perm = torch.randperm(n, device="cuda", generator=g)
        acc, cnt = torch.zeros(1, device="cuda"), 0
        lr_ep = lr * (0.5 ** (ep // 2))
        for b0 in range(0, n - batch + 1, batch):
            idx = perm[b0:b0 + batch]
            net.prepare(slices[idx].contiguous(), crops)
            net.train_step(crops.view(batch, 1, 128, 128), plac[idx].contiguous(), labels[idx].contiguous(), lr_ep,
                           loss)
            acc += loss
            cnt += 1
        hist.append(float(acc.item()) / max(cnt, 1))
        if log:
            log(f"epoch {ep}: loss {hist[-1]:.4f} (lr {lr_ep:g})")
    torch.cuda.synchronize()
    return hist, time.perf_counter() - t0


def propose(net: svr.PoseNet, observed, plac):
    """observed [M, H, W] (device), plac [M, 12] -> proposed poses [M, 6] (device, rad / mm)."""
    import torch
    M, H, W = observed.shape
    crops = torch.empty(M, 128, 128, device="cuda")
    out = torch.empty(M, 6, device="cuda")
    for b0 in range(0, M, net.max_batch):
        b1 = min(M, b0 + net.max_batch)
        net.prepare(observed[b0:b1].contiguous(), crops[b0:b1])
        net.forward(crops[b0:b1].view(b1 - b0, 1, 128, 128), plac[b0:b1].contiguous(), out[b0:b1])
    scale = torch.tensor([OMEGA_SCALE] * 3 + [TAU_SCALE] * 3, device="cuda")
    return out * scale


def accept(ctx, params4, pose_zero, pose_prop, target, mask):
    """Per slice, keep the proposal only where the forward-model error (masked
    SSE of the slice) is lower than at the current pose."""
    import torch
    P = ctx.n_pixels
    M = pose_zero.shape[0]
    pred = torch.empty(P, device="cuda")
    sse0 = torch.empty(M, device="cuda")
    sse1 = torch.empty(M, device="cuda")
    loss = torch.empty(1, device="cuda")
    ctx.svr_project_bin(*params4, pose_zero)
    ctx.svr_forward(pred, target, mask, loss=loss, slice_sse=sse0)
    ctx.svr_project_bin(*params4, pose_prop)
    ctx.svr_forward(pred, target, mask, loss=loss, slice_sse=sse1)
    keep = (sse1 < sse0).unsqueeze(1)
    return torch.where(keep, pose_prop, pose_zero), keep.squeeze(1)


# ---------------------------------------------------------------------------
# Evaluation: seconds to the plain method's PSNR, learned vs identity init
# ---------------------------------------------------------------------------

def _grid_probe(n_gauss, gt_params, shape=(64, 64, 64), h=0.5, half=16.0, device=0):
    """Volume probe over the cube on a 0.5 mm grid; the ground-truth volume is
    the library's read-out of the true Gaussians with a wide window (6 sigma)."""
    import torch
    from . import recon
    gt_probe = recon.VolumeProbe(n_gauss, shape, h, (0, 0, 0), np.zeros(1), np.zeros(1), device=device, cutoff=6.0)
    gt = gt_probe.render(*[torch.as_tensor(a, device="cuda") for a in gt_params]).cpu().numpy().copy()
    gt_probe.close()
    c = recon.voxel_centres(shape, h)
    vmask = np.all(np.abs(c) <= half, axis=1).astype(np.float32)
    return recon.VolumeProbe(n_gauss, shape, h, (0, 0, 0), gt, vmask, device=device)


def observe(geo, gt_params, seed, noise=0.01, device=0):
    """Observed slices of one subject: the library forward of the true
    Gaussians at the true motion with a 6-sigma window, plus N(0, noise^2)."""
    import torch
    ctx = svr.Context(device)
    ctx.svr_set_config(tile=16, batch=128, persistent=0, cutoff=6.0, forward_mode=1)
    ctx.svr_set_geometry(geo)
    pred = torch.empty(geo.n_pixels, device="cuda")
    ctx.svr_project_bin(*[torch.as_tensor(a, device="cuda") for a in gt_params],
                        torch.as_tensor(geo.pose, device="cuda"))
    ctx.svr_forward(pred)
    torch.cuda.synchronize()
    ctx.close()
    return pred + torch.as_tensor(synth.gaussian_noise(seed, geo.n_pixels, noise), device="cuda")


def evaluate_subject(net, seed, n_iter=300, psnr_every=10, tmpl=None, device=0, lr=None):
    """One held-out subject (cube geometry and motion of the given seed, volume
    = template perturbation of the seed): fits from the template with identity
    poses (plain) and from the network's accepted proposals (learned).  The
    learned clock includes the network and the acceptance forwards."""
    import torch
    from . import recon
    tmpl = tmpl if tmpl is not None else template()
    geo = synth.config1(seed)
    gt = subject_params(tmpl, seed)
    target = observe(geo, gt, seed, device=device)
    mask = torch.as_tensor(geo.mask, device="cuda")
    probe = _grid_probe(tmpl.n_gauss, gt, device=device)
    ctx = svr.Context(device)
    ctx.svr_set_config(tile=16, batch=128, persistent=0, cutoff=3.0, forward_mode=1)
    ctx.svr_set_geometry(geo)
    lr = lr or recon.PAPER_LR
    init = [tmpl.mean, tmpl.log_scale, tmpl.quat, tmpl.amp]
    zero = np.zeros((geo.n_slices, 6), np.float32)
    # one untimed iteration first, so that neither timed fit pays the
    # context's first-call allocations
    recon.fit(ctx, svr.Params.from_arrays(*init, zero), target, mask, 1, lr=lr)
    torch.cuda.synchronize()

    plain = recon.fit(ctx, svr.Params.from_arrays(*init, zero), target, mask, n_iter, lr=lr, probe=probe,
                      psnr_every=psnr_every)

    params = svr.Params.from_arrays(*init, zero)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    obs = target.view(geo.n_slices, int(geo.height[0]), int(geo.width[0]))
    prop = propose(net, obs, torch.as_tensor(placement(geo), device="cuda"))
    pose0, keep = accept(ctx, params.views()[:4], params.views()[4].clone(), prop, target, mask)
    params.views()[4].copy_(pose0)
    torch.cuda.synchronize()
    t_init = time.perf_counter() - t0
    learned = recon.fit(ctx, params, target, mask, n_iter, lr=lr, probe=probe, psnr_every=psnr_every)
    learned.times = [t + t_init for t in learned.times]
    learned.seconds += t_init

    goal = plain.final_psnr - 0.1
    true_pose = geo.pose.astype(np.float64)
    err0 = np.abs(true_pose).mean(0)
    err1 = np.abs(pose0.cpu().numpy().astype(np.float64) - true_pose).mean(0)
    probe.close()
    ctx.close()
    return dict(seed=seed, plain_final_psnr=plain.final_psnr, learned_final_psnr=learned.final_psnr,
                target_psnr=goal, t_plain=recon.time_to_target(plain, goal),
                t_learned=recon.time_to_target(learned, goal), t_init=t_init,
                accepted=int(keep.sum().item()), n_slices=geo.n_slices,
                pose_err_identity=[float(x) for x in err0], pose_err_proposed=[float(x) for x in err1])


def main(argv=None):
    import argparse
    import json
    import torch
    ap = argparse.ArgumentParser(description="Train the pose network on simulated slices and compare time to "
                                             "the plain method's PSNR with and without its proposals.")
    ap.add_argument("--volumes", type=int, default=1000)
    ap.add_argument("--renders", type=int, default=4)
    ap.add_argument("--epochs", type=int, default=8)
    ap.add_argument("--batch", type=int, default=256)
    ap.add_argument("--lr", type=float, default=1e-3)
    ap.add_argument("--iters", type=int, default=300)
    ap.add_argument("--subjects", type=int, default=16)
    ap.add_argument("--seed", type=int, default=0)
    a = ap.parse_args(argv)
    log = lambda s: print(s, flush=True)  # noqa: E731
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    slices, plac, labels = simulate(a.volumes, a.renders, seed=a.seed)
    torch.cuda.synchronize()
    t_sim = time.perf_counter() - t0
    log(f"simulated {slices.shape[0]} slices in {t_sim:.1f} s")
    net = svr.PoseNet(0, seed=a.seed, max_batch=a.batch)
    hist, t_train = train(net, slices, plac, labels, epochs=a.epochs, batch=a.batch, lr=a.lr, log=log)
    log(f"trained in {t_train:.1f} s")
    del slices, plac, labels
    tmpl = template()
    # load and warm the network's kernels once, as a reconstruction service would
    warm = torch.zeros(48, 32, 32, device="cuda")
    propose(net, warm, torch.zeros(48, 12, device="cuda"))
    torch.cuda.synchronize()
    rows = []
    for s in range(100, 100 + a.subjects):
        r = evaluate_subject(net, s, n_iter=a.iters, tmpl=tmpl)
        rows.append(r)
        log(json.dumps(r))
    tp = np.array([r["t_plain"] for r in rows])
    tl = np.array([r["t_learned"] for r in rows])
    out = dict(metric="seconds to the plain method's PSNR - 0.1 dB", n_subjects=len(rows),
               median_t_plain=float(np.median(tp)), median_t_learned=float(np.median(tl)),
               learned_faster=int(np.sum(tl < tp)), learned_reached=int(np.sum(np.isfinite(tl))),
               mean_accepted=float(np.mean([r["accepted"] / r["n_slices"] for r in rows])),
               train_seconds=t_train, simulate_seconds=t_sim, train_loss=hist,
               n_train=a.volumes * a.renders * 48)
    print(json.dumps(out), flush=True)
    net.close()


if __name__ == "__main__":
    main()
