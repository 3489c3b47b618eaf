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


def simulate(n_volumes, renders_per_volume, seed=0, max_deg=15.0, max_mm=8.0, noise=0.01, device=0, vol_seed0=1000):
    """Training set on the GPU: slices [n, 32, 32], placement [n, 12], labels
    [n, 6] (scaled).  n = n_volumes * renders_per_volume * 48; volume v is
    the template perturbation of seed vol_seed0 + v."""
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
        prm = [torch.as_tensor(a, device="cuda") for a in subject_params(geo, vol_seed0 + v)]
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


def accept(ctx, params4, pose_zero, pose_prop, target, mask, translation_only=True, full=True):
    """Per slice, keep a candidate pose only where the forward-model error
    (masked SSE of the slice) is lower than at the current pose.  The
    candidates are the proposal and, with ``translation_only``, the proposal
    with its rotation part replaced by the current one (the network's
    rotation estimates carry less information than its translations; the
    forward model decides per slice).  Returns the poses and, per slice, the
    candidate kept (0 current, 1 proposal, 2 translation-only proposal);
    ``full=False`` leaves the whole proposal out (its error is not computed
    and it is never kept)."""
    import torch
    P = ctx.n_pixels
    M = pose_zero.shape[0]
    pred = torch.empty(P, device="cuda")
    loss = torch.empty(1, device="cuda")
    cands = [pose_zero, pose_prop if full else pose_zero]
    if translation_only:
        cands.append(torch.cat([pose_zero[:, :3], pose_prop[:, 3:]], 1).contiguous())
    sse = torch.empty(len(cands), M, device="cuda")
    for k, c in enumerate(cands):
        ctx.svr_project_bin(*params4, c)
        ctx.svr_forward(pred, target, mask, loss=loss, slice_sse=sse[k])
    choice = torch.argmin(sse, 0)  # ties keep the earlier candidate (the current pose first)
    out = torch.stack(cands, 0).gather(0, choice.view(1, M, 1).expand(1, M, 6)).squeeze(0)
    return out.contiguous(), choice


def component_r2(net, n_volumes=8, renders=2, max_deg=5.0, max_mm=2.0, seed=77, vol_seed0=5000):
    """How much the network's proposal explains of each motion component on
    held-out volumes (seeds vol_seed0...) under motion of angle <= max_deg and
    translation <= max_mm: R^2 = 1 - E[(pred - label)^2] / E[label^2] per
    component (omega_x, omega_y, omega_z, tau_x, tau_y, tau_z); 1 is exact,
    0 is no better than proposing zero motion."""
    import torch
    slices, plac, labels = simulate(n_volumes, renders, seed=seed, max_deg=max_deg, max_mm=max_mm,
                                    vol_seed0=vol_seed0)
    pred = propose(net, slices, plac)
    lab = labels * torch.tensor([OMEGA_SCALE] * 3 + [TAU_SCALE] * 3, device="cuda")
    err = ((pred - lab) ** 2).mean(0)
    var = (lab ** 2).mean(0)
    return [float(x) for x in (1.0 - err / var).cpu()]


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
    pose0, choice = accept(ctx, params.views()[:4], params.views()[4].clone(), prop, target, mask)
    keep = choice > 0
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


class BatchedProbe:
    """PSNR of every subject of a batched fit against its own ground-truth
    volume, in one launch: the 0.5 mm cube grid (zero PSF, identity poses)
    is repeated once per subject, the fitted Gaussians of subject k render
    onto copy k, and the forward's per-slice masked SSE is summed per
    subject.  The ground truth is the read-out of each subject's true
    Gaussians with a 6-sigma window."""

    def __init__(self, gauss_offsets, gt_params, shape=(64, 64, 64), h=0.5, half=16.0, device=0):
        import dataclasses
        import torch
        from . import recon
        S = len(gauss_offsets) - 1
        grid = recon.volume_grid(shape, h)
        subs = []
        for k in range(S):
            n = int(gauss_offsets[k + 1] - gauss_offsets[k])
            subs.append(dataclasses.replace(grid, mean=np.zeros((n, 3), np.float32),
                                            log_scale=np.zeros((n, 3), np.float32),
                                            quat=np.zeros((n, 4), np.float32), amp=np.zeros(n, np.float32),
                                            gauss_offsets=np.array([0, n], np.int64)))
        self.geom = synth.concat(subs)
        c = recon.voxel_centres(shape, h)
        vm = np.all(np.abs(c) <= half, axis=1).astype(np.float32)
        self.S, self.nz = S, int(shape[0])
        self.msum = float(vm.sum())
        dev = torch.device("cuda", device)
        self.mask = torch.as_tensor(np.tile(vm, S), device=dev)
        self.pose = torch.zeros((self.geom.n_slices, 6), dtype=torch.float32, device=dev)
        self.vol = torch.empty(self.geom.n_pixels, dtype=torch.float32, device=dev)
        self.sse = torch.empty(self.geom.n_slices, dtype=torch.float32, device=dev)
        self.loss = torch.empty(1, dtype=torch.float32, device=dev)
        ref = svr.Context(device)
        ref.svr_set_config(tile=16, batch=128, persistent=0, cutoff=6.0, forward_mode=1)
        ref.svr_set_geometry(self.geom)
        ref.svr_project_bin(*[torch.as_tensor(np.concatenate([g[i] for g in gt_params]), device=dev)
                              for i in range(4)], self.pose)
        self.gt = torch.empty_like(self.vol)
        ref.svr_forward(self.gt)
        torch.cuda.synchronize()
        ref.close()
        g = (self.gt.view(S, -1) * self.mask.view(S, -1)).max(1).values
        self.max_gt = [float(x) for x in g.cpu()]
        self.ctx = svr.Context(device)
        self.ctx.svr_set_config(tile=16, batch=128, persistent=0, cutoff=3.0, forward_mode=1)
        self.ctx.svr_set_geometry(self.geom)
        self.last = []

    def psnr(self, mean, log_scale, quat, amp):
        """Mean PSNR over the subjects; the per-subject values go to .last."""
        self.ctx.svr_project_bin(mean, log_scale, quat, amp, self.pose)
        self.ctx.svr_forward(self.vol, self.gt, self.mask, loss=self.loss, slice_sse=self.sse)
        sse = self.sse.view(self.S, self.nz).sum(1).cpu().numpy().astype(np.float64)
        self.last = [10.0 * math.log10(m * m / max(e / self.msum, 1e-30)) for m, e in zip(self.max_gt, sse)]
        return float(np.mean(self.last))

    def close(self):
        self.ctx.close()


def _first_time(times, values, goal):
    for t, v in zip(times, values):
        if v >= goal:
            return t
    return float("inf")


def evaluate_batched(net, seeds, n_iter=300, psnr_every=10, tmpl=None, device=0, lr=None, translation_only=True,
                     full=True):
    """The held-out subjects (cube geometry, motion and volume of each seed)
    reconstructed together in one batched persistent launch per stage, twice:
    from the template with identity poses (plain) and from the network's
    accepted proposals (learned; the clock includes the network and the
    acceptance forwards).  Per subject, the target is the plain fit's final
    PSNR - 0.1 dB; returns the times to reach it and the whole batch's."""
    import torch
    from . import recon
    tmpl = tmpl if tmpl is not None else template()
    geos = [synth.config1(s) for s in seeds]
    gts = [subject_params(tmpl, s) for s in seeds]
    targets = [observe(g, gt, s, device=device) for g, gt, s in zip(geos, gts, seeds)]
    init_subj = [dataclasses_replace(g, tmpl) for g in geos]
    batch = synth.concat(init_subj)
    target = torch.cat(targets)
    mask = torch.as_tensor(batch.mask, device="cuda")
    probe = BatchedProbe(batch.gauss_offsets, gts, device=device)
    ctx = svr.Context(device)
    ctx.svr_set_config(tile=16, batch=128, persistent=1, cutoff=3.0, forward_mode=1)
    ctx.svr_set_geometry(batch)
    lr = lr or recon.PAPER_LR
    init = batch.params()
    zero = np.zeros((batch.n_slices, 6), np.float32)
    recon.fit(ctx, svr.Params.from_arrays(*init, zero), target, mask, 1, lr=lr)  # first-call allocations
    torch.cuda.synchronize()

    def run(params, t_init):
        rec = []
        cb = lambda it, el, p, l: rec.append((el + t_init, list(probe.last)))  # noqa: E731
        res = recon.fit(ctx, params, target, mask, n_iter, lr=lr, probe=probe, psnr_every=psnr_every, callback=cb)
        return res, [r[0] for r in rec], np.array([r[1] for r in rec])

    _, tp, psp = run(svr.Params.from_arrays(*init, zero), 0.0)
    params = svr.Params.from_arrays(*init, zero)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    obs = target.view(batch.n_slices, 32, 32)
    prop = propose(net, obs, torch.as_tensor(placement(batch), device="cuda"))
    pose0, choice = accept(ctx, params.views()[:4], params.views()[4].clone(), prop, target, mask,
                           translation_only=translation_only, full=full)
    params.views()[4].copy_(pose0)
    torch.cuda.synchronize()
    t_init = time.perf_counter() - t0
    _, tl, psl = run(params, t_init)
    goals = psp[-1] - 0.1
    S = len(seeds)
    t_plain = [_first_time(tp, psp[:, k], goals[k]) for k in range(S)]
    t_learned = [_first_time(tl, psl[:, k], goals[k]) for k in range(S)]
    all_p = _first_time(tp, (psp - goals[None, :]).min(1), 0.0)
    all_l = _first_time(tl, (psl - goals[None, :]).min(1), 0.0)
    ch = choice.cpu().numpy()
    true_pose = batch.pose.astype(np.float64)
    err0 = np.abs(true_pose).mean(0)
    err1 = np.abs(pose0.cpu().numpy().astype(np.float64) - true_pose).mean(0)
    probe.close()
    ctx.close()
    tpa, tla = np.array(t_plain), np.array(t_learned)
    return dict(subjects=S, iterations=n_iter, psnr_every=psnr_every,
                median_t_plain=float(np.median(tpa)), median_t_learned=float(np.median(tla)),
                learned_faster=int(np.sum(tla < tpa)), learned_reached=int(np.sum(np.isfinite(tla))),
                t_all_plain=float(all_p), t_all_learned=float(all_l), t_init=t_init,
                plain_final_psnr_mean=float(psp[-1].mean()), learned_final_psnr_mean=float(psl[-1].mean()),
                accepted_full=float(np.mean(ch == 1)), accepted_translation=float(np.mean(ch == 2)),
                pose_err_identity=[float(x) for x in err0], pose_err_accepted=[float(x) for x in err1],
                t_plain=t_plain, t_learned=t_learned, plain_final_psnr=[float(x) for x in psp[-1]],
                learned_final_psnr=[float(x) for x in psl[-1]])


def dataclasses_replace(geo: synth.Problem, tmpl: synth.Problem) -> synth.Problem:
    """The subject's geometry (slices, motion, mask) with the template's
    Gaussians as the starting volume."""
    import dataclasses
    return dataclasses.replace(geo, mean=tmpl.mean.copy(), log_scale=tmpl.log_scale.copy(), quat=tmpl.quat.copy(),
                               amp=tmpl.amp.copy(), gauss_offsets=np.array([0, tmpl.n_gauss], np.int64))


def run_learned_vs_plain(volumes=1000, renders=4, epochs=8, batch=256, lr=1e-3, iters=300, subjects=16, seed=0,
                         psnr_every=10, log=None):
    """Simulate the training slices, train the network, measure how much of
    each motion component it explains, and compare the batched
    reconstruction of the held-out subjects (seeds 100...) from identity poses
    and from the accepted proposals.  Training is timed apart from the fits."""
    import torch
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    slices, plac, labels = simulate(volumes, renders, seed=seed)
    torch.cuda.synchronize()
    t_sim = time.perf_counter() - t0
    if log:
        log(f"simulated {slices.shape[0]} slices in {t_sim:.1f} s")
    net = svr.PoseNet(0, seed=seed, max_batch=batch)
    hist, t_train = train(net, slices, plac, labels, epochs=epochs, batch=batch, lr=lr, log=log)
    if log:
        log(f"trained in {t_train:.1f} s")
    del slices, plac, labels
    r2_eval = component_r2(net, max_deg=5.0, max_mm=2.0)
    r2_train = component_r2(net, max_deg=15.0, max_mm=8.0, seed=78)
    # load and warm the network's kernels once, as a reconstruction service would
    propose(net, torch.zeros(48, 32, 32, device="cuda"), torch.zeros(48, 12, device="cuda"))
    torch.cuda.synchronize()
    res = evaluate_batched(net, list(range(100, 100 + subjects)), n_iter=iters, psnr_every=psnr_every)
    net.close()
    res.update(metric="seconds to the plain method's PSNR - 0.1 dB, learned-pose vs identity initialisation, "
                      "all subjects in one batched persistent launch",
               train_seconds=t_train, simulate_seconds=t_sim, n_train=volumes * renders * 48, train_loss=hist,
               r2_eval_motion=r2_eval, r2_train_motion=r2_train)
    return res


def main(argv=None):
    import argparse
    import json
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
    res = run_learned_vs_plain(a.volumes, a.renders, a.epochs, a.batch, a.lr, a.iters, a.subjects, a.seed, log=log)
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
