"""Reconstruction driver on top of the svr C ABI: volume read-out / PSNR and
the fitting loop.  Argument marshalling and control flow only -- every
numerical step (forward model, loss, adjoint, AdamW, read-out) runs in the
HIP kernels of libsvr.

* Volume read-out (target resolution 0.5 mm, Sec. 3.2 of the paper): the
  volume V(x) = sum_j c_j exp(-1/2 d^T Sigma_j^-1 d) on a voxel grid is the
  forward model with a zero PSF evaluated on axis-aligned grid planes (each
  z-plane of the grid is a "slice" with identity rotation and zero motion),
  so the same project_bin / forward kernels produce it.  PSNR (Sec. 3.3) is
  10 log10(MAX^2 / MSE) over a mask, MAX the largest ground-truth value in
  the mask; the masked MSE comes from the forward kernel's loss epilogue.
* Fitting (App. A.1): AdamW with per-group learning rates and a StepLR that
  halves every 200 iterations; poses start at the nominal (identity) pose.
"""
from __future__ import annotations

import math
import time
from dataclasses import dataclass, field

import numpy as np

from . import svr
from .synth import Problem

PAPER_LR = (2.5e-2, 2.5e-2, 1e-2, 1e-2, 2.5e-3, 1e-1)   # mean, log-scale, quat, amp, rotation, translation


def volume_grid(shape, spacing, centre=(0.0, 0.0, 0.0)):
    """Geometry of a voxel grid of shape (nz, ny, nx) and isotropic spacing:
    one axial slice per z-plane, zero PSF, zero motion.  Voxel (k, r, c) sits
    at centre + ((c-(nx-1)/2) h, (r-(ny-1)/2) h, (k-(nz-1)/2) h)."""
    nz, ny, nx = (int(s) for s in shape)
    h = float(spacing)
    cz = np.asarray(centre, np.float64)
    z = cz[2] + (np.arange(nz) - (nz - 1) / 2.0) * h
    rot0 = np.tile(np.eye(3).reshape(1, 9), (nz, 1)).astype(np.float32)
    trans0 = np.stack([np.full(nz, cz[0]), np.full(nz, cz[1]), z], axis=1).astype(np.float32)
    return Problem(np.zeros((0, 3), np.float32), np.zeros((0, 3), np.float32), np.zeros((0, 4), np.float32),
                   np.zeros(0, np.float32), np.array([0, 0], np.int64), np.zeros(nz, np.int32),
                   np.full(nz, ny, np.int32), np.full(nz, nx, np.int32), np.full((nz, 2), h, np.float32),
                   np.zeros((nz, 3), np.float32), rot0, trans0, np.zeros((nz, 6), np.float32),
                   np.ones(nz * ny * nx, np.float32), name="grid")


def voxel_centres(shape, spacing, centre=(0.0, 0.0, 0.0)):
    nz, ny, nx = (int(s) for s in shape)
    h = float(spacing)
    c = np.asarray(centre, np.float64)
    zz, yy, xx = np.meshgrid((np.arange(nz) - (nz - 1) / 2.0) * h + c[2], (np.arange(ny) - (ny - 1) / 2.0) * h + c[1],
                             (np.arange(nx) - (nx - 1) / 2.0) * h + c[0], indexing="ij")
    return np.stack([xx.ravel(), yy.ravel(), zz.ravel()], axis=1)


class VolumeProbe:
    """PSNR of the current Gaussians against a ground-truth volume on a grid.

    ``gt`` and ``mask`` are flat arrays over the grid (z-major, then rows,
    then columns).  ``cutoff`` is the footprint radius used for the read-out
    (the fitted model's own window by default).  ``model="topk"`` reads the
    volume out with the normalised Top-K model instead (K = ``topk_k``
    nearest means of every voxel inside the mask, rebuilt per read-out)."""

    def __init__(self, n_gauss, shape, spacing, centre, gt, mask, device=0, cutoff=3.0, tile=16, model="windowed",
                 topk_k=50, topk_delta=1e-6):
        import torch
        self.grid = volume_grid(shape, spacing, centre)
        g = self.grid
        self.geom = Problem(g.mean, g.log_scale, g.quat, g.amp, np.array([0, n_gauss], np.int64), g.slice_subject,
                            g.height, g.width, g.spacing, g.psf_fwhm, g.rot0, g.trans0, g.pose, g.mask)
        self.ctx = svr.Context(device)
        self.ctx.svr_set_config(tile=tile, batch=128, persistent=0, cutoff=cutoff, forward_mode=1)
        self.ctx.svr_set_geometry(self.geom)
        self.P = self.geom.n_pixels
        dev = torch.device("cuda", device)
        self.gt = torch.as_tensor(np.ascontiguousarray(gt, np.float32), device=dev)
        self.mask = torch.as_tensor(np.ascontiguousarray(mask, np.float32), device=dev)
        m = np.asarray(mask) > 0
        self.max_gt = float(np.asarray(gt)[m].max()) if m.any() else 1.0
        self.pose = torch.zeros((self.geom.n_slices, 6), dtype=torch.float32, device=dev)
        self.vol = torch.empty(self.P, dtype=torch.float32, device=dev)
        self.loss = torch.empty(1, dtype=torch.float32, device=dev)
        self.model, self.topk_k, self.topk_delta = model, topk_k, topk_delta
        self.n = int(n_gauss)
        if model == "topk":
            self.nbr = torch.empty(self.P, topk_k, dtype=torch.int32, device=dev)

    def _forward(self, mean, log_scale, quat, amp, with_loss):
        if mean.shape[0] != self.n:          # the mixture was densified since the last read-out
            self.n = int(mean.shape[0])
            self.geom.gauss_offsets = np.array([0, self.n], np.int64)
            self.ctx.svr_set_geometry(self.geom)
        tgt = (self.gt, self.mask) if with_loss else (None, None)
        if self.model == "topk":
            self.ctx.svr_topk_build(mean, self.pose, self.topk_k, self.nbr, mask=self.mask)
            self.ctx.svr_topk_forward(mean, log_scale, quat, amp, self.pose, self.nbr, self.topk_k, self.topk_delta,
                                      self.vol, *tgt, loss=self.loss if with_loss else None)
        else:
            self.ctx.svr_project_bin(mean, log_scale, quat, amp, self.pose)
            self.ctx.svr_forward(self.vol, *tgt, loss=self.loss if with_loss else None)

    def render(self, mean, log_scale, quat, amp):
        """The volume at the grid voxels (device tensor, flat)."""
        self._forward(mean, log_scale, quat, amp, False)
        return self.vol

    def psnr(self, mean, log_scale, quat, amp):
        self._forward(mean, log_scale, quat, amp, True)
        mse = float(self.loss.item())
        return 10.0 * math.log10(self.max_gt ** 2 / max(mse, 1e-30))

    def field(self, centres, width, beta, K):
        """The bias field b at the grid voxels (device tensor, flat); needs a
        read-out (render / psnr) first for the grid's frames."""
        import torch
        b = torch.ones_like(self.vol)
        self.ctx.svr_bias_apply(centres, width, beta, K, b)
        return b

    def psnr_biased(self, mean, log_scale, quat, amp, centres, width, beta, K):
        """PSNR of the volume times the bias field (what the slices see)."""
        self._forward(mean, log_scale, quat, amp, False)
        self.ctx.svr_bias_apply(centres, width, beta, K, self.vol)
        self.ctx.svr_slice_loss(self.vol, self.gt, self.mask, loss=self.loss)
        mse = float(self.loss.item())
        return 10.0 * math.log10(self.max_gt ** 2 / max(mse, 1e-30))

    def close(self):
        self.ctx.close()


@dataclass
class FitResult:
    times: list = field(default_factory=list)       # seconds of fitting (read-out excluded)
    iters: list = field(default_factory=list)
    psnr: list = field(default_factory=list)
    loss: list = field(default_factory=list)
    final_psnr: float = float("nan")
    seconds: float = 0.0


def fit(ctx, params, target, mask, n_iter, lr=PAPER_LR, probe=None, psnr_every=25, step_lr=200, gamma=0.5,
        psnr_target=None, callback=None, objective="mse", reg_lambda=2.5e-3, s_target=1.6, reg_reading="sum",
        outliers=False, outlier_lr=1e-3, model="windowed", topk_k=50, topk_refresh=50, topk_delta=1e-6,
        pose_start=0, densify=None, bias=None):
    """Runs n_iter fitting iterations of project_bin + forward + backward +
    AdamW on ``params`` (an svr.Params, updated in place).  The wall clock
    covers the iterations only; the PSNR read-out every ``psnr_every``
    iterations is timed out.  Stops early once ``psnr_target`` is reached.
    ``objective``: "mse" (masked mean squared error) or "l1+reg", the paper's
    Eq. 7 (masked L1 sum plus reg_lambda sum ||s - s_target||^2).
    ``reg_reading``: "sum" weighs the sums as written in Eq. 7; "mean" reads
    reg_lambda as weighting the mean L1 per masked pixel against the mean
    penalty per Gaussian, i.e. applies reg_lambda * sum(mask) / N to the sums.
    ``outliers`` adds the per-slice intensity scalar sigma_i and aleatoric
    weight omega_i = exp(rho_i) of Sec. 2.4 (svr_slice_loss), both learnt
    with AdamW at ``outlier_lr``; they are returned in the result as
    ``sigma`` and ``log_omega`` (host arrays).  ``model``: "windowed" (the
    exact-amplitude model with 3-sigma footprints) or "topk" (the paper's
    normalised Top-K model, Eqs. 2 and 5, with K = ``topk_k`` neighbour lists
    rebuilt every ``topk_refresh`` iterations for the masked pixels; the
    rebuilds are timed with the iterations).  The poses stay where they are
    for the first ``pose_start`` iterations (their rates are 0 there; the
    volume fits the slices first).

    ``densify`` (windowed model): dict(at=[iterations], fraction=f or
    grad_threshold=t, log_scale_threshold, split_offset, clone_offset,
    prune_amp, max_gauss).  Every step accumulates the mean-gradient
    statistic (svr_densify_accumulate); after the step of each listed
    iteration the mixture is densified (svr_densify) with the threshold t,
    or with the one that selects the fraction f of the Gaussians seen since
    the last densification with the largest mean gradient norm, unless the
    mixture already holds max_gauss; the Adam moments follow the new layout
    and the statistic restarts.  ``params`` then holds the new mixture.
    The sizes are recorded in ``res.n_gauss`` as (iteration, N).

    ``bias`` (windowed model): dict(centres [S, K, 3], width, beta [S*K]
    device tensors / floats, lr): the multiplicative bias field
    b = exp(sum_k beta_k phi_k) on the predicted pixels (svr_bias_apply),
    its coefficients learnt with AdamW at ``lr`` (updated in place in
    ``beta``), its pose terms added to the slices' pose gradients."""
    import torch
    if objective not in ("mse", "l1+reg"):
        raise ValueError(f"unknown objective {objective}")
    if reg_reading not in ("sum", "mean"):
        raise ValueError(f"unknown reg_reading {reg_reading}")
    if model not in ("windowed", "topk"):
        raise ValueError(f"unknown model {model}")
    if model == "topk" and (densify or bias):
        raise ValueError("densification and the bias field run with the windowed model")
    ctx.svr_set_loss(svr.SVR_LOSS_L1 if objective == "l1+reg" else svr.SVR_LOSS_MSE)
    N, M = params.N, params.M
    lam = reg_lambda * float(mask.sum().item()) / N if reg_reading == "mean" else reg_lambda
    grad = svr.Params(N, M, device=params.flat.device)
    m = torch.zeros_like(params.flat)
    v = torch.zeros_like(params.flat)
    P = ctx.n_pixels
    dev = params.flat.device
    pred = torch.empty(P, device=dev)
    gpred = torch.empty(P, device=dev)
    loss = torch.empty(1, device=dev)
    res = FitResult()
    elapsed = 0.0
    if model == "topk":
        nbr = torch.empty(P, topk_k, dtype=torch.int32, device=dev)
    if outliers:
        sig = torch.ones(M, device=dev)
        rho = torch.zeros(M, device=dev)
        g_sig = torch.empty(M, device=dev)
        g_rho = torch.empty(M, device=dev)
        st_o = [torch.zeros(M, device=dev) for _ in range(4)]
    if densify:
        d_at = set(int(x) for x in densify["at"])
        acc = torch.zeros(N, device=dev)
        cnt = torch.zeros(N, dtype=torch.int32, device=dev)
        res.n_gauss = [(0, N)]
        d_cfg = dict(log_scale_threshold=float(densify.get("log_scale_threshold", 0.0)),
                     split_offset=float(densify.get("split_offset", math.sqrt(3.0) / 2.0)),
                     clone_offset=float(densify.get("clone_offset", 0.5)),
                     prune_amp=float(densify.get("prune_amp", 0.0)))
    if bias:
        bK, bw, bc, beta = int(bias["K"]), float(bias["width"]), bias["centres"], bias["beta"]
        g_beta = torch.empty_like(beta)
        st_b = [torch.zeros_like(beta) for _ in range(2)]
        bvals = torch.empty(P, device=dev)
        b_pose = torch.zeros(M, 6, device=dev)
    sep_loss = outliers or bool(bias)
    torch.cuda.synchronize()
    for it in range(1, n_iter + 1):
        t0 = time.perf_counter()
        scale = gamma ** ((it - 1) // step_lr)
        pv = params.views()
        if model == "topk":
            if (it - 1) % topk_refresh == 0:
                ctx.svr_topk_build(pv[0], pv[4], topk_k, nbr, mask=mask)
            if outliers:
                ctx.svr_topk_forward(*pv, nbr, topk_k, topk_delta, pred)
            else:
                ctx.svr_topk_forward(*pv, nbr, topk_k, topk_delta, pred, target, mask, loss=loss, grad_pred=gpred)
        else:
            ctx.svr_project_bin(*pv)
            if sep_loss:
                ctx.svr_forward(pred)
            else:
                ctx.svr_forward(pred, target, mask, loss=loss, grad_pred=gpred)
        if bias:
            ctx.svr_bias_apply(bc, bw, beta, bK, pred, bvals)
        if sep_loss:
            ctx.svr_slice_loss(pred, target, mask, sig if outliers else None, rho if outliers else None, loss=loss,
                               grad_pred=gpred, g_sigma=g_sig if outliers else None,
                               g_log_omega=g_rho if outliers else None)
        if bias:
            b_pose.zero_()
            ctx.svr_bias_backward(bc, bw, beta, bK, pred, bvals, gpred, g_beta, b_pose)
        if model == "topk":
            ctx.svr_topk_backward(*pv, nbr, topk_k, gpred, *grad.views())
        else:
            ctx.svr_backward(gpred, *grad.views())
        if bias:
            grad.views()[4].add_(b_pose)
        if densify:
            ctx.svr_densify_accumulate(grad.views()[0], acc, cnt)
        if objective == "l1+reg":
            ctx.svr_scale_regularizer(params.views()[1], lam, s_target, grad.views()[1], loss)
        rates = [x * scale for x in lr]
        if it <= pose_start:
            rates[4] = rates[5] = 0.0
        ctx.svr_step(params.views(), grad.views(), m, v, rates, it)
        if outliers:
            ctx.svr_adam_vector(sig, g_sig, st_o[0], st_o[1], outlier_lr * scale, it)
            ctx.svr_adam_vector(rho, g_rho, st_o[2], st_o[3], outlier_lr * scale, it)
        if bias:
            ctx.svr_adam_vector(beta, g_beta, st_b[0], st_b[1], float(bias["lr"]) * scale, it)
        if densify and it in d_at and params.N < int(densify.get("max_gauss", 1 << 30)):
            cfg = dict(d_cfg)
            if "fraction" in densify:
                a_h, c_h = acc.cpu().numpy(), cnt.cpu().numpy()
                seen = c_h > 0
                mg = a_h[seen] / c_h[seen]
                k = int(round(float(densify["fraction"]) * len(mg)))
                k = min(k, int(densify.get("max_gauss", 1 << 30)) - params.N, len(mg))
                cfg["grad_threshold"] = float(np.sort(mg)[::-1][k - 1] * (1 - 1e-6)) if k > 0 else float("inf")
            else:
                cfg["grad_threshold"] = float(densify["grad_threshold"])
            if np.isfinite(cfg["grad_threshold"]):
                new, m, v, _ = ctx.densify_params(params, acc, cnt, cfg, m, v)
                params.N, params.flat = new.N, new.flat
                N = new.N
                grad = svr.Params(N, M, device=dev)
                acc = torch.zeros(N, device=dev)
                cnt = torch.zeros(N, dtype=torch.int32, device=dev)
                res.n_gauss.append((it, N))
        torch.cuda.synchronize()
        elapsed += time.perf_counter() - t0
        if probe is not None and (it % psnr_every == 0 or it == n_iter):
            p = probe.psnr(*params.views()[:4])
            res.times.append(elapsed)
            res.iters.append(it)
            res.psnr.append(p)
            res.loss.append(float(loss.item()))
            if callback:
                callback(it, elapsed, p, float(loss.item()))
            if psnr_target is not None and p >= psnr_target:
                break
    res.seconds = elapsed
    res.final_psnr = res.psnr[-1] if res.psnr else float("nan")
    if outliers:
        res.sigma = sig.cpu().numpy()
        res.log_omega = rho.cpu().numpy()
    return res


def adaptive_init(ctx, target, mask, n_gauss, n_slices, lambda_init=0.0, seed=0, scale=1.6, pose=None,
                  rescale=True):
    """Content-adaptive initialisation (Sec. 2.5, Eq. 6) for the context's
    geometry: means drawn by svr_init_means from the observed slices
    (lambda_init = 0 favours edges only, 1 is uniform over the mask),
    isotropic scales of ``scale`` mm (the target scale of Eq. 7), identity
    rotations, and amplitudes equal to the sampled intensities times the one
    factor that best fits (least squares over the mask) the slices rendered
    from them to the observed slices; that scalar is computed on the host
    from one rendered pass (skipped with ``rescale=False``, for the normalised
    model whose amplitudes are intensities).  Returns (svr.Params on the
    target's device, that factor)."""
    import torch
    from . import synth
    dev = target.device
    p = svr.Params(n_gauss, n_slices, device=dev)
    mean, log_scale, quat, amp, pz = p.views()
    if pose is not None:
        pz.copy_(pose)
    u = torch.as_tensor(synth.init_uniforms(seed, n_gauss), device=dev)
    ctx.svr_init_means(target, mask, pz, lambda_init, u, mean, None, amp)
    log_scale.fill_(math.log(scale))
    quat[:, 0] = 1.0
    if not rescale:
        return p, 1.0
    pred = torch.empty(ctx.n_pixels, dtype=torch.float32, device=dev)
    ctx.svr_project_bin(*p.views())
    ctx.svr_forward(pred)
    y = pred.cpu().numpy().astype(np.float64)
    t = target.cpu().numpy().astype(np.float64)
    m = mask.cpu().numpy().astype(np.float64)
    k = float((m * y * t).sum() / max((m * y * y).sum(), 1e-30))
    amp.mul_(k)
    return p, k


def time_to_target(res: FitResult, target):
    """First fitting time at which the PSNR reached ``target`` (inf if never)."""
    for t, p in zip(res.times, res.psnr):
        if p >= target:
            return t
    return float("inf")


def bias_basis(axes, kb, device=0):
    """kb^3 basis centres on a grid over the box [-axes, axes] (one subject,
    [1, kb^3, 3] device tensor) and their common width, the grid step
    averaged over the axes."""
    import torch
    ax = [np.linspace(-a, a, kb) for a in axes]
    g = np.stack(np.meshgrid(*ax, indexing="ij"), -1).reshape(1, -1, 3).astype(np.float32)
    width = float(np.mean([2 * a / max(kb - 1, 1) for a in axes]))
    return torch.as_tensor(g, device=torch.device("cuda", device)), width


class _BiasedProbe:
    """fit's read-out with the bias field applied (the beta tensor is read at
    every call, so it follows the fit)."""

    def __init__(self, probe, centres, width, beta, K):
        self.probe, self.args = probe, (centres, width, beta, K)

    def psnr(self, *params):
        return self.probe.psnr_biased(*params, *self.args)


def field_error(b_fit, b_true, mask, centred=False):
    """rms and max of |log b_fit - log b_true| over the mask (with the mean
    difference ``offset`` removed when ``centred``: a global factor trades
    against the amplitudes and against the window's lost mass), and the
    fraction of the true field's log-variance that the fitted field
    explains."""
    m = np.asarray(mask) > 0
    d = np.log(np.asarray(b_fit, np.float64)[m]) - np.log(np.asarray(b_true, np.float64)[m])
    lt = np.log(np.asarray(b_true, np.float64)[m])
    off = float(d.mean())
    if centred:
        d = d - off
    return dict(rms_log=float(np.sqrt(np.mean(d * d))), max_log=float(np.abs(d).max()), offset=off,
                true_rms_log=float(np.std(lt)), explained=float(1.0 - np.mean(d * d) / max(np.var(lt), 1e-30)))


# ---------------------------------------------------------------------------
# Fetal-scale convergence run: the head phantom fitted from its slices
# ---------------------------------------------------------------------------

def amplitude_lr(lr, kappa):
    """The paper's learning rates (App. A.1) with the amplitude rate scaled by
    kappa: its amplitudes are intensities (its mixture is normalised per
    point), while here an amplitude is an intensity times the density
    normalisation kappa of the unnormalised sum, so the same relative step
    needs a rate kappa times smaller."""
    out = list(lr)
    out[3] = lr[3] * kappa
    return tuple(out)


def head_convergence(n_iter=2000, psnr_every=50, seed=0, device=0, tile=16, log=None, scale_amp_lr=True,
                     known_poses=False, objective="mse", reg_lambda=2.5e-3, s_target=1.6, reg_reading="sum",
                     init="jitter", psf=True, corrupt=0.0, outliers=False, outlier_lr=1e-3, model="windowed",
                     pose_lr_scale=1.0, pose_start=0, observations="mixture", coarse=1, densify_at=(),
                     bias_grid=0, bias_lr=1e-2, motion=(4.0, 2.0)):
    """Fits the 500k-Gaussian head for ``n_iter`` iterations from identity
    poses, amplitudes reset to their mean and means jittered by 0.3 mm.
    ``observations="mixture"`` (the head workload's recipe): the slices are
    the forward model of the generating mixture at the true poses (the
    library's forward with a 6-sigma window) plus Rician noise at SNR 20,
    and PSNR is measured against the mixture's own volume; "phantom": the
    slices are simulated from the phantom itself (piecewise-constant tissue
    times the bias field, averaged across the slice thickness, Rician noise
    at SNR 20; neither the in-plane PSF nor the through-plane profile is the
    model's Gaussian), and PSNR is measured against the phantom.  Both on a
    0.5 mm grid over the head's bounding box, inside the head.  ``known_poses`` starts
    the poses at the truth and keeps them there (pose rates 0), separating
    the volume fit from motion correction.  ``objective``, ``reg_lambda``,
    ``s_target`` and ``reg_reading`` are passed to fit.  ``init``: "jitter"
    (the generating means moved by 0.3 mm, amplitudes at their mean),
    "adaptive" (Eq. 6 with lambda_init = 0, as in the paper) or "uniform"
    (lambda_init = 1), both from the observed slices via adaptive_init.
    ``psf=False`` fits with a zero PSF (the slices are still acquired with
    it), the paper's PSF ablation.  ``corrupt`` is the fraction of slices
    corrupted after acquisition (half of them with their intensity scaled
    by 1.5, half replaced by noise of the same mean); ``outliers`` fits the
    per-slice sigma_i and omega_i of Sec. 2.4 as well.  ``pose_lr_scale``
    scales the pose rates; ``pose_start`` holds the poses for that many
    iterations first (see fit).  ``model="topk"`` fits
    and reads out the paper's normalised Top-K model (K = 50, lists rebuilt
    every 50 iterations); its amplitudes are intensities, so they start at
    the sampled (or generating) intensities and use the paper's rates.
    ``coarse`` > 1 starts from N / coarse Gaussians with their scales times
    coarse^(1/3) (the same density normalisation, so the same amplitudes)
    and densifies after each iteration in ``densify_at`` (svr_densify; each
    time the fraction of Gaussians with the largest mean gradient that
    brings the mixture back to N in that many steps; Gaussians larger than
    1.5 h, h the generating spacing, split, the others clone).
    ``bias_grid`` = kb > 0 fits the multiplicative bias field on a kb^3 grid
    of basis Gaussians over the head's box along (rate ``bias_lr``); PSNR is
    then that of the volume times the field, and ``res.field`` holds the
    field's error against the phantom's bias inside the head (a global
    factor removed).  ``motion`` = (sd deg, sd mm) of the acquisition
    motion (the workload's N(0, 4 deg), N(0, 2 mm) by default).  Returns the FitResult, with the
    PSNR of the generating mixture itself (the representation's ceiling
    against the phantom) in ``gt_psnr``."""
    import torch
    from . import synth
    prob = synth.config2(seed, sd_deg=float(motion[0]), sd_mm=float(motion[1]))
    axes = prob.extra["axes"]
    if observations not in ("mixture", "phantom"):
        raise ValueError(f"unknown observations {observations}")
    if observations == "phantom":
        target = synth.head_observation(prob, seed + 1)
    else:
        ref = svr.Context(device)
        ref.svr_set_config(tile=tile, batch=128, persistent=0, cutoff=6.0, forward_mode=1)
        ref.svr_set_geometry(prob)
        clean = torch.empty(prob.n_pixels, device=torch.device("cuda", device))
        ref.svr_project_bin(*svr.Params.from_arrays(*prob.params(), prob.pose).views())
        ref.svr_forward(clean)
        c_np = clean.cpu().numpy()
        ref.close()
        target = synth.rician(c_np, seed + 1, float(c_np[prob.mask > 0].mean()) / 20.0)
    bad = np.zeros(0, np.int64)
    if corrupt > 0:
        rng_c = np.random.default_rng(seed + 3)
        bad = np.sort(rng_c.choice(prob.n_slices, max(1, int(round(corrupt * prob.n_slices))), replace=False))
        po = prob.pix_offset
        for k, i in enumerate(bad):
            sl = slice(po[i], po[i + 1])
            if k % 2 == 0:
                target[sl] *= 1.5
            else:
                target[sl] = rng_c.uniform(0.0, 2.0 * float(target[sl].mean()), po[i + 1] - po[i]).astype(np.float32)
    h = 0.5
    shape = tuple(int(2 * a / h) for a in axes[::-1])   # (nz, ny, nx)
    c = voxel_centres(shape, h)
    vmask = (np.linalg.norm(c / axes[None, :], axis=1) <= 1.0).astype(np.float32)
    if observations == "phantom":
        gt = synth.head_intensity(c, axes) * synth.head_bias(c, prob.extra["bias"], axes)
    else:
        gp = VolumeProbe(prob.n_gauss, shape, h, (0, 0, 0), np.zeros(len(c), np.float32), vmask, device=device,
                         tile=tile, cutoff=6.0)
        gt = gp.render(*[torch.as_tensor(a, device=torch.device("cuda", device)) for a in prob.params()]).cpu().numpy()
        gp.close()
    probe = VolumeProbe(prob.n_gauss, shape, h, (0, 0, 0), gt, vmask, device=device, tile=tile, model=model)
    ctx = svr.Context(device)
    if init not in ("jitter", "adaptive", "uniform"):
        raise ValueError(f"unknown init {init}")
    ctx.svr_set_config(tile=tile, batch=128, persistent=0, cutoff=3.0, forward_mode=1)
    import copy
    n0 = prob.n_gauss // max(int(coarse), 1)
    fit_geom = copy.copy(prob)
    fit_geom.gauss_offsets = np.array([0, n0], np.int64)
    if not psf:
        fit_geom.psf_fwhm = np.zeros_like(prob.psf_fwhm)
    ctx.svr_set_geometry(fit_geom)
    dev = torch.device("cuda", device)
    pose0 = prob.pose if known_poses else np.zeros((prob.n_slices, 6), np.float32)
    topk = model == "topk"
    # intensity at the generating means; the windowed model's amplitude is
    # intensity x kappa, the normalised model's is the intensity itself
    inten = (synth.head_intensity(prob.mean.astype(np.float64), axes) *
             synth.head_bias(prob.mean.astype(np.float64), prob.extra["bias"], axes)).astype(np.float32)
    if init == "jitter":
        rng = np.random.default_rng(seed + 2)
        mean = prob.mean + rng.normal(0.0, 0.3, prob.mean.shape).astype(np.float32)
        amp = np.full_like(prob.amp, inten.mean() if topk else prob.amp.mean())
        grow = np.float32(math.log(prob.n_gauss / n0) / 3.0)
        params = svr.Params.from_arrays(mean[:n0], prob.log_scale[:n0] + grow, prob.quat[:n0], amp[:n0], pose0)
    else:
        params, kappa_init = adaptive_init(ctx, torch.as_tensor(target, device=dev),
                                           torch.as_tensor(prob.mask, device=dev), n0, prob.n_slices,
                                           0.0 if init == "adaptive" else 1.0, seed + 2,
                                           s_target * (prob.n_gauss / n0) ** (1.0 / 3.0),
                                           torch.as_tensor(pose0, device=dev), rescale=not topk)
    if topk:
        kappa = 1.0
    else:
        kappa = float(np.median(prob.amp / np.maximum(inten, 1e-6))) if init == "jitter" else kappa_init
    lr = amplitude_lr(PAPER_LR, kappa) if scale_amp_lr else PAPER_LR
    if known_poses:
        lr = lr[:4] + (0.0, 0.0)
    else:
        lr = tuple(lr[:4]) + (lr[4] * pose_lr_scale, lr[5] * pose_lr_scale)
    gt = svr.Params.from_arrays(prob.mean, prob.log_scale, prob.quat, inten if topk else prob.amp, prob.pose)
    gt_psnr = probe.psnr(*gt.views()[:4])
    del gt
    p0 = probe.psnr(*params.views()[:4])
    if log:
        log(f"head: N={prob.n_gauss} M={prob.n_slices} P={prob.n_pixels} grid={shape}; initial PSNR {p0:.2f} dB, "
            f"generating mixture {gt_psnr:.2f} dB")
    if log:
        log(f"learning rates {lr} (amplitude scale kappa = {kappa:.4g})")
    densify = None
    if n0 < prob.n_gauss and len(densify_at):
        g = (prob.n_gauss / n0) ** (1.0 / len(densify_at))
        densify = dict(at=list(densify_at), fraction=min(g - 1.0, 1.0), max_gauss=prob.n_gauss,
                       log_scale_threshold=math.log(1.5 * prob.extra["h"]))
    bias = None
    fit_probe = probe
    if bias_grid:
        bc, bw = bias_basis(axes, int(bias_grid), device)
        bias = dict(centres=bc, width=bw, K=int(bias_grid) ** 3, lr=bias_lr,
                    beta=torch.zeros(int(bias_grid) ** 3, device=dev))
        fit_probe = _BiasedProbe(probe, bc, bw, bias["beta"], bias["K"])
    res = fit(ctx, params, torch.as_tensor(target, device=dev), torch.as_tensor(prob.mask, device=dev), n_iter,
              lr=lr, probe=fit_probe, psnr_every=psnr_every, objective=objective, reg_lambda=reg_lambda,
              s_target=s_target, reg_reading=reg_reading, outliers=outliers, outlier_lr=outlier_lr, model=model,
              callback=(lambda it, t, p, l: log(f"iter {it}: {t:.2f} s, PSNR {p:.2f} dB, loss {l:.5g}"
                                                f"{'' if not densify else f', N {params.N}'}")) if log else None,
              pose_start=pose_start, densify=densify, bias=bias)
    if bias:
        probe.render(*params.views()[:4])
        b_fit = probe.field(bias["centres"], bias["width"], bias["beta"], bias["K"]).cpu().numpy()
        b_true = synth.head_bias(c, prob.extra["bias"], axes)
        res.field = field_error(b_fit, b_true, vmask, centred=True)
        res.plain_psnr = probe.psnr(*params.views()[:4])
    true_pose = prob.pose.astype(np.float64)
    est = params.views()[4].cpu().numpy().astype(np.float64)
    po = prob.pix_offset
    seen = np.array([prob.mask[po[i]:po[i + 1]].mean() >= 0.05 for i in range(prob.n_slices)])
    res.initial_psnr = p0
    res.gt_psnr = gt_psnr
    res.corrupted = bad.tolist()
    res.pose_err = dict(rot_deg_identity=float(np.degrees(np.abs(true_pose[:, :3]).mean())),
                        rot_deg_fitted=float(np.degrees(np.abs(est[:, :3] - true_pose[:, :3]).mean())),
                        trans_mm_identity=float(np.abs(true_pose[:, 3:]).mean()),
                        trans_mm_fitted=float(np.abs(est[:, 3:] - true_pose[:, 3:]).mean()),
                        seen_slices=int(seen.sum()),
                        seen_rot_deg_identity=float(np.degrees(np.abs(true_pose[seen, :3]).mean())),
                        seen_rot_deg_fitted=float(np.degrees(np.abs(est[seen, :3] - true_pose[seen, :3]).mean())),
                        seen_trans_mm_identity=float(np.abs(true_pose[seen, 3:]).mean()),
                        seen_trans_mm_fitted=float(np.abs(est[seen, 3:] - true_pose[seen, 3:]).mean()))
    probe.close()
    ctx.close()
    return res


class _NoProbe:
    """A stand-in read-out for fit: its callback then fires every psnr_every
    iterations without rendering a volume."""

    def psnr(self, *params):
        return 0.0


def pose_recovery(n_iter=400, observations="mixture", seed=0, device=0, tile=32, every=25, log=None, lr=None):
    """Motion correction alone on the head workload: the Gaussians are held at
    the generating mixture (their rates are 0) and only the 128 slice poses
    are fitted, from identity, by the same iteration as fit (masked MSE,
    AdamW at the paper's pose rates, StepLR).  ``observations``: "mixture",
    the library's forward of the generating mixture at the true poses plus
    Rician noise at SNR 20 (the model can then explain the slices exactly,
    so the fit should find the true poses up to noise), or "phantom", the
    phantom's own slices (synth.head_observation), which the mixture
    approximates only (16 dB against the phantom).  Returns a list of
    (iteration, seconds, mean |rotation error| deg, mean |translation error|
    mm, max rotation error deg, max translation error mm) over the slices
    that see the head (at least 5 % of their pixels inside the mask; the
    others carry no information about their pose), and the final per-slice
    errors and mask fractions."""
    import torch
    from . import synth
    prob = synth.config2(seed)
    dev = torch.device("cuda", device)
    ctx = svr.Context(device)
    ctx.svr_set_config(tile=tile, batch=128, persistent=0, cutoff=3.0, forward_mode=1)
    ctx.svr_set_geometry(prob)
    mask = torch.as_tensor(prob.mask, device=dev)
    if observations == "mixture":
        gt = svr.Params.from_arrays(*prob.params(), prob.pose)
        ctx.svr_project_bin(*gt.views())
        clean = torch.empty(prob.n_pixels, device=dev)
        ctx.svr_forward(clean)
        c = clean.cpu().numpy()
        sigma = float(c[prob.mask > 0].mean()) / 20.0
        target = synth.rician(c, seed + 1, sigma)
        del gt
    elif observations == "phantom":
        target = synth.head_observation(prob, seed + 1)
    else:
        raise ValueError(f"unknown observations {observations}")
    params = svr.Params.from_arrays(*prob.params(), np.zeros((prob.n_slices, 6), np.float32))
    base = lr or PAPER_LR
    rates = (0.0, 0.0, 0.0, 0.0, base[4], base[5])
    true_pose = prob.pose.astype(np.float64)
    po = prob.pix_offset
    frac = np.array([prob.mask[po[i]:po[i + 1]].mean() for i in range(prob.n_slices)])
    seen = frac >= 0.05
    rows = []

    def err(it, t):
        est = params.views()[4].cpu().numpy().astype(np.float64)
        d = np.abs(est - true_pose)[seen]
        rows.append((it, t, float(np.degrees(d[:, :3].mean())), float(d[:, 3:].mean()),
                     float(np.degrees(d[:, :3].max())), float(d[:, 3:].max())))
        if log:
            log(f"iter {it}: rotation {rows[-1][2]:.4f} deg (max {rows[-1][4]:.3f}), translation {rows[-1][3]:.4f} mm "
                f"(max {rows[-1][5]:.3f})")

    err(0, 0.0)
    fit(ctx, params, torch.as_tensor(target, device=dev), mask, n_iter, lr=rates, probe=_NoProbe(), psnr_every=every,
        callback=lambda it, t, p, l: err(it, t))
    final = np.abs(params.views()[4].cpu().numpy().astype(np.float64) - true_pose)
    ctx.close()
    return rows, dict(rot_deg=np.degrees(final[:, :3]).tolist(), trans_mm=final[:, 3:].tolist(), mask_frac=frac.tolist(),
                      seen=int(seen.sum()))


def bias_recovery(n_iter=400, observations="mixture", kb=4, lr=1e-2, seed=0, device=0, tile=32, every=25,
                  log=None, cutoff=None):
    """The bias field alone on the head workload: the Gaussians are held at
    the tissue-only mixture (the generating amplitudes divided by the
    phantom's bias at their means) and the poses at the truth; only the
    field's kb^3 coefficients are fitted, from 0 (b = 1), by fit's
    iteration (masked MSE, AdamW at ``lr``, StepLR).  ``observations``:
    "mixture", the library's forward of the tissue-only mixture at the true
    poses (6-sigma window) times the phantom's bias at every pixel centre,
    Rician noise at SNR 20 (the field model can explain that up to its
    basis), or "phantom", the phantom's own slices (synth.head_observation).
    The fit's window is ``cutoff`` (default: the generating 6 sigma for
    mixture observations, so that the model matches them exactly, else the
    fitted model's 3 sigma).  Returns rows (iteration, seconds, rms
    |log b - log b_true| with the mean difference removed, its max, the
    mean difference (a global factor), the fraction of the true log-field
    variance explained) over the voxels of the 0.5 mm grid inside the head,
    and the final error dict."""
    import torch
    from . import synth
    prob = synth.config2(seed)
    axes, bp = prob.extra["axes"], prob.extra["bias"]
    dev = torch.device("cuda", device)
    tissue = (prob.amp / synth.head_bias(prob.mean.astype(np.float64), bp, axes)).astype(np.float32)
    ctx = svr.Context(device)
    ctx.svr_set_geometry(prob)
    if observations == "mixture":
        ctx.svr_set_config(tile=tile, batch=128, persistent=0, cutoff=6.0, forward_mode=1)
        tp = svr.Params.from_arrays(prob.mean, prob.log_scale, prob.quat, tissue, prob.pose)
        ctx.svr_project_bin(*tp.views())
        clean = torch.empty(prob.n_pixels, device=dev)
        ctx.svr_forward(clean)
        bpix = np.concatenate([synth.head_bias(x, bp, axes) for x in synth.pixel_world_positions(
            prob.rot0, prob.trans0, prob.pose, prob.height, prob.width, prob.spacing)])
        c = clean.cpu().numpy() * bpix
        target = synth.rician(c, seed + 1, float(c[prob.mask > 0].mean()) / 20.0)
        del tp
    elif observations == "phantom":
        target = synth.head_observation(prob, seed + 1)
    else:
        raise ValueError(f"unknown observations {observations}")
    cut = (6.0 if observations == "mixture" else 3.0) if cutoff is None else float(cutoff)
    ctx.svr_set_config(tile=tile, batch=128, persistent=0, cutoff=cut, forward_mode=1)
    params = svr.Params.from_arrays(prob.mean, prob.log_scale, prob.quat, tissue, prob.pose)
    h = 0.5
    shape = tuple(int(2 * a / h) for a in axes[::-1])
    vc = voxel_centres(shape, h)
    vmask = (np.linalg.norm(vc / axes[None, :], axis=1) <= 1.0).astype(np.float32)
    b_true = synth.head_bias(vc, bp, axes)
    probe = VolumeProbe(prob.n_gauss, shape, h, (0, 0, 0), np.zeros(len(vc), np.float32), vmask, device=device,
                        tile=tile)
    probe.render(*params.views()[:4])
    bc, bw = bias_basis(axes, kb, device)
    K = kb ** 3
    beta = torch.zeros(K, device=dev)
    rows = []

    def err(it, t):
        e = field_error(probe.field(bc, bw, beta, K).cpu().numpy(), b_true, vmask, centred=True)
        rows.append((it, t, e["rms_log"], e["max_log"], e["offset"], e["explained"]))
        if log:
            log(f"iter {it}: rms |log b - log b_true| {e['rms_log']:.4f} (max {e['max_log']:.3f}, mean offset "
                f"{e['offset']:+.4f}), explained {e['explained']:.4f} of the true log-variance "
                f"{e['true_rms_log'] ** 2:.3e}")

    err(0, 0.0)
    fit(ctx, params, torch.as_tensor(target, device=dev), torch.as_tensor(prob.mask, device=dev), n_iter,
        lr=(0.0,) * 6, probe=_NoProbe(), psnr_every=every, callback=lambda it, t, p, l: err(it, t),
        bias=dict(centres=bc, width=bw, K=K, beta=beta, lr=lr))
    final = field_error(probe.field(bc, bw, beta, K).cpu().numpy(), b_true, vmask, centred=True)
    probe.close()
    ctx.close()
    return rows, final


def main(argv=None):
    import argparse
    import json
    ap = argparse.ArgumentParser(description="Head-phantom convergence run (PSNR against the phantom).")
    ap.add_argument("--iters", type=int, default=2000)
    ap.add_argument("--psnr-every", type=int, default=50)
    ap.add_argument("--paper-amp-lr", action="store_true", help="use the paper's amplitude rate unscaled")
    ap.add_argument("--known-poses", action="store_true", help="poses fixed at the truth")
    ap.add_argument("--objective", choices=("mse", "l1+reg"), default="mse")
    ap.add_argument("--reg-lambda", type=float, default=2.5e-3)
    ap.add_argument("--s-target", type=float, default=1.6)
    ap.add_argument("--reg-reading", choices=("sum", "mean"), default="sum")
    ap.add_argument("--init", choices=("jitter", "adaptive", "uniform"), default="jitter")
    ap.add_argument("--no-psf", action="store_true", help="fit with a zero PSF")
    ap.add_argument("--corrupt", type=float, default=0.0, help="fraction of corrupted slices")
    ap.add_argument("--outliers", action="store_true", help="fit the per-slice sigma_i and omega_i")
    ap.add_argument("--outlier-lr", type=float, default=1e-3, help="AdamW rate of sigma_i and log omega_i")
    ap.add_argument("--model", choices=("windowed", "topk"), default="windowed",
                    help="windowed: exact amplitude, 3-sigma footprints; topk: the paper's normalised Top-K model")
    ap.add_argument("--pose-lr-scale", type=float, default=1.0, help="factor on the paper's pose rates")
    ap.add_argument("--pose-start", type=int, default=0, help="iterations with the poses held first")
    ap.add_argument("--coarse", type=int, default=1, help="start from N / coarse Gaussians and densify")
    ap.add_argument("--densify-at", default="", help="comma-separated iterations after which to densify")
    ap.add_argument("--bias-grid", type=int, default=0, help="fit a bias field on a kb^3 basis grid (0: none)")
    ap.add_argument("--bias-lr", type=float, default=1e-2, help="AdamW rate of the bias coefficients")
    ap.add_argument("--motion", default="4,2", help="sd of the acquisition motion: degrees,mm")
    ap.add_argument("--observations", choices=("mixture", "phantom"), default="mixture",
                    help="mixture: the forward model of the generating mixture (PSNR against its volume); "
                         "phantom: slices of the phantom itself (PSNR against the phantom)")
    a = ap.parse_args(argv)
    res = head_convergence(a.iters, a.psnr_every, log=lambda s: print(s, flush=True),
                           scale_amp_lr=not a.paper_amp_lr, known_poses=a.known_poses, objective=a.objective,
                           reg_lambda=a.reg_lambda, s_target=a.s_target, reg_reading=a.reg_reading,
                           init=a.init, psf=not a.no_psf, corrupt=a.corrupt, outliers=a.outliers,
                           outlier_lr=a.outlier_lr, model=a.model, pose_lr_scale=a.pose_lr_scale,
                           pose_start=a.pose_start, observations=a.observations, coarse=a.coarse,
                           densify_at=[int(x) for x in a.densify_at.split(",") if x], bias_grid=a.bias_grid,
                           bias_lr=a.bias_lr, motion=[float(x) for x in a.motion.split(",")])
    extra = {}
    if a.coarse > 1:
        extra["n_gauss"] = getattr(res, "n_gauss", None)
    if a.bias_grid:
        extra.update(bias_grid=a.bias_grid, bias_lr=a.bias_lr, field=res.field, psnr_without_field=res.plain_psnr)
    if a.outliers:
        bad = np.asarray(res.corrupted, np.int64)
        clean = np.setdiff1d(np.arange(len(res.sigma)), bad)
        # the loss uses the centred values (one subject here)
        om = np.exp(res.log_omega - res.log_omega.mean())
        res.sigma = res.sigma / np.exp(np.log(res.sigma).mean())
        extra.update(omega_clean=float(om[clean].mean()), omega_scaled=float(om[bad[0::2]].mean()) if len(bad) else None,
                     omega_noise=float(om[bad[1::2]].mean()) if len(bad) > 1 else None,
                     sigma_clean=float(res.sigma[clean].mean()),
                     sigma_scaled=float(res.sigma[bad[0::2]].mean()) if len(bad) else None)
    print(json.dumps(dict(run="head convergence", iters=res.iters[-1] if res.iters else 0, **extra,
                          known_poses=a.known_poses, objective=a.objective, reg_lambda=a.reg_lambda,
                          reg_reading=a.reg_reading, init=a.init, psf=not a.no_psf, corrupt=a.corrupt,
                          outliers=a.outliers, outlier_lr=a.outlier_lr, model=a.model, observations=a.observations,
                          pose_lr_scale=a.pose_lr_scale, coarse=a.coarse, motion=a.motion,
                          pose_start=a.pose_start, fit_seconds=res.seconds, initial_psnr=res.initial_psnr,
                          generating_mixture_psnr=res.gt_psnr, final_psnr=res.final_psnr,
                          best_psnr=max(res.psnr) if res.psnr else None, pose_err=res.pose_err,
                          curve=[[i, round(t, 3), round(p, 3)] for i, t, p in zip(res.iters, res.times, res.psnr)])),
          flush=True)


if __name__ == "__main__":
    main()
