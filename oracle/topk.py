"""Normalised Top-K forward model of Eqs. 2 and 5 (Sec. 2.2-2.5), FP64 on the
CPU with plain PyTorch ops; gradients by autograd.

TEST INFRASTRUCTURE ONLY: the HIP path never imports it.

For pixel p of slice i at world position x = R_i u_p + t_i (Sec. 2.4, the
same pixel embedding as the windowed model):
    y_p = sigma_i * sum_{j in S^K(x)} c_j e_j / (sum_{j in S^K(x)} e_j + delta)
    e_j = exp(-1/2 v^T Sigma_obs^-1 v),  v = x - mu_j,
    Sigma_obs = Sigma_j + R_i Sigma_PSF R_i^T                       (Eq. 4)
with S^K(x) the K means of the slice's subject nearest to x in L2 (Sec. 2.5,
Top-K), Sigma_j = R(q_j) diag(s_j^2) R(q_j)^T, s = exp(log_scale),
Sigma_PSF = diag((FWHM / 2.355)^2) in the slice frame, and sigma_i the
slice's intensity scalar of Sec. 2.4 (1 when not given).  Eq. 5 carries no
sqrt(det) factor and is read as printed.

The neighbour lists are an input of the forward (the paper refreshes its
neighbour index only every 50 epochs); ``knn`` computes them from the means
and poses.
"""
from __future__ import annotations

import numpy as np
import torch
from scipy.spatial import cKDTree

DT = torch.float64


def _t(a):
    return torch.as_tensor(np.asarray(a, np.float64), dtype=DT)


def rotvec_matrix(w):
    """Exp of rotation vectors w [M,3] (Rodrigues), differentiable; the
    small-angle branch uses the series to second order."""
    th2 = (w * w).sum(-1, keepdim=True)
    th = torch.sqrt(torch.clamp(th2, min=1e-300))
    small = th2 < 1e-12
    a = torch.where(small, 1.0 - th2 / 6.0, torch.sin(th) / torch.where(small, torch.ones_like(th), th))
    b = torch.where(small, 0.5 - th2 / 24.0, (1.0 - torch.cos(th)) / torch.where(small, torch.ones_like(th2), th2))
    z = torch.zeros_like(w[:, 0])
    K = torch.stack([torch.stack([z, -w[:, 2], w[:, 1]], -1),
                     torch.stack([w[:, 2], z, -w[:, 0]], -1),
                     torch.stack([-w[:, 1], w[:, 0], z], -1)], -2)
    eye = torch.eye(3, dtype=w.dtype).expand_as(K)
    return eye + a[..., None] * K + b[..., None] * (K @ K)


def quat_matrix(q):
    """Rotation of quaternions q [N,4] = (w, x, y, z), normalised on use."""
    q = q / torch.linalg.norm(q, dim=-1, keepdim=True)
    w, x, y, z = q.unbind(-1)
    return torch.stack([
        torch.stack([1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)], -1),
        torch.stack([2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)], -1),
        torch.stack([2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)], -1)], -2)


def slice_frames(prob, pose):
    """(R [M,3,3], t [M,3]) of every slice under ``pose`` (torch, differentiable)."""
    R = rotvec_matrix(pose[:, :3]) @ _t(prob.rot0).reshape(-1, 3, 3)
    t = _t(prob.trans0) + pose[:, 3:]
    return R, t


def pixel_slices(prob, pixels=None):
    """Slice index and in-slice offset u (FP64, z = 0) of every pixel (or of
    the global pixel ids ``pixels``)."""
    po = np.asarray(prob.pix_offset)
    pid = np.arange(po[-1]) if pixels is None else np.asarray(pixels, np.int64)
    sl = np.searchsorted(po, pid, side="right") - 1
    loc = pid - po[sl]
    W = np.asarray(prob.width, np.int64)[sl]
    H = np.asarray(prob.height, np.int64)[sl]
    r, k = loc // W, loc % W
    sp = np.asarray(prob.spacing, np.float64)[sl]
    u = np.stack([(k - (W - 1) / 2.0) * sp[:, 0], (r - (H - 1) / 2.0) * sp[:, 1], np.zeros(len(sl))], 1)
    return sl, u


def pixel_positions(prob, pose, pixels=None):
    """World position x [P,3] of every pixel centre (torch FP64)."""
    R, t = slice_frames(prob, pose)
    sl, u = pixel_slices(prob, pixels)
    sl = torch.as_tensor(sl)
    return (R[sl] @ _t(u)[..., None])[..., 0] + t[sl]


def knn(prob, mean, pose, K, pixels=None):
    """For every pixel (or the pixel ids ``pixels``), the K means of its
    subject nearest to it (ascending distance; int64 [P,K] global Gaussian
    ids) and the squared distances of the K+1 nearest [P,K+1] (inf where the
    subject has only K), by a k-d tree query per subject."""
    x = pixel_positions(prob, _t(pose), pixels).numpy()
    mean = np.asarray(mean, np.float64)
    go = np.asarray(prob.gauss_offsets)
    sl, _ = pixel_slices(prob, pixels)
    subj = np.asarray(prob.slice_subject)[sl]
    idx = np.zeros((len(x), K), np.int64)
    d2 = np.full((len(x), K + 1), np.inf)
    for s in range(len(go) - 1):
        a, b = int(go[s]), int(go[s + 1])
        rows = np.nonzero(subj == s)[0]
        if len(rows) == 0:
            continue
        if b - a < K:
            raise ValueError(f"subject {s} has fewer than K = {K} Gaussians")
        kk = min(K + 1, b - a)
        d, j = cKDTree(mean[a:b]).query(x[rows], k=kk)
        d = d.reshape(len(rows), kk)
        j = j.reshape(len(rows), kk)
        idx[rows] = a + j[:, :K]
        d2[rows, :kk] = d * d
    return idx, d2


def gaussian_covariances(log_scale, quat):
    R = quat_matrix(quat)
    s2 = torch.exp(2.0 * log_scale)
    return R @ (s2[..., None] * R.transpose(-1, -2))


def psf_covariances(prob, R):
    """R_i Sigma_PSF R_i^T per slice."""
    sig = _t(prob.psf_fwhm) / 2.355
    return R @ (sig[..., None] ** 2 * R.transpose(-1, -2))


def forward(prob, mean, log_scale, quat, amp, pose, nbr, delta, sigma=None, pixels=None):
    """(y [P], numerator [P], denominator sum e [P]) as torch FP64 tensors
    (rows of ``pixels`` only, if given; ``nbr`` then has their rows); the
    parameter arguments may be tensors that require grad."""
    R, t = slice_frames(prob, pose)
    sl, u = pixel_slices(prob, pixels)
    sl_t = torch.as_tensor(sl)
    x = (R[sl_t] @ _t(u)[..., None])[..., 0] + t[sl_t]              # [P,3]
    Sg = gaussian_covariances(log_scale, quat)                      # [N,3,3]
    Sp = psf_covariances(prob, R)                                   # [M,3,3]
    nbr = torch.as_tensor(np.asarray(nbr, np.int64))
    v = x[:, None, :] - mean[nbr]                                   # [P,K,3]
    Sobs = Sg[nbr] + Sp[sl_t][:, None]                               # [P,K,3,3]
    w = torch.linalg.solve(Sobs, v[..., None])[..., 0]
    e = torch.exp(-0.5 * (v * w).sum(-1))                            # [P,K]
    num = (amp[nbr] * e).sum(-1)
    den = e.sum(-1)
    y = num / (den + delta)
    if sigma is not None:
        y = sigma[sl_t] * y
    return y, num, den


def forward_np(prob, params, pose, nbr, delta, sigma=None, pixels=None):
    mean, ls, q, c = params
    with torch.no_grad():
        y, n, d = forward(prob, _t(mean), _t(ls), _t(q), _t(c), _t(pose), nbr, delta,
                          None if sigma is None else _t(sigma), pixels)
    return y.numpy(), n.numpy(), d.numpy()


def gradients(prob, params, pose, nbr, delta, grad_y, sigma=None, pixels=None):
    """Gradients of sum(grad_y * y) (over ``pixels`` if given) with respect to
    mean, log_scale, quat, amp, pose and (if given) sigma, by autograd in
    FP64."""
    ts = [_t(a).requires_grad_(True) for a in (*params, pose)]
    sg = None if sigma is None else _t(sigma).requires_grad_(True)
    y, _, _ = forward(prob, *ts, nbr, delta, sg, pixels)
    (y * _t(grad_y)).sum().backward()
    out = [a.grad.numpy() for a in ts]
    if sg is not None:
        out.append(sg.grad.numpy())
    return out
