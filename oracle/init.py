"""Content-adaptive initialisation of the Gaussian means (Sec. 2.5, Eq. 6),
FP64 NumPy, written from the paper.

TEST INFRASTRUCTURE ONLY: the HIP path never imports it.

Eq. 6 draws the means from a density over the slices' pixels proportional to
(1 - lambda_init) ||grad I_i(u)|| + lambda_init.  Readings where the paper is
silent:

* grad I is taken within each slice, in intensity per mm: central
  differences (I[k+1] - I[k-1]) / (2 dx) inside, one-sided differences on the
  border, 0 along an axis of length 1;
* ||grad I|| is divided by its largest value over the subject's masked pixels
  (mask > 0), so that both terms of Eq. 6 are dimensionless; masked-out
  pixels get weight 0; a subject whose masked gradients are all 0 uses the
  uniform term alone;
* the weight is quantised to w = floor(2^20 p), so that the discrete draw is
  an exact integer decision: with the subject's total W and a uniform u0 in
  [0, 1), t = min(floor(u0 W), W - 1) and the draw is the first pixel whose
  inclusive cumulative weight exceeds t;
* the mean is the pixel centre plus a uniform offset within the pixel,
  ((u1 - 1/2) dx, (u2 - 1/2) dy), and within the slice thickness,
  (u3 - 1/2) times the through-plane PSF FWHM, mapped to the world by the
  slice pose R = Exp(omega) R0, t = t0 + tau (Sec. 2.4);
* each subject's Gaussians are drawn from that subject's slices only.

The uniforms u [N, 4] are inputs, so the draw is a deterministic function of
them.  Arithmetic order of the weights (so that the integer decision is
reproducible): g = sqrt(gx*gx + gy*gy) with gx = (I[k+1] - I[k-1]) * (0.5/dx)
(one-sided: (I[1] - I[0]) * (1/dx)), p = (1 - lambda) * (g / gmax) + lambda,
each operation rounded once in FP64.
"""
from __future__ import annotations

import numpy as np
from scipy.spatial.transform import Rotation

QUANT = 2.0 ** 20


def _axis_gradient(img, step, axis):
    """Central / one-sided difference along ``axis`` of a 2-D slice, per mm."""
    n = img.shape[axis]
    out = np.zeros_like(img)
    if n < 2:
        return out
    a = np.moveaxis(img, axis, 0)
    o = np.moveaxis(out, axis, 0)
    o[1:-1] = (a[2:] - a[:-2]) * (0.5 / step)
    o[0] = (a[1] - a[0]) * (1.0 / step)
    o[-1] = (a[-1] - a[-2]) * (1.0 / step)
    return out


def gradient_magnitude(image, height, width, spacing, pix_offset):
    """||grad I|| per pixel [P] (FP64), slice by slice."""
    image = np.asarray(image, np.float64)
    g = np.zeros(int(pix_offset[-1]), np.float64)
    for i in range(len(height)):
        H, W = int(height[i]), int(width[i])
        dx, dy = float(spacing[i][0]), float(spacing[i][1])
        img = image[pix_offset[i]:pix_offset[i + 1]].reshape(H, W)
        gx = _axis_gradient(img, dx, 1)
        gy = _axis_gradient(img, dy, 0)
        g[pix_offset[i]:pix_offset[i + 1]] = np.sqrt(gx * gx + gy * gy).ravel()
    return g


def _subject_pixels(prob):
    """[(first pixel, end pixel)] of each subject."""
    po = np.asarray(prob.pix_offset)
    subj = np.asarray(prob.slice_subject)
    out = []
    for s in range(prob.n_subjects):
        idx = np.nonzero(subj == s)[0]
        out.append((int(po[idx[0]]), int(po[idx[-1] + 1])))
    return out


def sampling_weights(prob, image, lam):
    """Quantised Eq. 6 weights w [P] (int64)."""
    g = gradient_magnitude(image, prob.height, prob.width, prob.spacing, prob.pix_offset)
    m = np.asarray(prob.mask) > 0
    lam = float(np.float32(lam))
    w = np.zeros(len(g), np.int64)
    for a, b in _subject_pixels(prob):
        gs, ms = g[a:b], m[a:b]
        gmax = gs[ms].max() if ms.any() else 0.0
        p = (1.0 - lam) * (gs / gmax) + lam if gmax > 0 else np.full_like(gs, lam)
        w[a:b] = np.where(ms, np.floor(p * QUANT), 0.0).astype(np.int64)
    return w


def sampling_cdf(prob, image, lam):
    """Inclusive cumulative weights, restarting at each subject's first pixel."""
    w = sampling_weights(prob, image, lam)
    c = np.zeros_like(w)
    for a, b in _subject_pixels(prob):
        c[a:b] = np.cumsum(w[a:b])
    return c


def adaptive_means(prob, image, pose, u, lam, gauss_ids=None):
    """Means drawn from Eq. 6 for the Gaussians ``gauss_ids`` (default all),
    Gaussian j using the uniforms u[j].  Returns (mean [n,3] FP64, pixel [n]
    int64, intensity at the pixel [n])."""
    N = prob.n_gauss
    gauss_ids = np.arange(N) if gauss_ids is None else np.asarray(gauss_ids, np.int64)
    u = np.asarray(u, np.float64)[gauss_ids]
    cdf = sampling_cdf(prob, image, lam)
    spx = _subject_pixels(prob)
    goff = np.asarray(prob.gauss_offsets)
    subj = np.searchsorted(goff, gauss_ids, side="right") - 1
    pix = np.zeros(len(gauss_ids), np.int64)
    for s, (a, b) in enumerate(spx):
        sel = np.nonzero(subj == s)[0]
        if len(sel) == 0:
            continue
        total = int(cdf[b - 1])
        if total <= 0:
            raise ValueError(f"subject {s} has no pixel with positive weight")
        t = np.minimum(np.floor(u[sel, 0] * float(total)).astype(np.int64), total - 1)
        pix[sel] = a + np.searchsorted(cdf[a:b], t, side="right")
    po = np.asarray(prob.pix_offset)
    sl = np.searchsorted(po, pix, side="right") - 1
    H = np.asarray(prob.height, np.int64)[sl]
    W = np.asarray(prob.width, np.int64)[sl]
    loc = pix - po[sl]
    r, k = loc // W, loc % W
    sp = np.asarray(prob.spacing, np.float64)[sl]
    thick = np.asarray(prob.psf_fwhm, np.float64)[sl, 2]
    ub = np.stack([(k - (W - 1) / 2.0 + (u[:, 1] - 0.5)) * sp[:, 0],
                   (r - (H - 1) / 2.0 + (u[:, 2] - 0.5)) * sp[:, 1],
                   (u[:, 3] - 0.5) * thick], axis=1)
    pose = np.asarray(pose, np.float64)
    R = Rotation.from_rotvec(pose[sl, :3]).as_matrix() @ np.asarray(prob.rot0, np.float64)[sl].reshape(-1, 3, 3)
    t = np.asarray(prob.trans0, np.float64)[sl] + pose[sl, 3:]
    mean = np.einsum("nab,nb->na", R, ub) + t
    return mean, pix, np.asarray(image, np.float64)[pix]
