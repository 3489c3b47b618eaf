"""Adaptive densification of the Gaussian mixture, NumPy.

TEST INFRASTRUCTURE ONLY: the HIP path never imports it.

The paper names progressive densification after 3D Gaussian Splatting as
future work (Sec. 4, "Coarse-to-Fine Optimization": start from few large
primitives, then split adaptively) without giving a rule.  Reading, after the
clone/split scheme of 3DGS with the statistics moved to this model's world
frame:

* Statistic.  While fitting, every Gaussian j accumulates
  A_j += ||dL/dmu_j||_2 and n_j += 1 on each step where that gradient is
  not zero (the Gaussian took part in the loss).  FP32, as the fit keeps it.
* Decision (FP32, so that both sides take it bit for bit):
      prune   |c_j| < prune_amp                                 -> 0 outputs
      densify n_j > 0 and A_j > fl(grad_threshold * n_j)       -> 2 outputs
      keep    otherwise                                         -> 1 output
  i.e. the mean gradient norm A_j / n_j above the threshold, written without
  a division.  A densified Gaussian is split when it is large,
  max_k log s_jk > log_scale_threshold, and cloned otherwise.
* Children (FP64 here).  e = the principal axis of Sigma_j (the column of
  R(q_j) of the largest scale s_a; the first such axis on ties).
      split: means mu +- a s_a e, log s_a += 1/2 log(1 - a^2), amplitude
             c / (2 sqrt(1 - a^2)), other scales and the rotation unchanged.
             The pair's mixture keeps the parent's integral and its first two
             moments for every 0 < a < 1; a = sqrt(3)/2 halves s_a and keeps c.
      clone: means mu +- b s_a e, scales and rotation unchanged, amplitude
             c / 2: the integral and the mean are kept, the spread grows by
             b^2 s_a^2 along e.
* Layout.  Outputs stay grouped by subject and in parent order; a parent's
  children take two consecutive places, the "-" child first.  src[k] = j for
  a kept Gaussian, -(j + 1) for a child of j.  Optimiser moments follow src
  (children start from zero, as in 3DGS); the per-slice pose part is kept.
"""
from __future__ import annotations

import numpy as np
from scipy.spatial.transform import Rotation

DEFAULTS = dict(grad_threshold=2e-4, log_scale_threshold=float(np.log(2.0)), split_offset=float(np.sqrt(3.0) / 2.0),
                clone_offset=0.5, prune_amp=0.0)


def accumulate(acc, cnt, g_mean):
    """One step of the statistic: (A + ||g||, n + [g != 0]) in FP32."""
    g = np.asarray(g_mean, np.float32).reshape(-1, 3)
    nrm = np.sqrt((g.astype(np.float64) ** 2).sum(1))
    acc = np.asarray(acc, np.float32) + nrm.astype(np.float32)
    cnt = np.asarray(cnt, np.int32) + (g != 0).any(1).astype(np.int32)
    return acc.astype(np.float32), cnt.astype(np.int32)


def decide(acc, cnt, log_scale, amp, grad_threshold, log_scale_threshold, prune_amp=0.0, **_):
    """Per Gaussian: (outputs in {0, 1, 2}, split flag) by the FP32 rule."""
    acc = np.asarray(acc, np.float32)
    cnt = np.asarray(cnt, np.int32)
    f32 = np.float32
    bound = (f32(grad_threshold) * cnt.astype(np.float32)).astype(np.float32)   # one FP32 product
    dens = (cnt > 0) & (acc > bound)
    prune = np.abs(np.asarray(amp, np.float32)) < f32(prune_amp)
    n_out = np.where(prune, 0, np.where(dens, 2, 1)).astype(np.int32)
    large = np.asarray(log_scale, np.float32).max(1) > f32(log_scale_threshold)
    return n_out, large & (n_out == 2)


def principal_axis(log_scale, quat):
    """(axis index a, unit axis e [N, 3], s_a) of each Gaussian; quat (w, x, y, z), any norm."""
    ls = np.asarray(log_scale, np.float64)
    q = np.asarray(quat, np.float64)
    R = Rotation.from_quat(q[:, [1, 2, 3, 0]]).as_matrix()
    a = np.argmax(ls, axis=1)
    e = R[np.arange(len(a)), :, a]
    return a, e, np.exp(ls[np.arange(len(a)), a])


def children(mean, log_scale, quat, amp, split, split_offset, clone_offset, **_):
    """Both children of every given parent: ((mean-, mean+), log_scale, quat, amp) in FP64."""
    mean = np.asarray(mean, np.float64)
    ls = np.asarray(log_scale, np.float64).copy()
    amp = np.asarray(amp, np.float64)
    a, e, sa = principal_axis(ls, quat)
    off = np.where(split, split_offset, clone_offset)
    d = (off * sa)[:, None] * e
    ls_child = ls.copy()
    shrink = 0.5 * np.log1p(-split_offset * split_offset)
    ls_child[np.arange(len(a)), a] += np.where(split, shrink, 0.0)
    amp_child = np.where(split, amp / (2.0 * np.sqrt(1.0 - split_offset * split_offset)), 0.5 * amp)
    return (mean - d, mean + d), ls_child, np.asarray(quat, np.float64), amp_child


def densify(gauss_offsets, mean, log_scale, quat, amp, acc, cnt, cfg=None, exp_avg=None, exp_avg_sq=None):
    """The densified mixture.  Returns dict(mean, log_scale, quat, amp, src, offsets, n_out, split
    [, exp_avg, exp_avg_sq]); moments are laid out as mean (3N), log_scale (3N), quat (4N),
    amp (N), pose (6M)."""
    cfg = dict(DEFAULTS, **(cfg or {}))
    N = len(amp)
    n_out, split = decide(acc, cnt, log_scale, amp, **cfg)
    (cm, cp), cls, cq, ca = children(mean, log_scale, quat, amp, split, **cfg)
    src, rows = [], []
    for j in range(N):
        if n_out[j] == 1:
            src.append(j)
            rows.append((np.asarray(mean[j], np.float64), np.asarray(log_scale[j], np.float64),
                         np.asarray(quat[j], np.float64), float(amp[j])))
        elif n_out[j] == 2:
            src += [-(j + 1), -(j + 1)]
            rows.append((cm[j], cls[j], cq[j], float(ca[j])))
            rows.append((cp[j], cls[j], cq[j], float(ca[j])))
    go = np.asarray(gauss_offsets, np.int64)
    pos = np.concatenate([[0], np.cumsum(n_out)])
    out = dict(src=np.asarray(src, np.int32), offsets=pos[go].astype(np.int64), n_out=n_out, split=split,
               mean=np.array([r[0] for r in rows]).reshape(-1, 3), log_scale=np.array([r[1] for r in rows]).reshape(-1, 3),
               quat=np.array([r[2] for r in rows]).reshape(-1, 4), amp=np.array([r[3] for r in rows]))
    if exp_avg is not None:
        out["exp_avg"] = remap_moments(exp_avg, out["src"], N)
        out["exp_avg_sq"] = remap_moments(exp_avg_sq, out["src"], N)
    return out


def remap_moments(mom, src, N):
    """Optimiser moments after densification: gathered for kept Gaussians, zero for children."""
    mom = np.asarray(mom)
    src = np.asarray(src, np.int64)
    K = len(src)
    parts, off = [], 0
    for w in (3, 3, 4, 1):
        blk = mom[off:off + w * N].reshape(N, w)
        new = np.zeros((K, w), mom.dtype)
        keep = src >= 0
        new[keep] = blk[src[keep]]
        parts.append(new.ravel())
        off += w * N
    parts.append(mom[off:])
    return np.concatenate(parts)
