"""NumPy brute force of the slice acquisition model: every (slice, pixel,
Gaussian) triple, no pruning, linear algebra by numpy.linalg and rotations by
scipy.  Tiny inputs only.  Test infrastructure only.

Follows Sec. 2.1 (Eq. 1, T_i(u) = R_i u + t_i), Sec. 2.2 (Sigma = R S S^T R^T,
log-space scales) and Sec. 2.3 (Eq. 4: Sigma_obs = Sigma_j + R_i Sigma_PSF R_i^T),
with the sqrt(det Sigma_j / det Sigma_obs) amplitude of the exact convolution.
"""
from __future__ import annotations

import numpy as np
from scipy.spatial.transform import Rotation


def gaussian_cov(quat_wxyz, log_scale):
    q = np.asarray(quat_wxyz, np.float64)
    R = Rotation.from_quat([q[1], q[2], q[3], q[0]]).as_matrix()   # scipy is scalar-last
    S = np.diag(np.exp(np.asarray(log_scale, np.float64)))
    return R @ S @ S.T @ R.T


def slice_frame(rot0, trans0, pose):
    R = Rotation.from_rotvec(np.asarray(pose[:3], np.float64)).as_matrix() @ np.asarray(rot0, np.float64).reshape(3, 3)
    t = np.asarray(trans0, np.float64) + np.asarray(pose[3:], np.float64)
    return R, t


def pixel_coords(h, w, dx, dy):
    cols = (np.arange(w) - (w - 1) / 2.0) * dx
    rows = (np.arange(h) - (h - 1) / 2.0) * dy
    uu, vv = np.meshgrid(cols, rows)
    return np.stack([uu.ravel(), vv.ravel(), np.zeros(h * w)], axis=1)


def forward(prob, tau=np.inf, params=None, pose=None):
    mean, log_scale, quat, amp = params if params is not None else prob.params()
    pose = prob.pose if pose is None else pose
    etau = 0.0 if not np.isfinite(tau) else np.exp(-0.5 * tau * tau)
    mean = np.asarray(mean, np.float64)
    q = np.asarray(quat, np.float64)
    Rg = Rotation.from_quat(q[:, [1, 2, 3, 0]]).as_matrix()          # [N,3,3]
    s2 = np.exp(2.0 * np.asarray(log_scale, np.float64))             # [N,3]
    Sj = np.einsum("nak,nk,nbk->nab", Rg, s2, Rg)
    detj = np.linalg.det(Sj)
    out = []
    for i in range(len(prob.height)):
        R, t = slice_frame(prob.rot0[i], prob.trans0[i], pose[i])
        sig = np.asarray(prob.psf_fwhm[i], np.float64) / 2.355
        P = R @ np.diag(sig ** 2) @ R.T
        u = pixel_coords(int(prob.height[i]), int(prob.width[i]), float(prob.spacing[i, 0]),
                         float(prob.spacing[i, 1]))
        x = u @ R.T + t
        sub = int(prob.slice_subject[i])
        g0, g1 = int(prob.gauss_offsets[sub]), int(prob.gauss_offsets[sub + 1])
        So = Sj[g0:g1] + P[None]
        Li = np.linalg.inv(So)
        rho = np.sqrt(detj[g0:g1] / np.linalg.det(So))
        y = np.zeros(len(x))
        for c0 in range(0, len(x), 256):
            d = x[c0:c0 + 256, None, :] - mean[None, g0:g1, :]            # [p,n,3]
            qf = np.einsum("pna,nab,pnb->pn", d, Li, d)
            v = np.asarray(amp[g0:g1], np.float64)[None] * rho[None] * (np.exp(-0.5 * qf) - etau)
            if np.isfinite(tau):
                v = np.where(qf <= tau * tau, v, 0.0)
            y[c0:c0 + 256] = v.sum(axis=1)
        out.append(y)
    return np.concatenate(out)
