"""Multiplicative low-frequency bias field per subject, FP64 NumPy.

TEST INFRASTRUCTURE ONLY: the HIP path never imports it.

The paper lists bias-field Gaussians among its future work (Sec. 4,
"Bias Correction & Robustness") without a form.  Reading: subject s carries K
fixed broad basis Gaussians (centres m_{s,k}, one width w) and learnable
coefficients beta_{s,k}; the bias at a world point x is

    b(x) = exp( sum_k beta_k phi_k(x) ),   phi_k(x) = exp(-|x - m_k|^2 / (2 w^2)),

and the acquired pixel is y'_p = b(x_p) y_p, with x_p = R_i u_p + t_i the
pixel centre of slice i under its current pose (Sec. 2.1: the field moves
with the subject).  beta = 0 gives b = 1 and leaves every pixel unchanged.

Gradients of sum_p g_p y'_p (g = dL/dy'):
    dL/dy_p     = g_p b_p,
    dL/dbeta_k  = sum_p g_p y'_p phi_k(x_p),
    dL/dx_p     = g_p y'_p sum_k beta_k phi_k(x_p) (m_k - x_p) / w^2,
    dL/dtau_i   = sum_{p in i} dL/dx_p,
    dL/ddelta_i = sum_{p in i} (R_i u_p) x dL/dx_p  (left perturbation
                  R_i <- Exp(delta) R_i, as for the Gaussians' pose terms),
    dL/domega_i = J_l(omega_i)^T dL/ddelta_i.
"""
from __future__ import annotations

import numpy as np

from .brute import pixel_coords, slice_frame


def left_jacobian(w):
    """SO(3) left Jacobian J_l(w) = I + (1 - cos t)/t^2 [w]x + (t - sin t)/t^3 [w]x^2."""
    w = np.asarray(w, np.float64)
    t = float(np.linalg.norm(w))
    K = np.array([[0.0, -w[2], w[1]], [w[2], 0.0, -w[0]], [-w[1], w[0], 0.0]])
    if t < 1e-8:
        return np.eye(3) + 0.5 * K
    return np.eye(3) + (1.0 - np.cos(t)) / t ** 2 * K + (t - np.sin(t)) / t ** 3 * (K @ K)


def _slices(prob, pose):
    po = np.concatenate([[0], np.cumsum(prob.height.astype(np.int64) * prob.width.astype(np.int64))])
    for i in range(len(prob.height)):
        R, t = slice_frame(prob.rot0[i], prob.trans0[i], pose[i])
        u = pixel_coords(int(prob.height[i]), int(prob.width[i]), float(prob.spacing[i, 0]), float(prob.spacing[i, 1]))
        yield i, po[i], po[i + 1], R, t, u


def field(prob, centres, width, beta, pose=None):
    """b(x_p) for every pixel [P]; centres [S, K, 3], beta [S, K]."""
    pose = prob.pose if pose is None else pose
    C = np.asarray(centres, np.float64)
    B = np.asarray(beta, np.float64)
    out = np.zeros(int(np.sum(prob.height.astype(np.int64) * prob.width.astype(np.int64))))
    for i, p0, p1, R, t, u in _slices(prob, pose):
        s = int(prob.slice_subject[i])
        x = u @ R.T + t
        phi = np.exp(-((x[:, None, :] - C[s][None, :, :]) ** 2).sum(-1) / (2.0 * width * width))
        out[p0:p1] = np.exp(phi @ B[s])
    return out


def apply(prob, y, centres, width, beta, pose=None):
    """(b y, b) for the predicted pixels y [P]."""
    b = field(prob, centres, width, beta, pose)
    return b * np.asarray(y, np.float64), b


def gradients(prob, y, g, centres, width, beta, pose=None):
    """Gradients of sum_p g_p b_p y_p: dict(pred [P], beta [S, K], pose [M, 6])."""
    pose = prob.pose if pose is None else pose
    C = np.asarray(centres, np.float64)
    B = np.asarray(beta, np.float64)
    y = np.asarray(y, np.float64)
    g = np.asarray(g, np.float64)
    out = dict(pred=np.zeros_like(y), beta=np.zeros_like(B), pose=np.zeros((len(prob.height), 6)))
    for i, p0, p1, R, t, u in _slices(prob, pose):
        s = int(prob.slice_subject[i])
        ru = u @ R.T
        x = ru + t
        d = C[s][None, :, :] - x[:, None, :]                       # m_k - x_p
        phi = np.exp(-(d ** 2).sum(-1) / (2.0 * width * width))     # [n, K]
        b = np.exp(phi @ B[s])
        yb = y[p0:p1] * b
        gp = g[p0:p1]
        out["pred"][p0:p1] = gp * b
        out["beta"][s] += (gp * yb) @ phi
        gx = (gp * yb)[:, None] * ((phi * B[s][None, :])[:, :, None] * d).sum(1) / (width * width)
        dtau = gx.sum(0)
        ddelta = np.cross(ru, gx).sum(0)
        out["pose"][i, 3:] = dtau
        out["pose"][i, :3] = left_jacobian(pose[i, :3]).T @ ddelta
    return out
