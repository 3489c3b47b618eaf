"""Masked-MSE loss and AdamW, FP64 NumPy, written from their definitions.
Test infrastructure only.

* Loss: L = sum_p m_p (y_p - I_p)^2 / sum_p m_p, the masked mean squared error
  that replaces the paper's L1 data term (Eq. 7) on this hot path; its
  gradient is dL/dy_p = 2 m_p (y_p - I_p) / sum m, and the per-slice masked sum
  of squares SSE_i is reported alongside.
* AdamW (the optimiser of App. A.1, Loshchilov & Hutter): decoupled weight decay
  p <- p (1 - lr wd), first/second moments with bias correction,
  p <- p - lr m_hat / (sqrt(v_hat) + eps).
* StepLR: the learning rate halves every 200 iterations (App. A.1).
* The paper's own objective (Sec. 2.5, Eq. 7): an L1 data term summed over the
  slices' pixels, L = sum_p m_p |y_p - I_p| (the mask m as on the rest of this
  path), with subgradient dL/dy_p = m_p sign(y_p - I_p) (0 where y = I), plus
  a scale regulariser lambda sum_j ||s_j - s_target||^2 on the scales
  s = exp(log s), whose gradient with respect to the log-scales is
  2 lambda (s - s_target) s.
"""
from __future__ import annotations

import numpy as np


def masked_mse(pred, target, mask, pix_offset):
    y = np.asarray(pred, np.float64)
    t = np.asarray(target, np.float64)
    m = np.asarray(mask, np.float64)
    r = y - t
    msum = m.sum()
    sq = m * r * r
    loss = sq.sum() / msum
    grad = 2.0 * m * r / msum
    po = np.asarray(pix_offset, np.int64)
    sse = np.array([sq[po[i]:po[i + 1]].sum() for i in range(len(po) - 1)])
    return loss, grad, sse


def adamw_step(p, g, m, v, step, lr, beta1=0.9, beta2=0.999, eps=1e-8, wd=0.0):
    """One AdamW update in float64; returns (p, m, v).  step counts from 1."""
    p = np.asarray(p, np.float64) * (1.0 - lr * wd)
    g = np.asarray(g, np.float64)
    m = beta1 * np.asarray(m, np.float64) + (1.0 - beta1) * g
    v = beta2 * np.asarray(v, np.float64) + (1.0 - beta2) * g * g
    mhat = m / (1.0 - beta1 ** step)
    vhat = v / (1.0 - beta2 ** step)
    p = p - lr * mhat / (np.sqrt(vhat) + eps)
    return p, m, v


class StepLR:
    def __init__(self, base_lr, step_size=200, gamma=0.5):
        self.base_lr, self.step_size, self.gamma = base_lr, step_size, gamma

    def lr(self, it):
        """Learning rate used by iteration ``it`` (0-based)."""
        return self.base_lr * self.gamma ** (it // self.step_size)


def masked_l1(pred, target, mask, pix_offset):
    """Eq. 7's data term with the mask: (loss, dL/dy, per-slice sums)."""
    y = np.asarray(pred, np.float64)
    t = np.asarray(target, np.float64)
    m = np.asarray(mask, np.float64)
    r = y - t
    ab = m * np.abs(r)
    loss = ab.sum()
    grad = m * np.sign(r)
    po = np.asarray(pix_offset, np.int64)
    per_slice = np.array([ab[po[i]:po[i + 1]].sum() for i in range(len(po) - 1)])
    return loss, grad, per_slice


def scale_regularizer(log_scale, lam, s_target):
    """Eq. 7's regulariser: (value, d value / d log_scale) for scales exp(log_scale)."""
    s = np.exp(np.asarray(log_scale, np.float64))
    d = s - float(s_target)
    return float(lam) * float(np.sum(d * d)), 2.0 * float(lam) * d * s
