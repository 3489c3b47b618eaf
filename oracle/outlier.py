"""Per-slice outlier terms of Sec. 2.4 on top of a data term, FP64 NumPy.

TEST INFRASTRUCTURE ONLY: the HIP path never imports it.

The paper names a learnable intensity scalar sigma_i per slice (global
intensity shifts) and an aleatoric weight omega_i per slice that down-weights
corrupted slices in the loss, without giving the weighting's form.  Reading
(a negative log-likelihood with a per-slice scale, as in the uncertainty
weighting the paper cites NeSVoR for), with rho_i = log omega_i:

* the prediction of slice i is sigma_i y_p; r_p = sigma_i y_p - I_p;
* masked MSE kind (Gaussian likelihood with standard deviation omega_i):
      L = ( sum_i e^{-2 rho_i} S_i + 2 n_i rho_i ) / sum_p m_p,
      S_i = sum_{p in i} m_p r_p^2,  n_i = sum_{p in i} m_p;
* masked L1 kind (Laplace likelihood with scale omega_i):
      L = sum_i e^{-rho_i} S_i + n_i rho_i,  S_i = sum_{p in i} m_p |r_p|.
At sigma = 1 and rho = 0 both reduce to the plain masked MSE and L1 terms.

Gauge: a common factor on every sigma_i of a subject trades against its
amplitudes, and a common shift of its rho_i rescales the whole data term
against the regulariser, so neither is identifiable.  Reading: the loss
uses the per-subject centred values sigma'_i = sigma_i / geomean_s(sigma)
and rho'_i = rho_i - mean_s(rho) (means over the subject's slices); the
terms then only redistribute intensity and weight between slices, and the
gradients with respect to log sigma and rho sum to zero per subject.
Gradients: with respect to y_p, sigma_i and rho_i (the L1 subgradient takes
sign(0) = 0).
"""
from __future__ import annotations

import numpy as np


def slice_loss(pred, target, mask, pix_offset, kind, sigma=None, log_omega=None, slice_subject=None):
    """(loss, dL/dy [P], per-slice data sums S [M], dL/dsigma [M],
    dL/drho [M]) for kind 0 (masked MSE) or 1 (masked L1); slice_subject
    [M] groups the slices for the centring (default: one subject)."""
    y = np.asarray(pred, np.float64)
    t = np.asarray(target, np.float64)
    m = np.asarray(mask, np.float64)
    po = np.asarray(pix_offset, np.int64)
    M = len(po) - 1
    sig_raw = np.ones(M) if sigma is None else np.asarray(sigma, np.float64)
    rho_raw = np.zeros(M) if log_omega is None else np.asarray(log_omega, np.float64)
    subj = np.zeros(M, np.int64) if slice_subject is None else np.asarray(slice_subject, np.int64)
    ls_mean = np.zeros(M)
    rho_mean = np.zeros(M)
    for s in np.unique(subj):
        k = subj == s
        ls_mean[k] = np.log(sig_raw[k]).mean()
        rho_mean[k] = rho_raw[k].mean()
    sig = sig_raw * np.exp(-ls_mean)
    rho = rho_raw - rho_mean
    sl = np.repeat(np.arange(M), np.diff(po))
    yh = sig[sl] * y
    r = yh - t
    n = np.array([m[po[i]:po[i + 1]].sum() for i in range(M)])
    if kind == 0:
        phi = m * r * r
        S = np.array([phi[po[i]:po[i + 1]].sum() for i in range(M)])
        msum = m.sum()
        w = np.exp(-2.0 * rho)
        loss = float((w * S + 2.0 * n * rho).sum() / msum)
        g_yh = w[sl] * 2.0 * m * r / msum
        g_rho = (-2.0 * w * S + 2.0 * n) / msum
    elif kind == 1:
        phi = m * np.abs(r)
        S = np.array([phi[po[i]:po[i + 1]].sum() for i in range(M)])
        w = np.exp(-rho)
        loss = float((w * S + n * rho).sum())
        g_yh = w[sl] * m * np.sign(r)
        g_rho = -w * S + n
    else:
        raise ValueError(kind)
    g_y = g_yh * sig[sl]
    g_sigc = np.array([(g_yh * y)[po[i]:po[i + 1]].sum() for i in range(M)])   # dL/dsigma'_i
    a = sig * g_sigc                                                            # dL/dlog sigma'_i
    g_sig = np.zeros(M)
    g_rho_raw = np.zeros(M)
    for s in np.unique(subj):
        k = subj == s
        g_sig[k] = (a[k] - a[k].mean()) / sig_raw[k]
        g_rho_raw[k] = g_rho[k] - g_rho[k].mean()
    return loss, g_y, S, g_sig, g_rho_raw
