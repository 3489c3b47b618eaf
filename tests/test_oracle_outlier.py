"""Pins of the per-slice outlier-term oracle (Sec. 2.4): reduction to the
plain data terms, autograd gradients, and the likelihood optimum."""
import numpy as np
import pytest
import torch

import oracle
from oracle import outlier


def _data(seed=0, sizes=(30, 0, 45, 25)):
    rng = np.random.default_rng(seed)
    po = np.concatenate([[0], np.cumsum(sizes)])
    P = int(po[-1])
    y, t = rng.standard_normal(P), rng.standard_normal(P)
    m = (rng.uniform(size=P) < 0.8).astype(np.float64)
    return y, t, m, po


@pytest.mark.parametrize("kind", [0, 1])
def test_reduces_to_plain_terms(kind):
    y, t, m, po = _data()
    loss, g, S, _, _ = outlier.slice_loss(y, t, m, po, kind)
    ref = oracle.masked_mse(y, t, m, po) if kind == 0 else oracle.masked_l1(y, t, m, po)
    assert abs(loss - ref[0]) < 1e-12 and np.abs(g - ref[1]).max() < 1e-14 and np.abs(S - ref[2]).max() < 1e-12


@pytest.mark.parametrize("kind", [0, 1])
def test_gradients_match_autograd(kind):
    y, t, m, po = _data(1)
    rng = np.random.default_rng(2)
    M = len(po) - 1
    sig, rho = rng.uniform(0.7, 1.3, M), rng.normal(0, 0.3, M)
    loss, g, S, gs, gr = outlier.slice_loss(y, t, m, po, kind, sig, rho)
    yt = torch.tensor(y, requires_grad=True)
    st = torch.tensor(sig, requires_grad=True)
    rt = torch.tensor(rho, requires_grad=True)
    sl = torch.as_tensor(np.repeat(np.arange(M), np.diff(po)))
    r = st[sl] * yt - torch.tensor(t)
    mt = torch.tensor(m)
    n = torch.zeros(M, dtype=torch.float64).index_add(0, sl, mt)
    if kind == 0:
        Sx = torch.zeros(M, dtype=torch.float64).index_add(0, sl, mt * r * r)
        L = (torch.exp(-2 * rt) * Sx + 2 * n * rt).sum() / mt.sum()
    else:
        Sx = torch.zeros(M, dtype=torch.float64).index_add(0, sl, mt * r.abs())
        L = (torch.exp(-rt) * Sx + n * rt).sum()
    L.backward()
    assert abs(loss - L.item()) < 1e-12
    assert np.abs(g - yt.grad.numpy()).max() < 1e-13
    assert np.abs(gs - st.grad.numpy()).max() < 1e-12
    assert np.abs(gr - rt.grad.numpy()).max() < 1e-12


@pytest.mark.parametrize("kind", [0, 1])
def test_weight_optimum_is_the_slice_scale(kind):
    # dL/drho_i = 0 at omega_i^2 = S_i / n_i (Gaussian) or omega_i = S_i / n_i (Laplace)
    y, t, m, po = _data(3, sizes=(40, 50, 60))
    _, _, S, _, _ = outlier.slice_loss(y, t, m, po, kind)
    n = np.array([m[po[i]:po[i + 1]].sum() for i in range(3)])
    rho = 0.5 * np.log(S / n) if kind == 0 else np.log(S / n)
    _, _, _, _, gr = outlier.slice_loss(y, t, m, po, kind, None, rho)
    assert np.abs(gr).max() < 1e-12
