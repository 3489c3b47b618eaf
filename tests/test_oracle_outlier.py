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
    subj = np.array([0, 0, 1, 1])
    sig, rho = rng.uniform(0.7, 1.3, M), rng.normal(0, 0.3, M)
    loss, g, S, gs, gr = outlier.slice_loss(y, t, m, po, kind, sig, rho, subj)
    yt = torch.tensor(y, requires_grad=True)
    st = torch.tensor(sig, requires_grad=True)
    rt = torch.tensor(rho, requires_grad=True)
    sub = torch.as_tensor(subj)
    cnt = torch.zeros(2, dtype=torch.float64).index_add(0, sub, torch.ones(M, dtype=torch.float64))
    lsm = torch.zeros(2, dtype=torch.float64).index_add(0, sub, torch.log(st)) / cnt
    rm = torch.zeros(2, dtype=torch.float64).index_add(0, sub, rt) / cnt
    sc = st * torch.exp(-lsm[sub])
    rc = rt - rm[sub]
    sl = torch.as_tensor(np.repeat(np.arange(M), np.diff(po)))
    r = sc[sl] * yt - torch.tensor(t)
    mt = torch.tensor(m)
    n = torch.zeros(M, dtype=torch.float64).index_add(0, sl, mt)
    if kind == 0:
        Sx = torch.zeros(M, dtype=torch.float64).index_add(0, sl, mt * r * r)
        L = (torch.exp(-2 * rc) * Sx + 2 * n * rc).sum() / mt.sum()
    else:
        Sx = torch.zeros(M, dtype=torch.float64).index_add(0, sl, mt * r.abs())
        L = (torch.exp(-rc) * Sx + n * rc).sum()
    L.backward()
    assert abs(loss - L.item()) < 1e-12
    assert np.abs(g - yt.grad.numpy()).max() < 1e-13
    assert np.abs(gs - st.grad.numpy()).max() < 1e-12
    assert np.abs(gr - rt.grad.numpy()).max() < 1e-12
    # gauge: a common factor on a subject's sigma or shift of its rho changes nothing
    l2 = outlier.slice_loss(y, t, m, po, kind, sig * np.array([2.0, 2.0, 0.5, 0.5]), rho + np.array([1, 1, -3, -3]),
                            subj)[0]
    assert abs(l2 - loss) < 1e-12 * max(1.0, abs(loss))


@pytest.mark.parametrize("kind", [0, 1])
def test_weight_optimum_is_the_slice_scale(kind):
    # slices of equal mask sums n: the (centred) weights are stationary at
    # omega_i^2 proportional to S_i / n (Gaussian) or omega_i to S_i / n
    # (Laplace), the per-slice likelihood scales, whatever the common factor
    y, t, m, po = _data(3, sizes=(50, 50, 50))
    m[:] = 1.0
    S = outlier.slice_loss(y, t, m, po, kind)[2]
    assert np.ptp(S) > 0.1 * S.mean()          # the slices differ
    rho = 0.5 * np.log(S / 50.0) if kind == 0 else np.log(S / 50.0)
    for shift in (0.0, 0.7, -2.0):
        gr = outlier.slice_loss(y, t, m, po, kind, None, rho + shift)[4]
        assert np.abs(gr).max() < 1e-12
    gr = outlier.slice_loss(y, t, m, po, kind, None, np.zeros(3))[4]
    assert np.abs(gr).max() > 1e-2
