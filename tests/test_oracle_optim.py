"""Pins of the oracle's loss and optimiser against library routines."""
import numpy as np
import torch

import oracle


def test_masked_mse_matches_torch():
    rng = np.random.default_rng(0)
    y, t = rng.standard_normal(500), rng.standard_normal(500)
    m = (rng.uniform(size=500) < 0.7).astype(np.float64)
    po = np.array([0, 100, 260, 500])
    loss, grad, sse = oracle.masked_mse(y, t, m, po)
    yt = torch.tensor(y, requires_grad=True)
    sel = torch.tensor(m > 0)
    ref = torch.nn.functional.mse_loss(yt[sel], torch.tensor(t)[sel])
    ref.backward()
    assert abs(loss - ref.item()) < 1e-14
    assert np.abs(grad - yt.grad.numpy()).max() < 1e-15
    for i in range(3):
        s = slice(po[i], po[i + 1])
        ref_i = torch.nn.functional.mse_loss(yt[s][sel[s]], torch.tensor(t)[s][sel[s]], reduction="sum")
        assert abs(sse[i] - ref_i.item()) < 1e-12


def test_adamw_matches_torch():
    rng = np.random.default_rng(1)
    p0 = rng.standard_normal(64)
    pt = torch.tensor(p0.copy(), requires_grad=True)
    opt = torch.optim.AdamW([pt], lr=2.5e-2, betas=(0.9, 0.999), eps=1e-8, weight_decay=0.01)
    p, m, v = p0.copy(), np.zeros(64), np.zeros(64)
    for step in range(1, 8):
        g = rng.standard_normal(64)
        pt.grad = torch.tensor(g)
        opt.step()
        p, m, v = oracle.adamw_step(p, g, m, v, step, 2.5e-2, wd=0.01)
        assert np.abs(p - pt.detach().numpy()).max() < 1e-14


def test_steplr_matches_torch():
    pt = torch.zeros(1, requires_grad=True)
    opt = torch.optim.SGD([pt], lr=0.1)
    sch = torch.optim.lr_scheduler.StepLR(opt, step_size=200, gamma=0.5)
    ref = oracle.StepLR(0.1)
    for it in range(650):
        assert abs(opt.param_groups[0]["lr"] - ref.lr(it)) < 1e-15
        opt.step()
        sch.step()


def test_masked_l1_matches_torch():
    """Eq. 7's L1 data term (masked, summed) against torch's l1_loss and autograd."""
    rng = np.random.default_rng(3)
    y, t = rng.standard_normal(400), rng.standard_normal(400)
    m = (rng.uniform(size=400) < 0.6).astype(np.float64)
    po = np.array([0, 150, 400])
    loss, grad, per_slice = oracle.masked_l1(y, t, m, po)
    yt = torch.tensor(y, requires_grad=True)
    sel = torch.tensor(m > 0)
    ref = torch.nn.functional.l1_loss(yt[sel], torch.tensor(t)[sel], reduction="sum")
    ref.backward()
    assert abs(loss - ref.item()) < 1e-12
    assert np.abs(grad - yt.grad.numpy()).max() == 0.0
    for i in range(2):
        s = slice(po[i], po[i + 1])
        ref_i = torch.nn.functional.l1_loss(yt[s][sel[s]], torch.tensor(t)[s][sel[s]], reduction="sum")
        assert abs(per_slice[i] - ref_i.item()) < 1e-12


def test_scale_regularizer_value_and_gradient():
    """Eq. 7's regulariser on s = exp(log s): torch autograd and central differences."""
    rng = np.random.default_rng(4)
    ls = rng.uniform(np.log(0.3), np.log(3.0), size=(50, 3))
    val, g = oracle.scale_regularizer(ls, 2.5e-3, 1.6)
    lt = torch.tensor(ls, requires_grad=True)
    ref = 2.5e-3 * ((torch.exp(lt) - 1.6) ** 2).sum()
    ref.backward()
    assert abs(val - ref.item()) < 1e-15
    assert np.abs(g - lt.grad.numpy()).max() < 1e-15
    h = 1e-6
    for idx in [(0, 0), (17, 2), (49, 1)]:
        lp, lm = ls.copy(), ls.copy()
        lp[idx] += h
        lm[idx] -= h
        fd = (oracle.scale_regularizer(lp, 2.5e-3, 1.6)[0] - oracle.scale_regularizer(lm, 2.5e-3, 1.6)[0]) / (2 * h)
        assert abs(fd - g[idx]) < 1e-9
    # at s = s_target the regulariser and its gradient vanish
    v0, g0 = oracle.scale_regularizer(np.full((4, 3), np.log(1.6)), 1.0, 1.6)
    assert v0 < 1e-28 and np.abs(g0).max() < 1e-14
