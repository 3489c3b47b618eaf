"""BF16-MFMA kernels of the pose-proposal CNN against float64 references.

The references are plain torch CPU ops in float64 on operands rounded to
BF16 (round to nearest even) exactly where the kernels round them: both
operands of every GEMM (activations / upstream gradients and weights).
Accumulation is FP32 on the GPU, so the bar is the usual 1e-4 relative
(norm-wise, and element-wise with a floor at 1e-4 of the block maximum).
"""
import numpy as np
import pytest

from helpers import check_close

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

import torch.nn.functional as F  # noqa: E402

from paper_2512_11624_amd import svr  # noqa: E402


def bf(t):
    return t.to(torch.bfloat16).to(torch.float64)


def rnd(shape, seed, scale=1.0, dist="normal"):
    g = torch.Generator().manual_seed(seed)
    if dist == "normal":
        return (torch.randn(*shape, generator=g, dtype=torch.float64) * scale).to(torch.float32)
    return ((torch.rand(*shape, generator=g, dtype=torch.float64) - 0.3) * scale).to(torch.float32)


CONV_SHAPES = [(3, 1, 128, 128, 32), (3, 32, 64, 64, 32), (4, 32, 32, 32, 64), (4, 64, 16, 16, 64),
               (5, 64, 8, 8, 128), (6, 128, 4, 4, 128), (2, 5, 13, 9, 7)]


@pytest.mark.parametrize("shape", CONV_SHAPES, ids=[str(s) for s in CONV_SHAPES])
def test_conv_forward_dgrad_wgrad(shape):
    B, Ci, H, W, Co = shape
    OH, OW = (H + 1) // 2, (W + 1) // 2
    x = rnd((B, Ci, H, W), 1, dist="uniform")
    w = rnd((Co, Ci, 3, 3), 2, scale=(2.0 / (Ci * 9)) ** 0.5)
    b = rnd((Co,), 3, 0.1)
    xd, wd, bd = x.cuda(), w.cuda(), b.cuda()
    y = torch.empty(B, Co, OH, OW, device="cuda")
    svr.conv3x3s2_forward(xd, wd, bd, y, relu=1)
    ref = torch.relu(F.conv2d(bf(x), bf(w), b.double(), stride=2, padding=1))
    torch.cuda.synchronize()
    print(check_close(y.cpu().numpy(), ref.numpy(), "conv fwd"))
    # backward through the ReLU: mask = y > 0 (use the reference output, bitwise
    # independent of the kernel's)
    dy = rnd((B, Co, OH, OW), 4)
    yref = ref.to(torch.float32)
    dmask = dy * (yref > 0)
    dx = torch.empty(B, Ci, H, W, device="cuda")
    svr.conv3x3s2_dgrad(dy.cuda(), yref.cuda(), wd, dx)
    dw = torch.empty_like(wd)
    db = torch.empty_like(bd)
    svr.conv3x3s2_wgrad(dy.cuda(), yref.cuda(), xd, dw, db)
    torch.cuda.synchronize()
    dx_ref = torch.nn.grad.conv2d_input((B, Ci, H, W), bf(w), bf(dmask), stride=2, padding=1)
    dw_ref = torch.nn.grad.conv2d_weight(bf(x), (Co, Ci, 3, 3), bf(dmask), stride=2, padding=1)
    db_ref = bf(dmask).sum(dim=(0, 2, 3))
    print(check_close(dx.cpu().numpy(), dx_ref.numpy(), "conv dgrad"))
    print(check_close(dw.cpu().numpy(), dw_ref.numpy(), "conv wgrad"))
    print(check_close(db.cpu().numpy(), db_ref.numpy(), "conv bias grad"))


@pytest.mark.parametrize("shape", [(7, 524, 256, 1), (7, 256, 6, 0), (70, 33, 65, 1)])
def test_linear_forward_dgrad_wgrad(shape):
    B, Fin, Fout, relu = shape
    x = rnd((B, Fin), 5, dist="uniform")
    w = rnd((Fout, Fin), 6, scale=(2.0 / Fin) ** 0.5)
    b = rnd((Fout,), 7, 0.1)
    y = torch.empty(B, Fout, device="cuda")
    svr.linear_forward(x.cuda(), w.cuda(), b.cuda(), y, relu)
    ref = bf(x) @ bf(w).T + b.double()
    if relu:
        ref = torch.relu(ref)
    torch.cuda.synchronize()
    print(check_close(y.cpu().numpy(), ref.numpy(), "linear fwd"))
    dy = rnd((B, Fout), 8)
    yref = ref.to(torch.float32)
    dmask = dy * (yref > 0) if relu else dy
    dx = torch.empty(B, Fin, device="cuda")
    dw = torch.empty(Fout, Fin, device="cuda")
    db = torch.empty(Fout, device="cuda")
    ymask = yref.cuda() if relu else None
    svr.linear_dgrad(dy.cuda(), ymask, w.cuda(), dx)
    svr.linear_wgrad(dy.cuda(), ymask, x.cuda(), dw, db)
    torch.cuda.synchronize()
    print(check_close(dx.cpu().numpy(), (bf(dmask) @ bf(w)).numpy(), "linear dgrad"))
    print(check_close(dw.cpu().numpy(), (bf(dmask).T @ bf(x)).numpy(), "linear wgrad"))
    print(check_close(db.cpu().numpy(), bf(dmask).sum(0).numpy(), "linear bias grad"))


def _net_reference(params, crops, orient, target):
    """float64 network with BF16 rounding of every GEMM operand; returns loss
    and the flat parameter gradient (same layout as svr_posenet_get_params)."""
    ch = [1, 32, 32, 64, 64, 128, 128]
    p = torch.from_numpy(params).double()
    o = 0
    W, Bs = [], []
    for l in range(6):
        n = ch[l + 1] * ch[l] * 9
        W.append(p[o:o + n].view(ch[l + 1], ch[l], 3, 3)); o += n
        Bs.append(p[o:o + ch[l + 1]]); o += ch[l + 1]
    W1 = p[o:o + 256 * 524].view(256, 524); o += 256 * 524
    b1 = p[o:o + 256]; o += 256
    W2 = p[o:o + 6 * 256].view(6, 256); o += 6 * 256
    b2 = p[o:o + 6]; o += 6
    B = crops.shape[0]
    acts = [crops.double()]
    for l in range(6):
        acts.append(torch.relu(F.conv2d(bf(acts[-1]), bf(W[l]), Bs[l], stride=2, padding=1)))
    feat = torch.cat([acts[6].reshape(B, 512), orient.double()], 1)
    h = torch.relu(bf(feat) @ bf(W1).T + b1)
    y = bf(h) @ bf(W2).T + b2
    r = y - target.double()
    loss = (r * r).sum() / B
    dy = 2 * r / B
    g = []
    dW2 = bf(dy).T @ bf(h)
    db2 = bf(dy).sum(0)
    dh = (bf(dy) @ bf(W2)) * (h > 0)
    dW1 = bf(dh).T @ bf(feat)
    db1 = bf(dh).sum(0)
    dfeat = bf(dh) @ bf(W1)
    da = dfeat[:, :512].reshape(B, 128, 2, 2)
    convg = [None] * 6
    for l in range(5, -1, -1):
        dm = da * (acts[l + 1] > 0)
        dWl = torch.nn.grad.conv2d_weight(bf(acts[l]), W[l].shape, bf(dm), stride=2, padding=1)
        dbl = bf(dm).sum(dim=(0, 2, 3))
        convg[l] = (dWl, dbl)
        if l > 0:
            da = torch.nn.grad.conv2d_input(acts[l].shape, bf(W[l]), bf(dm), stride=2, padding=1)
    for l in range(6):
        g += [convg[l][0].reshape(-1), convg[l][1]]
    g += [dW1.reshape(-1), db1, dW2.reshape(-1), db2]
    return loss.item(), torch.cat(g).numpy(), y.numpy()


def test_network_loss_and_gradient():
    """Whole network against the float64 reference.  Unlike the single-layer
    tests, the two sides no longer feed identical operands to every GEMM: an
    activation that the GPU computes in FP32 and the reference in float64 can
    round to neighbouring BF16 values (a relative step of 2^-8) when it lies
    near a rounding boundary, and such steps propagate through the eight
    layers.  The bar is therefore set from BF16's unit roundoff u = 2^-9:
    norm-wise 8u (1.6e-2) on the output, loss and gradient, with no
    element-wise test; the per-layer tests above hold 1e-4."""
    net = svr.PoseNet(0, seed=11, max_batch=8)
    params = net.get_params()
    B = 5
    crops = rnd((B, 1, 128, 128), 20, dist="uniform")
    orient = rnd((B, 12), 21)
    target = rnd((B, 6), 22)
    loss_ref, g_ref, y_ref = _net_reference(params, crops, orient, target)
    loss = torch.empty(1, device="cuda")
    grads = torch.empty(net.n_params, device="cuda")
    net.grads(crops.cuda(), orient.cuda(), target.cuda(), loss, grads)
    out = torch.empty(B, 6, device="cuda")
    net.forward(crops.cuda(), orient.cuda(), out)
    torch.cuda.synchronize()
    tol = 8 * 2.0 ** -9

    def rel(a, b):
        return float(np.linalg.norm(np.asarray(a, np.float64) - b) / max(np.linalg.norm(b), 1e-300))

    e_out, e_g = rel(out.cpu().numpy(), y_ref), rel(grads.cpu().numpy(), g_ref)
    e_loss = abs(loss.item() - loss_ref) / abs(loss_ref)
    print(f"network: output {e_out:.2e}, loss {e_loss:.2e}, gradient {e_g:.2e} (bar {tol:.2e})")
    assert e_out <= tol and e_loss <= tol and e_g <= tol
    net.close()


def test_train_step_lowers_loss_and_params_roundtrip():
    net = svr.PoseNet(0, seed=3, max_batch=16)
    p0 = net.get_params()
    net.set_params(p0)
    assert np.array_equal(net.get_params(), p0)
    crops = rnd((16, 1, 128, 128), 30, dist="uniform").cuda()
    orient = rnd((16, 12), 31).cuda()
    target = rnd((16, 6), 32).cuda()
    loss = torch.empty(1, device="cuda")
    first = None
    for _ in range(30):
        net.train_step(crops, orient, target, 1e-3, loss)
        torch.cuda.synchronize()
        first = loss.item() if first is None else first
    assert loss.item() < 0.5 * first, (first, loss.item())
    net.close()


def test_prepare_upsamples_centre_window():
    net = svr.PoseNet(0, seed=0, max_batch=4)
    s = rnd((2, 32, 32), 40).cuda()
    crops = torch.empty(2, 128, 128, device="cuda")
    net.prepare(s, crops)
    ref = F.interpolate(s.cpu().double().unsqueeze(1), scale_factor=4, mode="bilinear", align_corners=False)[:, 0]
    torch.cuda.synchronize()
    print(check_close(crops.cpu().numpy(), ref.numpy(), "upsample", rtol=1e-5))
    net.close()
