"""GPU parity of the per-slice outlier terms (Sec. 2.4: intensity scalar
sigma_i and aleatoric weight omega_i) and of the vector AdamW, through the C
ABI against the FP64 oracle."""
import numpy as np
import pytest

from helpers import check_close, to_dev
from paper_2512_11624_amd import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

import oracle  # noqa: E402
from oracle import outlier  # noqa: E402
from paper_2512_11624_amd import svr  # noqa: E402


@pytest.fixture(scope="module")
def ctx():
    c = svr.Context(0)
    yield c
    c.svr_set_loss(svr.SVR_LOSS_MSE)
    c.close()


def _ragged():
    return synth.concat([synth.config1(3, n_gauss=300, size=24, n_per_stack=6),
                         synth.tiny(5, n_gauss=40, n_slices=3, size=(13, 29))])


@pytest.mark.parametrize("kind", [svr.SVR_LOSS_MSE, svr.SVR_LOSS_L1])
@pytest.mark.parametrize("name", ["head", "ragged"])
def test_slice_loss_matches_oracle(ctx, name, kind):
    prob = synth.config2(0) if name == "head" else _ragged()
    ctx.svr_set_geometry(prob)
    ctx.svr_set_loss(kind)
    rng = np.random.default_rng(4)
    P, M = prob.n_pixels, prob.n_slices
    pred = rng.uniform(0, 1, P).astype(np.float32)
    target = (pred + rng.normal(0, 0.05, P)).astype(np.float32)
    sigma = rng.uniform(0.8, 1.2, M).astype(np.float32)
    rho = rng.normal(0, 0.3, M).astype(np.float32)
    mask = prob.mask.astype(np.float32)
    out = dict(loss=torch.empty(1, device="cuda"), grad_pred=torch.empty(P, device="cuda"),
               slice_sums=torch.empty(M, device="cuda"), g_sigma=torch.empty(M, device="cuda"),
               g_log_omega=torch.empty(M, device="cuda"))
    ctx.svr_slice_loss(to_dev(pred), to_dev(target), to_dev(mask), to_dev(sigma), to_dev(rho), **out)
    torch.cuda.synchronize()
    loss, g, S, gs, gr = outlier.slice_loss(pred, target, mask, prob.pix_offset, kind, sigma, rho,
                                            prob.slice_subject)
    check_close([out["loss"].item()], [loss], "loss")
    gp = out["grad_pred"].cpu().numpy()
    if kind == svr.SVR_LOSS_L1:
        # the sign of r may differ where |r| is at FP32 rounding level
        sc = sigma.astype(np.float64)
        for s_ in np.unique(prob.slice_subject):
            k_ = prob.slice_subject == s_
            sc[k_] /= np.exp(np.log(sc[k_]).mean())
        r = sc[np.repeat(np.arange(M), np.diff(prob.pix_offset))] * pred - target
        keep = np.abs(r) > 1e-5
        check_close(gp[keep], g[keep], "grad_pred")
    else:
        check_close(gp, g, "grad_pred")
    check_close(out["slice_sums"].cpu().numpy(), S, "slice_sums")
    check_close(out["g_sigma"].cpu().numpy(), gs, "g_sigma")
    check_close(out["g_log_omega"].cpu().numpy(), gr, "g_log_omega")
    # defaults: sigma = 1, rho = 0 give the plain masked data term
    ctx.svr_slice_loss(to_dev(pred), to_dev(target), to_dev(mask), loss=out["loss"])
    ref = oracle.masked_mse(pred, target, mask, prob.pix_offset) if kind == 0 else \
        oracle.masked_l1(pred, target, mask, prob.pix_offset)
    check_close([out["loss"].item()], [ref[0]], "plain loss")
    ctx.svr_set_loss(svr.SVR_LOSS_MSE)


def test_adam_vector_matches_oracle(ctx):
    ctx.svr_set_geometry(synth.tiny(1))
    rng = np.random.default_rng(6)
    n = 1000
    p0 = rng.standard_normal(n)
    p = to_dev(p0.astype(np.float32))
    m = torch.zeros(n, device="cuda")
    v = torch.zeros(n, device="cuda")
    pr, mr, vr = p0.copy(), np.zeros(n), np.zeros(n)
    for step in range(1, 6):
        g = rng.standard_normal(n).astype(np.float32)
        ctx.svr_adam_vector(p, to_dev(g), m, v, 1e-2, step, weight_decay=0.01)
        pr, mr, vr = oracle.adamw_step(pr, g, mr, vr, step, 1e-2, wd=0.01)
    torch.cuda.synchronize()
    check_close(p.cpu().numpy(), pr, "p")
