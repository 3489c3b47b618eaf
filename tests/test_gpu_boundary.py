"""GPU tests of the boundary's modes and error paths, through the C ABI:
fixed-capacity binning (no host synchronisation), finite checks, non-finite
amplitudes, the per-lane emission fallback, and interleaved autograd calls.
"""
import numpy as np
import pytest

from helpers import BAND, check_band, check_close, gpu_params, to_dev
from paper_2512_11624_amd import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

import oracle  # noqa: E402
from paper_2512_11624_amd import svr  # noqa: E402

CFG = dict(tile=32, batch=128, persistent=0, cutoff=3.0, forward_mode=1)


@pytest.fixture(scope="module")
def ctx():
    c = svr.Context(0)
    yield c
    c.close()


def _iteration(ctx, prob, dev, target, mask):
    """project_bin + forward (masked MSE) + backward; device outputs."""
    ctx.svr_project_bin(*dev)
    P = prob.n_pixels
    out = dict(pred=torch.empty(P, device="cuda"), loss=torch.empty(1, device="cuda"),
               gpred=torch.empty(P, device="cuda"))
    ctx.svr_forward(out["pred"], target, mask, loss=out["loss"], grad_pred=out["gpred"])
    grads = [torch.empty_like(x) for x in dev]
    ctx.svr_backward(out["gpred"], *grads)
    for k, g in zip(("mean", "log_scale", "quat", "amp", "pose"), grads):
        out[k] = g
    return out


def _host(out):
    torch.cuda.synchronize()
    return {k: v.cpu().numpy() for k, v in out.items()}


def test_fixed_capacity_matches_synchronised_binning(ctx):
    """A fixed-capacity iteration (no count read-back) gives the same forward
    bits and the same gradients as the synchronising one, for capacities just
    above the counts and well above them."""
    prob = synth.config1(0, n_gauss=1500)
    params = synth.perturb_params(prob, 4)
    ctx.svr_set_config(**CFG)
    ctx.svr_set_geometry(prob)
    dev = gpu_params(params, prob.pose)
    target = to_dev((oracle.forward(prob, np.inf) + synth.gaussian_noise(5, prob.n_pixels, 0.01)).astype(np.float32))
    mask = to_dev(prob.mask)
    ref = _host(_iteration(ctx, prob, dev, target, mask))
    st = ctx.svr_get_stats(sync=True)
    nrec, ninst = st["n_records"], st["n_instances"]
    try:
        for extra in (0, 1, 5000):
            ctx.svr_set_capacity(nrec + extra, ninst + extra)
            out = _host(_iteration(ctx, prob, dev, target, mask))
            assert ctx.svr_check_status() == (svr.SVR_OK, 0, 0)
            st2 = ctx.svr_get_stats(sync=True)
            assert (st2["n_records"], st2["n_instances"]) == (nrec, ninst)
            assert np.array_equal(out["pred"], ref["pred"]), extra
            assert np.array_equal(out["gpred"], ref["gpred"]), extra
            assert out["loss"][0] == ref["loss"][0]
            for k in ("mean", "log_scale", "quat", "amp", "pose"):
                print(check_close(out[k], ref[k], f"{k} (capacity +{extra})", rtol=1e-6))
    finally:
        ctx.svr_set_capacity(0, 0)


def test_fixed_capacity_overflow_is_reported_and_writes_nothing(ctx):
    """Capacities below the counts: the iteration bins nothing (zero
    prediction and gradients, no write out of bounds) and svr_check_status
    returns SVR_ERR_CAPACITY with the counts the synchronising mode finds;
    after growing the capacity the next iteration is correct again."""
    prob = synth.config1(1, n_gauss=1200)
    params = synth.perturb_params(prob, 6)
    ctx.svr_set_config(**CFG)
    ctx.svr_set_geometry(prob)
    dev = gpu_params(params, prob.pose)
    target = to_dev(np.full(prob.n_pixels, 0.3, np.float32))
    mask = to_dev(prob.mask)
    ref = _host(_iteration(ctx, prob, dev, target, mask))
    st = ctx.svr_get_stats(sync=True)
    nrec, ninst = st["n_records"], st["n_instances"]
    try:
        for cap in ((nrec - 1, ninst + 100), (nrec + 100, ninst - 1), (1, 1)):
            ctx.svr_set_capacity(*cap)
            out = _host(_iteration(ctx, prob, dev, target, mask))
            rc, need_r, need_i = ctx.svr_check_status()
            assert rc == svr.SVR_ERR_CAPACITY and (need_r, need_i) == (nrec, ninst), (cap, rc, need_r, need_i)
            assert ctx.svr_check_status()[0] == svr.SVR_OK  # cleared
            assert np.all(out["pred"] == 0.0)
            for k in ("mean", "log_scale", "quat", "amp", "pose"):
                assert np.all(out[k] == 0.0), k
        ctx.svr_set_capacity(need_r, need_i)
        out = _host(_iteration(ctx, prob, dev, target, mask))
        assert ctx.svr_check_status()[0] == svr.SVR_OK
        assert np.array_equal(out["pred"], ref["pred"])
    finally:
        ctx.svr_set_capacity(0, 0)


def test_nonfinite_amplitude_reaches_the_prediction(ctx):
    """One NaN (then infinite) amplitude: every pixel inside that Gaussian's
    footprint is non-finite in every forward mode (the fixed-point modes have
    no quantum for it and mark their pass), and the finite checks report it."""
    prob = synth.config1(2, n_gauss=900)
    params = [a.copy() for a in synth.perturb_params(prob, 8)]
    j = int(np.argmax(params[3]))
    one = [np.zeros_like(a) if k == 3 else a for k, a in enumerate(params)]
    one[3][j] = 1.0
    footprint = oracle.forward(prob, 3.0, params=one, pose=prob.pose) > 0
    assert footprint.sum() > 20
    for bad in (np.nan, np.inf):
        params[3][j] = bad
        for persistent, mode in ((0, 1), (1, 1), (0, 0), (0, 2)):
            ctx.svr_set_config(tile=32, batch=128, persistent=persistent, cutoff=3.0, forward_mode=mode)
            ctx.svr_set_geometry(prob)
            dev = gpu_params(params, prob.pose)
            ctx.svr_project_bin(*dev)
            pred = torch.empty(prob.n_pixels, device="cuda")
            ctx.svr_forward(pred)
            p = pred.cpu().numpy()
            assert not np.isfinite(p[footprint]).any(), (bad, persistent, mode)
            assert np.isfinite(p[~footprint]).sum() > 0
        # the finite checks: project_bin refuses the parameters ...
        ctx.svr_set_checks(svr.SVR_CHECK_FINITE)
        try:
            with pytest.raises(svr.SvrError) as e:
                ctx.svr_project_bin(*dev)
            assert e.value.status == svr.SVR_ERR_NONFINITE
            # ... and the forward's check of the prediction is reported later
            ctx.svr_set_checks(0)
            ctx.svr_project_bin(*dev)
            ctx.svr_set_checks(svr.SVR_CHECK_FINITE)
            ctx.svr_forward(pred)
            assert ctx.svr_check_status()[0] == svr.SVR_ERR_NONFINITE
            assert ctx.svr_check_status()[0] == svr.SVR_OK
            # finite parameters pass every check
            params[3][j] = 0.5
            dev = gpu_params(params, prob.pose)
            out = _iteration(ctx, prob, dev, to_dev(np.zeros(prob.n_pixels, np.float32)), to_dev(prob.mask))
            assert ctx.svr_check_status()[0] == svr.SVR_OK
            assert torch.isfinite(out["pred"]).all()
        finally:
            ctx.svr_set_checks(0)


def test_emission_fallback_blocks_match_the_oracle(ctx):
    """Large Gaussians (scale about 3 mm) over many 1 mm slices: 256-Gaussian
    blocks hold about 9,900 records, more than the coalesced emission's LDS
    list (6,144), so they go through the per-lane emission; the first block
    has small Gaussians and takes the coalesced path.  Both are compared with
    the oracle."""
    prob = synth.config1(3, n_gauss=768, n_per_stack=24, thickness=1.0, size=32)
    rng = np.random.default_rng(1)
    prob.log_scale[:] = (np.log(3.0) + rng.uniform(-0.05, 0.05, prob.log_scale.shape)).astype(np.float32)
    prob.log_scale[:256] = (np.log(0.7) + rng.uniform(-0.05, 0.05, (256, 3))).astype(np.float32)
    params = synth.perturb_params(prob, 9, d_mu=0.2, d_ls=0.02, d_q=0.05, d_c=0.05)
    target = (oracle.forward(prob, np.inf) + synth.gaussian_noise(10, prob.n_pixels, 0.01)).astype(np.float32)
    ctx.svr_set_config(**CFG)
    ctx.svr_set_geometry(prob)
    dev = gpu_params(params, prob.pose)
    out = _host(_iteration(ctx, prob, dev, to_dev(target), to_dev(prob.mask)))
    st = ctx.svr_get_stats(sync=True)
    print(st)
    assert st["n_fallback_blocks"] >= 1, st
    assert st["n_fallback_blocks"] < 3, st  # the small-Gaussian block is emitted the coalesced way
    y = oracle.forward(prob, 3.0, params=params, pose=prob.pose)
    yc, yb = oracle.forward_band(prob, 3.0, BAND, params=params, pose=prob.pose)
    loss, g, _ = oracle.masked_mse(y, target, prob.mask, prob.pix_offset)
    core, bnd = oracle.backward_band(prob, g, 3.0, BAND, params=params, pose=prob.pose)
    print(check_band(out["pred"], yc, yb, "pred"))
    assert abs(out["loss"][0] - loss) <= 1e-4 * loss
    for k in ("mean", "log_scale", "quat", "amp", "pose"):
        print(check_band(out[k], core[k], bnd[k], k))


def test_interleaved_render_loss_calls(ctx):
    """Two render_loss calls on one context before either backward: each
    backward still gives its own loss's oracle gradient (the second binning
    replaced the first; backward bins the saved parameters again)."""
    prob = synth.config1(4, n_gauss=700, n_per_stack=5)
    ctx.svr_set_config(**CFG)
    ctx.svr_set_geometry(prob)
    target = (oracle.forward(prob, np.inf) + synth.gaussian_noise(11, prob.n_pixels, 0.01)).astype(np.float32)
    pa = synth.perturb_params(prob, 12)
    pb = synth.perturb_params(prob, 13)
    da = [t.clone().requires_grad_(True) for t in gpu_params(pa, prob.pose)]
    db = [t.clone().requires_grad_(True) for t in gpu_params(pb, prob.pose)]
    la, _ = svr.render_loss(ctx, *da, to_dev(target), to_dev(prob.mask))
    lb, _ = svr.render_loss(ctx, *db, to_dev(target), to_dev(prob.mask))
    la.backward()
    lb.backward()
    for params, d in ((pa, da), (pb, db)):
        y = oracle.forward(prob, 3.0, params=params, pose=prob.pose)
        _, g, _ = oracle.masked_mse(y, target, prob.mask, prob.pix_offset)
        core, bnd = oracle.backward_band(prob, g, 3.0, BAND, params=params, pose=prob.pose)
        for k, t in zip(("mean", "log_scale", "quat", "amp", "pose"), d):
            print(check_band(t.grad.cpu().numpy(), core[k], bnd[k], k))
