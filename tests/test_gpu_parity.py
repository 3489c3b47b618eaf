"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle.

Inputs are seeded synthetic problems (paper_2512_11624_amd.synth).  Targets
are the oracle's exact forward (tau = inf) of the ground truth plus noise; the
evaluated parameters are a seeded perturbation of the ground truth so that
residuals and gradients are non-trivial.
"""
import numpy as np
import pytest

from helpers import BAND, BENCH_CONFIG_IDS, BENCH_CONFIGS, check_band, check_close, gpu_params, to_dev
from paper_2512_11624_amd import synth

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

import oracle  # noqa: E402
from paper_2512_11624_amd import svr  # noqa: E402


def _setup(prob, seed=1, pose_jitter=0.01, tau_target=np.inf, noise=0.01):
    params = synth.perturb_params(prob, seed)
    rng = np.random.default_rng(seed + 100)
    pose = (prob.pose + rng.normal(0, pose_jitter, prob.pose.shape)).astype(np.float32)
    target = (oracle.forward(prob, tau_target) + synth.gaussian_noise(seed + 200, prob.n_pixels, noise)).astype(np.float32)
    return params, pose, target


def _run(ctx, prob, params, pose, target, mask=None, cfg=None):
    if cfg:
        ctx.svr_set_config(**cfg)
    ctx.svr_set_geometry(prob)
    dev = gpu_params(params, pose)
    ctx.svr_project_bin(*dev)
    P = prob.n_pixels
    pred = torch.empty(P, device="cuda")
    loss = torch.empty(1, device="cuda")
    sse = torch.empty(prob.n_slices, device="cuda")
    gpred = torch.empty(P, device="cuda")
    t = to_dev(target)
    m = to_dev(prob.mask if mask is None else mask)
    ctx.svr_forward(pred, t, m, loss=loss, slice_sse=sse, grad_pred=gpred)
    grads = [torch.empty_like(x) for x in dev]
    ctx.svr_backward(gpred, *grads)
    torch.cuda.synchronize()
    return dict(pred=pred.cpu().numpy(), loss=loss.item(), sse=sse.cpu().numpy(), gpred=gpred.cpu().numpy(),
                mean=grads[0].cpu().numpy(), log_scale=grads[1].cpu().numpy(), quat=grads[2].cpu().numpy(),
                amp=grads[3].cpu().numpy(), pose=grads[4].cpu().numpy())


def _oracle(prob, params, pose, target, mask=None):
    """Oracle outputs; pred and the parameter gradients as (core, bound) band
    splits (see helpers.check_band)."""
    y = oracle.forward(prob, 3.0, params=params, pose=pose)
    yc, yb = oracle.forward_band(prob, 3.0, BAND, params=params, pose=pose)
    m = prob.mask if mask is None else mask
    loss, g, sse = oracle.masked_mse(y, target, m, prob.pix_offset)
    core, bnd = oracle.backward_band(prob, g, 3.0, BAND, params=params, pose=pose)
    return dict(pred=y, pred_band=(yc, yb), loss=loss, sse=sse, gpred=g, grad_band=(core, bnd))


def _compare(out, ref):
    infos = [check_band(out["pred"], *ref["pred_band"], "pred"), check_close(out["sse"], ref["sse"], "sse"),
             check_close(out["gpred"], ref["gpred"], "gpred")]
    core, bnd = ref["grad_band"]
    for b in ("mean", "log_scale", "quat", "amp", "pose"):
        infos.append(check_band(out[b], core[b], bnd[b], b))
    assert abs(out["loss"] - ref["loss"]) <= 1e-4 * abs(ref["loss"]), (out["loss"], ref["loss"])
    print("\n".join(infos))


@pytest.fixture(scope="module")
def ctx():
    c = svr.Context(0)
    yield c
    c.close()


def test_cube_forward_backward_parity(ctx):
    """Cube phantom (2,000 Gaussians, 48 slices of 32x32): every output block."""
    prob = synth.config1(0)
    params, pose, target = _setup(prob)
    ref = _oracle(prob, params, pose, target)
    for fm in (0, 2):
        out = _run(ctx, prob, params, pose, target,
                   cfg=dict(tile=16, batch=128, persistent=0, cutoff=3.0, forward_mode=fm))
        _compare(out, ref)


@pytest.mark.parametrize("tile,batch,persistent,mode", [(8, 32, 0, 0), (16, 64, 1, 0), (32, 256, 0, 0), (32, 96, 1, 0),
                                                        (8, 128, 1, 1), (16, 128, 0, 1), (32, 128, 1, 1),
                                                        (8, 128, 0, 2), (16, 128, 1, 2), (32, 128, 0, 2)])
def test_cube_parity_all_configs(ctx, tile, batch, persistent, mode):
    prob = synth.config1(0, n_gauss=800)
    params, pose, target = _setup(prob, seed=3)
    out = _run(ctx, prob, params, pose, target,
               cfg=dict(tile=tile, batch=batch, persistent=persistent, cutoff=3.0, forward_mode=mode))
    ref = _oracle(prob, params, pose, target)
    _compare(out, ref)


def test_ragged_slices_and_subjects(ctx):
    """Ragged slice sizes (not multiples of any tile) and three subjects batched."""
    subs = [synth.config1(5, n_gauss=300, size=37, n_per_stack=5),
            synth.tiny(7, n_gauss=40, n_slices=3, size=(23, 19)),
            synth.config1(6, n_gauss=500, size=45, n_per_stack=4, n_stacks=2)]
    prob = synth.concat(subs)
    params, pose, target = _setup(prob, seed=5)
    for tile, mode in ((8, 0), (16, 1), (32, 0), (32, 1), (16, 2), (32, 2), (8, 2)):
        out = _run(ctx, prob, params, pose, target,
                   cfg=dict(tile=tile, batch=128, persistent=int(tile == 16), cutoff=3.0, forward_mode=mode))
        ref = _oracle(prob, params, pose, target)
        _compare(out, ref)


def test_head_subproblem_parity(ctx):
    """Head phantom at fetal-scale density, reduced: 20k Gaussians in a small
    head, four stacks of 4 slices of 72x72 px (4.5 tiles: ragged) at 0.8 x 0.8 x 3.5 mm."""
    prob = synth.config2(0, n_gauss=20000, n_per_stack=4, size=72, axes=(22.0, 26.0, 23.0))
    params, pose, target = _setup(prob, seed=9, tau_target=6.0)
    out = _run(ctx, prob, params, pose, target)
    ref = _oracle(prob, params, pose, target)
    _compare(out, ref)


def test_empty_and_degenerate(ctx):
    """No Gaussians; a Gaussian far outside every slice; a zero mask."""
    prob = synth.config1(0, n_gauss=3, n_per_stack=2)
    prob.mean[:] = 500.0       # nowhere near any slice
    params = prob.params()
    target = np.ones(prob.n_pixels, np.float32)
    out = _run(ctx, prob, params, prob.pose, target)
    assert np.all(out["pred"] == 0.0)
    assert np.all(out["mean"] == 0.0) and np.all(out["pose"] == 0.0)
    st = ctx.svr_get_stats()
    assert st["n_records"] == 0 and st["n_instances"] == 0
    # zero mask: loss 0, grad 0
    prob2 = synth.config1(0, n_gauss=50, n_per_stack=2)
    out2 = _run(ctx, prob2, prob2.params(), prob2.pose, target, mask=np.zeros(prob2.n_pixels, np.float32))
    assert out2["loss"] == 0.0 and np.all(out2["gpred"] == 0.0)
    # zero Gaussians
    e = synth.config1(0, n_gauss=1, n_per_stack=2)
    empty = synth.Problem(e.mean[:0], e.log_scale[:0], e.quat[:0], e.amp[:0], np.array([0, 0], np.int64),
                          e.slice_subject, e.height, e.width, e.spacing, e.psf_fwhm, e.rot0, e.trans0, e.pose,
                          e.mask)
    ctx.svr_set_geometry(empty)
    z = torch.zeros(0, 3, device="cuda")
    ctx.svr_project_bin(z, z, torch.zeros(0, 4, device="cuda"), torch.zeros(0, device="cuda"), to_dev(e.pose))
    pred = torch.full((empty.n_pixels,), 7.0, device="cuda")
    ctx.svr_forward(pred)
    torch.cuda.synchronize()
    assert torch.all(pred == 0)


@pytest.mark.parametrize("mode", [0, 1, 2])
def test_forward_is_deterministic(ctx, mode):
    """Forward modes 0 and 2 sum in a fixed order and mode 1 sums exact
    integers per round: repeating a forward (after a fresh binning) gives the
    same bits."""
    prob = synth.config1(2, n_gauss=1500)
    params, pose, _ = _setup(prob, seed=13)
    ctx.svr_set_config(tile=16, batch=128, persistent=1, cutoff=3.0, forward_mode=mode)
    ctx.svr_set_geometry(prob)
    dev = gpu_params(params, pose)
    outs = []
    for _ in range(3):
        ctx.svr_project_bin(*dev)
        pred = torch.empty(prob.n_pixels, device="cuda")
        ctx.svr_forward(pred)
        outs.append(pred)
    torch.cuda.synchronize()
    assert torch.equal(outs[0], outs[1]) and torch.equal(outs[0], outs[2])


def test_pose_gradient_is_deterministic(ctx):
    """The slices' pose gradients are summed in a fixed order (per workgroup
    in fixed point, then over workgroups in two ordered levels): repeating the
    adjoint gives the same bits, on several subjects."""
    subs = [synth.config1(s, n_gauss=1200 + 400 * s, n_per_stack=6 + 2 * s) for s in range(3)]
    prob = synth.concat(subs)
    params, pose, _ = _setup(prob, seed=17)
    g = to_dev(np.random.default_rng(18).standard_normal(prob.n_pixels).astype(np.float32))
    ctx.svr_set_config(tile=16, batch=128, persistent=0, cutoff=3.0, forward_mode=1)
    ctx.svr_set_geometry(prob)
    dev = gpu_params(params, pose)
    outs = []
    for _ in range(3):
        ctx.svr_project_bin(*dev)
        grads = [torch.empty_like(x) for x in dev]
        ctx.svr_backward(g, *grads)
        outs.append(grads[4])
    torch.cuda.synchronize()
    assert torch.equal(outs[0], outs[1]) and torch.equal(outs[0], outs[2])
    core, bnd = oracle.backward_band(prob, g.cpu().numpy().astype(np.float64), 3.0, BAND, params=params, pose=pose)
    print(check_band(outs[0].cpu().numpy(), core["pose"], bnd["pose"], "pose"))


def test_backward_with_random_upstream(ctx):
    """Adjoint alone: an arbitrary seeded upstream gradient (not a loss gradient)."""
    prob = synth.config1(1, n_gauss=1000)
    params, pose, _ = _setup(prob, seed=11)
    g = np.random.default_rng(12).standard_normal(prob.n_pixels).astype(np.float32)
    ctx.svr_set_config(tile=16, batch=128, persistent=0, cutoff=3.0, forward_mode=2)
    ctx.svr_set_geometry(prob)
    dev = gpu_params(params, pose)
    ctx.svr_project_bin(*dev)
    grads = [torch.empty_like(x) for x in dev]
    scale = torch.tensor([0.5], device="cuda")
    ctx.svr_backward(to_dev(g), *grads, grad_scale=scale)
    torch.cuda.synchronize()
    core, bnd = oracle.backward_band(prob, 0.5 * g.astype(np.float64), 3.0, BAND, params=params, pose=pose)
    for k, t in zip(("mean", "log_scale", "quat", "amp", "pose"), grads):
        print(check_band(t.cpu().numpy(), core[k], bnd[k], k))


def test_incut_pair_count_brackets(ctx):
    """The in-cut pair count is decided by float comparisons: the GPU (FP32)
    count must lie between the oracle's counts at slightly smaller and larger
    cutoffs."""
    prob = synth.config1(0)
    params, pose, _ = _setup(prob)
    ctx.svr_set_geometry(prob)
    ctx.svr_set_config(tile=16, batch=128, persistent=0, cutoff=3.0)
    dev = gpu_params(params, pose)
    ctx.svr_project_bin(*dev)
    ctx.svr_set_count_pairs(True)
    pred = torch.empty(prob.n_pixels, device="cuda")
    ctx.svr_forward(pred)
    st = ctx.svr_get_stats(sync=True)
    ctx.svr_set_count_pairs(False)
    _, lo, _ = oracle.forward(prob, 3.0 * (1 - 1e-4), params=params, pose=pose, counts=True)
    _, hi, _ = oracle.forward(prob, 3.0 * (1 + 1e-4), params=params, pose=pose, counts=True)
    assert lo <= st["n_incut"] <= hi, (lo, st["n_incut"], hi)


def test_timing_stage_mask(ctx):
    """With a stage mask only the selected stage is bracketed by events (and
    counted); the mask does not change any result."""
    prob = synth.config1(0)
    params, pose, target = _setup(prob)
    ref = _run(ctx, prob, params, pose, target, cfg=dict(tile=16, batch=128, persistent=0, cutoff=3.0))
    ctx.svr_set_timing_stages(["backward_tile"])
    ctx.svr_set_timing(True)
    out = _run(ctx, prob, params, pose, target)
    t = ctx.svr_get_timing()
    ctx.svr_set_timing(False)
    ctx.svr_set_timing_stages(None)
    assert t["backward_tile"][0] == 1 and t["backward_tile"][1] > 0.0, t
    assert all(c == 0 for k, (c, _) in t.items() if k != "backward_tile"), t
    assert np.array_equal(out["pred"], ref["pred"])  # the forward is deterministic
    for k in ("mean", "log_scale", "quat", "amp", "pose"):  # per-Gaussian sums may add in another order
        assert np.allclose(out[k], ref[k], rtol=1e-5, atol=1e-6 * np.abs(ref[k]).max()), k
    with pytest.raises(ValueError):
        ctx.svr_set_timing_stages(["no_such_stage"])


def test_autotune_picks_a_timed_config_and_stays_correct(ctx, tmp_path):
    """The autotuner times every candidate, installs the fastest, caches it
    (in the context and in a file: a second call returns the same choice), and
    the chosen configuration still matches the oracle."""
    prob = synth.config1(0)
    params, pose, target = _setup(prob)
    ctx.svr_set_config(tile=16, batch=128, persistent=0, cutoff=3.0, forward_mode=1)
    ctx.svr_set_geometry(prob)
    dev = gpu_params(params, pose)
    gp = torch.ones(prob.n_pixels, device="cuda")
    cache = str(tmp_path / "tune.txt")
    flags = svr.SVR_TUNE_TILE | svr.SVR_TUNE_MODE | svr.SVR_TUNE_PERSISTENT
    cfg, times = ctx.svr_autotune(*dev, gp, flags=flags, cache_path=cache)
    assert len(times) == 3 * 2 * 3 and all(t > 0 for t in times), times
    assert cfg["tile"] in (8, 16, 32) and cfg["forward_mode"] in (0, 1, 2) and cfg["persistent"] in (0, 1)
    assert ctx.svr_get_config()["tile"] == cfg["tile"]
    cfg2, times2 = ctx.svr_autotune(*dev, gp, flags=flags, cache_path=cache)
    assert cfg2 == cfg and times2 == []  # answered from the cache
    out = _run(ctx, prob, params, pose, target)
    ref = _oracle(prob, params, pose, target)
    ctx.svr_set_config(tile=16, batch=128, persistent=0, cutoff=3.0, forward_mode=1)  # the module's default
    _compare(out, ref)


def test_radix_sort_matches_stable_argsort(ctx):
    """The binning sort is a stable LSD radix sort: bit-exact against numpy's
    stable argsort, for key widths that take one to four passes of 8- or
    9-bit digits, sizes spanning many blocks with a ragged tail, and heavy
    key duplication.  Bits above key_bits are ignored (cases with "hi"): the
    order is that of the low bits, and the keys travel unchanged."""
    rng = np.random.default_rng(0)
    cases = [(1, 8, False), (5000, 3, False), (4096 * 7 + 123, 15, False), (300001, 20, False),
             (70000, 32, False), (100, 9, False), (200003, 19, False), (90001, 11, False),
             (150000, 30, False), (4096 * 3 + 17, 16, True), (100000, 19, True), (5000, 5, True),
             (100000, 17, False), (4096 * 5 + 1, 18, True), (3000, 9, True)]
    for n, bits, high in cases:
        hi = 2 ** bits
        keys = rng.integers(0, min(hi, 2**32 - 1), size=n, dtype=np.uint64).astype(np.uint32)
        if n > 1000:
            keys[: n // 3] = keys[0]
        if high:
            keys |= rng.integers(0, 2**32 - 1, size=n, dtype=np.uint64).astype(np.uint32) & ~np.uint32(hi - 1)
            keys[rng.integers(0, n, size=max(n // 50, 1))] = 0xFFFFFFFF
        vals = np.arange(n, dtype=np.uint32)
        k = torch.from_numpy(keys.view(np.int32).copy()).cuda()
        v = torch.from_numpy(vals.view(np.int32).copy()).cuda()
        ctx.svr_sort_pairs(k, v, bits)
        torch.cuda.synchronize()
        low = keys & np.uint32(hi - 1) if bits < 32 else keys
        order = np.argsort(low, kind="stable")
        assert np.array_equal(k.cpu().numpy().view(np.uint32), keys[order]), (n, bits, high)
        assert np.array_equal(v.cpu().numpy().view(np.uint32), vals[order]), (n, bits, high)


def test_adam_step_matches_oracle(ctx):
    prob = synth.config1(0, n_gauss=500, n_per_stack=3)
    ctx.svr_set_geometry(prob)
    N, M = prob.n_gauss, prob.n_slices
    rng = np.random.default_rng(4)
    p = svr.Params.from_arrays(*synth.perturb_params(prob, 2), prob.pose)
    p0 = p.flat.cpu().numpy().astype(np.float64)
    m = torch.zeros_like(p.flat)
    v = torch.zeros_like(p.flat)
    lr = [2.5e-2, 2.5e-2, 1e-2, 1e-2, 2.5e-3, 1e-1]
    lr_vec = np.concatenate([np.full(3 * N, lr[0]), np.full(3 * N, lr[1]), np.full(4 * N, lr[2]),
                             np.full(N, lr[3]), np.tile([lr[4]] * 3 + [lr[5]] * 3, M)])
    mo, vo, po = np.zeros_like(p0), np.zeros_like(p0), p0.copy()
    for step in range(1, 4):
        g = rng.standard_normal(p.flat.numel()).astype(np.float32)
        gt = svr.Params(N, M)
        gt.flat.copy_(torch.from_numpy(g))
        ctx.svr_step(p.views(), gt.views(), m, v, lr, step, weight_decay=0.01)
        po, mo, vo = oracle.adamw_step(po, g, mo, vo, step, lr_vec, wd=0.01)
    torch.cuda.synchronize()
    check_close(p.flat.cpu().numpy(), po, "params", rtol=1e-6)
    check_close(m.cpu().numpy(), mo, "exp_avg", rtol=1e-6)
    check_close(v.cpu().numpy(), vo, "exp_avg_sq", rtol=1e-5)


def test_autograd_function(ctx):
    """SvrRender behind torch.autograd: loss.backward() gives the oracle gradient."""
    prob = synth.config1(0, n_gauss=600, n_per_stack=4)
    params, pose, target = _setup(prob, seed=21)
    ctx.svr_set_config(tile=16, batch=128, persistent=0, cutoff=3.0)
    ctx.svr_set_geometry(prob)
    dev = [t.clone().requires_grad_(True) for t in gpu_params(params, pose)]
    loss, pred = svr.render_loss(ctx, *dev, to_dev(target), to_dev(prob.mask))
    (3.0 * loss).backward()
    ref = _oracle(prob, params, pose, target)
    assert abs(loss.item() - ref["loss"]) <= 1e-4 * ref["loss"]
    core, bnd = ref["grad_band"]
    for k, t in zip(("mean", "log_scale", "quat", "amp", "pose"), dev):
        print(check_band(t.grad.cpu().numpy(), 3.0 * core[k], 3.0 * bnd[k], k))


# --------------------------------------------------------------- full size ---
# The full workloads in the launch configurations the benchmark uses.  The
# oracle (FP64, OpenMP) is fast enough to evaluate every pixel and every
# gradient at these sizes, so every output block is compared in full.


@pytest.fixture(scope="module")
def head_full():
    prob = synth.config2(0)
    target = synth.head_observation(prob, 5, thickness_samples=3)
    params = synth.perturb_params(prob, 7, d_mu=0.2, d_ls=0.05, d_q=0.05, d_c=0.02)
    pose = np.zeros((prob.n_slices, 6), np.float32)      # identity pose initialisation
    ref = _oracle(prob, params, pose, target)
    return prob, params, pose, target, ref


@pytest.mark.parametrize("cfg", BENCH_CONFIGS, ids=BENCH_CONFIG_IDS)
def test_head_full_size_parity(ctx, head_full, cfg):
    """Head phantom at full size: 500k Gaussians, 128 slices of 256x256."""
    prob, params, pose, target, ref = head_full
    out = _run(ctx, prob, params, pose, target, cfg=cfg)
    _compare(out, ref)


@pytest.fixture(scope="module")
def stress_full():
    prob = synth.config3(0)
    params = synth.perturb_params(prob, 3, d_mu=0.1, d_ls=0.03, d_q=0.03, d_c=0.01)
    pose = prob.pose + np.random.default_rng(4).normal(0, 0.002, prob.pose.shape).astype(np.float32)
    target = (0.6 * prob.mask + synth.gaussian_noise(8, prob.n_pixels, 0.05)).astype(np.float32)
    ref = _oracle(prob, params, pose, target)
    return prob, params, pose, target, ref


@pytest.mark.parametrize("cfg", BENCH_CONFIGS[:2], ids=BENCH_CONFIG_IDS[:2])
def test_stress_full_size_parity(ctx, stress_full, cfg):
    """Differentiation stress at full size: 1.2M Gaussians, 240 slices of
    320x320 with interleaved motion segments; all 240 six-DoF pose gradients."""
    prob, params, pose, target, ref = stress_full
    out = _run(ctx, prob, params, pose, target, cfg=cfg)
    _compare(out, ref)


# --------------------------------------------------- the paper's objective ---

def test_l1_data_term_matches_oracle(ctx):
    """Eq. 7's L1 term (SVR_LOSS_L1): loss, per-slice sums and the subgradient
    m sign(y - I) against the oracle.  The sign is decided in each side's own
    precision; it may differ only where the oracle's |y - I| is within the
    forward's FP32 error."""
    prob = synth.config1(0, n_gauss=1200)
    params, pose, target = _setup(prob, seed=21)
    ctx.svr_set_loss(svr.SVR_LOSS_L1)
    try:
        out = _run(ctx, prob, params, pose, target,
                   cfg=dict(tile=16, batch=128, persistent=0, cutoff=3.0, forward_mode=1))
    finally:
        ctx.svr_set_loss(svr.SVR_LOSS_MSE)
    y = oracle.forward(prob, 3.0, params=params, pose=pose)
    loss, g, per_slice = oracle.masked_l1(y, target, prob.mask, prob.pix_offset)
    assert abs(out["loss"] - loss) <= 1e-4 * abs(loss), (out["loss"], loss)
    print(check_close(out["sse"], per_slice, "per-slice L1"))
    r = np.abs(y - target)
    undecided = r <= 1e-5 * np.abs(y).max()
    mism = (out["gpred"] != g) & ~undecided
    assert not mism.any(), np.nonzero(mism)[0][:10]
    assert np.all(np.isin(out["gpred"], (-1.0, 0.0, 1.0)))


def test_scale_regularizer_matches_oracle(ctx):
    """Eq. 7's regulariser: value added to the loss and gradient added to the
    log-scale gradient, against the oracle."""
    rng = np.random.default_rng(22)
    n = 70001
    ls = rng.uniform(np.log(0.3), np.log(3.0), size=(n, 3)).astype(np.float32)
    g0 = rng.standard_normal((n, 3)).astype(np.float32)
    val, g = oracle.scale_regularizer(ls.astype(np.float64), 2.5e-3, 1.6)
    lsd, gd = to_dev(ls), to_dev(g0)
    loss = torch.tensor([0.25], device="cuda")
    ctx.svr_scale_regularizer(lsd, 2.5e-3, 1.6, gd, loss)
    torch.cuda.synchronize()
    assert abs(loss.item() - (0.25 + val)) <= 1e-4 * (0.25 + val)
    print(check_close(gd.cpu().numpy() - g0, g, "regulariser gradient"))
    with pytest.raises(svr.SvrError):
        ctx.svr_scale_regularizer(lsd, -1.0, 1.6, gd, loss)
