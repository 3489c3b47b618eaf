"""Densification (svr_densify_accumulate / svr_densify) against the oracle
(oracle/densify.py): the statistic, the selected set and the layout bit for
bit (ties planted at every threshold), the children to FP32 rounding, the
optimiser moments exactly, the context taking the new mixture (its forward
against the oracle's forward of the oracle's densified mixture), the
capacity error, an empty subject, everything pruned, and the selection at
the 500k-Gaussian head size."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

import oracle  # noqa: E402
from oracle import densify as od  # noqa: E402
from helpers import BAND, check_band, check_close, gpu_params, to_dev  # noqa: E402
from paper_2512_11624_amd import svr, synth  # noqa: E402

CFG = dict(grad_threshold=0.5, log_scale_threshold=0.25, split_offset=float(np.sqrt(3.0) / 2.0), clone_offset=0.5,
           prune_amp=0.05)


def _statistic(n, seed, thr=0.5):
    """Seeded (A, n) with ties planted: A = thr * n exactly, one ulp above, unseen Gaussians."""
    rng = np.random.default_rng(seed)
    cnt = rng.integers(0, 9, n).astype(np.int32)
    acc = (rng.uniform(0.0, 1.0, n) * cnt).astype(np.float32)
    tie = rng.random(n) < 0.1
    acc[tie] = (np.float32(thr) * cnt[tie].astype(np.float32)).astype(np.float32)
    up = rng.random(n) < 0.05
    acc[up] = np.nextafter(np.float32(thr) * cnt[up].astype(np.float32), np.float32(np.inf)).astype(np.float32)
    return acc, cnt


def _params(prob, seed):
    mean, ls, q, amp = synth.perturb_params(prob, seed)
    rng = np.random.default_rng(seed + 7)
    n = len(amp)
    ls = ls.copy()
    amp = amp.copy()
    at = rng.random(n) < 0.05                               # largest log-scale exactly at the threshold
    ls[at, 0] = np.float32(0.25)
    ls[at, 1:] = np.minimum(ls[at, 1:], np.float32(0.2))
    amp[rng.random(n) < 0.03] = np.float32(0.05)            # |c| exactly at the prune bound: kept
    amp[rng.random(n) < 0.03] = np.float32(0.01)            # pruned
    return mean, ls, q, amp


def _run(ctx, prob, params, acc, cnt, cfg=CFG, moments=True, capacity=None):
    N, M = prob.n_gauss, prob.n_slices
    cap = 2 * N if capacity is None else capacity
    out = [torch.full((cap * w,), np.nan, device="cuda") for w in (3, 3, 4, 1)]
    src = torch.full((max(cap, 1),), -7, dtype=torch.int32, device="cuda")
    rng = np.random.default_rng(3)
    m_in = [to_dev(rng.normal(size=11 * N + 6 * M).astype(np.float32)) for _ in range(2)]
    m_out = [torch.full((11 * cap + 6 * M,), np.nan, device="cuda") for _ in range(2)]
    dev = [to_dev(a) for a in params]
    off = ctx.svr_densify(dev, to_dev(acc), to_dev(cnt), cfg, out, cap, src,
                          m_in if moments else None, m_out if moments else None)
    K = int(off[-1])
    torch.cuda.synchronize()
    res = dict(offsets=off, src=src[:K].cpu().numpy(), mean=out[0][:3 * K].cpu().numpy().reshape(-1, 3),
               log_scale=out[1][:3 * K].cpu().numpy().reshape(-1, 3), quat=out[2][:4 * K].cpu().numpy().reshape(-1, 4),
               amp=out[3][:K].cpu().numpy(), dev=[t[:w * K] for t, w in zip(out, (3, 3, 4, 1))])
    if moments:
        res["m_in"] = [t.cpu().numpy() for t in m_in]
        res["m_out"] = [t[:11 * K + 6 * M].cpu().numpy() for t in m_out]
    return res


def _compare(res, ref, params):
    assert np.array_equal(res["offsets"], ref["offsets"]), (res["offsets"], ref["offsets"])
    assert np.array_equal(res["src"], ref["src"])
    keep = res["src"] >= 0
    for k, a in zip(("mean", "log_scale", "quat", "amp"), params):
        assert np.array_equal(res[k][keep], np.asarray(a)[res["src"][keep]]), k    # copies are exact
        print(check_close(res[k][~keep], ref[k][~keep], k + " (children)"))
    assert np.isfinite(res["mean"]).all()


def test_accumulate_two_steps():
    prob = synth.config1(0, n_gauss=3000)
    ctx = svr.Context(0)
    ctx.svr_set_geometry(prob)
    rng = np.random.default_rng(1)
    acc = np.zeros(prob.n_gauss, np.float32)
    cnt = np.zeros(prob.n_gauss, np.int32)
    a_d, c_d = to_dev(acc), to_dev(cnt)
    for step in range(2):
        g = rng.normal(size=(prob.n_gauss, 3)).astype(np.float32)
        g[rng.random(prob.n_gauss) < 0.3] = 0.0
        g[rng.random(prob.n_gauss) < 0.02, 1] = 1e-30       # squares underflow in FP32; still counted
        ctx.svr_densify_accumulate(to_dev(g), a_d, c_d)
        acc, cnt = od.accumulate(acc, cnt, g)
    torch.cuda.synchronize()
    assert np.array_equal(c_d.cpu().numpy(), cnt)
    print(check_close(a_d.cpu().numpy(), acc, "grad_acc"))
    ctx.close()


@pytest.mark.parametrize("split_offset", [float(np.sqrt(3.0) / 2.0), 0.6])
def test_densify_cube_matches_oracle(split_offset):
    prob = synth.config1(1, n_gauss=4000)
    params = _params(prob, 11)
    acc, cnt = _statistic(prob.n_gauss, 12)
    cfg = dict(CFG, split_offset=split_offset)
    ctx = svr.Context(0)
    ctx.svr_set_geometry(prob)
    res = _run(ctx, prob, params, acc, cnt, cfg)
    ref = od.densify(prob.gauss_offsets, *params, acc, cnt, cfg, exp_avg=res["m_in"][0], exp_avg_sq=res["m_in"][1])
    n_out = ref["n_out"]
    print("kept", int((n_out == 1).sum()), "densified", int((n_out == 2).sum()), "pruned", int((n_out == 0).sum()),
          "split", int(ref["split"].sum()))
    assert (n_out == 2).sum() > 100 and (n_out == 0).sum() > 50 and ref["split"].sum() > 20
    _compare(res, ref, params)
    assert np.array_equal(res["m_out"][0], ref["exp_avg"])
    assert np.array_equal(res["m_out"][1], ref["exp_avg_sq"])
    assert ctx.n_gauss == int(ref["offsets"][-1])
    ctx.close()


def test_context_takes_the_new_mixture_and_forward_matches():
    subs = [synth.config1(s, n_gauss=300 + 100 * s, n_per_stack=4 + 2 * s) for s in range(3)]
    prob = synth.concat(subs)
    params = _params(prob, 21)
    acc, cnt = _statistic(prob.n_gauss, 22)
    ctx = svr.Context(0)
    ctx.svr_set_config(tile=16, batch=128, persistent=0, cutoff=3.0, forward_mode=1)
    ctx.svr_set_geometry(prob)
    res = _run(ctx, prob, params, acc, cnt, moments=False)
    ref = od.densify(prob.gauss_offsets, *params, acc, cnt, CFG)
    _compare(res, ref, params)
    new = synth.Problem(*[ref[k].astype(np.float32) for k in ("mean", "log_scale", "quat", "amp")],
                        ref["offsets"], prob.slice_subject, prob.height, prob.width, prob.spacing, prob.psf_fwhm,
                        prob.rot0, prob.trans0, prob.pose, prob.mask)
    pose = to_dev(prob.pose)
    ctx.svr_project_bin(*res["dev"], pose)
    pred = torch.empty(prob.n_pixels, device="cuda")
    ctx.svr_forward(pred)
    torch.cuda.synchronize()
    yc, yb = oracle.forward_band(new, 3.0, BAND)
    print(check_band(pred.cpu().numpy(), yc, yb, "pred of the densified mixture"))
    ctx.close()


def test_capacity_error_leaves_the_context_unchanged():
    prob = synth.config1(2, n_gauss=1000)
    params = _params(prob, 31)
    acc, cnt = _statistic(prob.n_gauss, 32)
    ref = od.densify(prob.gauss_offsets, *params, acc, cnt, CFG)
    K = int(ref["offsets"][-1])
    ctx = svr.Context(0)
    ctx.svr_set_config(tile=16, batch=128, persistent=0, cutoff=3.0, forward_mode=1)
    ctx.svr_set_geometry(prob)
    dev = gpu_params(params, prob.pose)
    pred0 = torch.empty(prob.n_pixels, device="cuda")
    ctx.svr_project_bin(*dev)
    ctx.svr_forward(pred0)
    with pytest.raises(svr.SvrError) as e:
        _run(ctx, prob, params, acc, cnt, capacity=K - 1)
    assert e.value.status == svr.SVR_ERR_CAPACITY
    assert np.array_equal(e.value.offsets, ref["offsets"])
    pred1 = torch.empty(prob.n_pixels, device="cuda")
    ctx.svr_project_bin(*dev)                                 # the old mixture still binds
    ctx.svr_forward(pred1)
    torch.cuda.synchronize()
    assert torch.equal(pred0, pred1)
    with pytest.raises(svr.SvrError):
        ctx.svr_densify([d for d in dev[:4]], to_dev(acc), to_dev(cnt), dict(CFG, split_offset=1.0),
                        [torch.empty(1, device="cuda")] * 4, 2 * prob.n_gauss)
    ctx.close()


def test_empty_subject_and_everything_pruned():
    subs = [synth.config1(s, n_gauss=200, n_per_stack=4) for s in range(3)]
    cat = synth.concat(subs)
    keep = np.r_[0:200, 400:600]                              # subject 1 has slices but no Gaussians
    go = np.array([0, 200, 200, 400], np.int64)
    prob = synth.Problem(cat.mean[keep], cat.log_scale[keep], cat.quat[keep], cat.amp[keep], go, cat.slice_subject,
                         cat.height, cat.width, cat.spacing, cat.psf_fwhm, cat.rot0, cat.trans0, cat.pose, cat.mask)
    params = _params(prob, 41)
    acc, cnt = _statistic(prob.n_gauss, 42)
    ctx = svr.Context(0)
    ctx.svr_set_geometry(prob)
    res = _run(ctx, prob, params, acc, cnt)
    ref = od.densify(go, *params, acc, cnt, CFG, exp_avg=res["m_in"][0], exp_avg_sq=res["m_in"][1])
    _compare(res, ref, params)
    assert res["offsets"][1] == res["offsets"][2]
    assert np.array_equal(res["m_out"][0], ref["exp_avg"])
    # now prune everything: K = 0, the context holds no Gaussians
    dev = [to_dev(ref[k].astype(np.float32)) for k in ("mean", "log_scale", "quat", "amp")]
    K = int(ref["offsets"][-1])
    off = ctx.svr_densify(dev, torch.zeros(K, device="cuda"), torch.zeros(K, dtype=torch.int32, device="cuda"),
                          dict(CFG, prune_amp=1e30), [torch.empty(1, device="cuda")] * 4, 0)
    assert off.tolist() == [0, 0, 0, 0]
    assert ctx.n_gauss == 0
    ctx.close()


def test_head_size_selection():
    prob = synth.config2(0)
    params = _params(prob, 51)
    acc, cnt = _statistic(prob.n_gauss, 52)
    ctx = svr.Context(0)
    ctx.svr_set_geometry(prob)
    res = _run(ctx, prob, params, acc, cnt, moments=False)
    n_out, split = od.decide(acc, cnt, params[1], params[3], **CFG)
    off = np.concatenate([[0], np.cumsum(n_out)])
    assert np.array_equal(res["offsets"], off[prob.gauss_offsets])
    j = np.arange(prob.n_gauss)
    src = np.repeat(np.where(n_out == 1, j, -(j + 1)), n_out)
    assert np.array_equal(res["src"], src)
    # children of a sample of parents against the oracle's
    par = np.nonzero(n_out == 2)[0]
    pick = np.random.default_rng(53).choice(par, 2000, replace=False)
    (cm, cp), cls, _, ca = od.children(*[np.asarray(a)[pick] for a in params], split[pick], **CFG)
    where = off[pick]
    print(check_close(res["mean"][where], cm, "head children -"), check_close(res["mean"][where + 1], cp,
                                                                            "head children +"))
    print(check_close(res["log_scale"][where], cls, "head children log_scale"),
          check_close(res["amp"][where + 1], ca, "head children amp"))
    ctx.close()
