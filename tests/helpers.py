"""Shared test helpers: tolerance checks and marshalling of seeded problems.

Parity bar for floating-point outputs (GPU FP32 against the FP64 oracle),
applied per output block:
  norm-wise     ||gpu - ora||_2 <= RTOL ||ora||_2
  element-wise  |gpu - ora| <= RTOL |ora| + RTOL max|ora|
with RTOL = 1e-4.  A pure element-wise relative bound is ill-posed where the
reference is ~0 (background pixels, cancelling gradients), hence the floor
tied to the block's largest magnitude.
"""
import numpy as np

RTOL = 1e-4


def check_close(gpu, ora, name, rtol=RTOL, atol_frac=None):
    gpu = np.asarray(gpu, np.float64).ravel()
    ora = np.asarray(ora, np.float64).ravel()
    assert gpu.shape == ora.shape, (name, gpu.shape, ora.shape)
    assert np.all(np.isfinite(gpu)), f"{name}: non-finite GPU values"
    scale = np.abs(ora).max() if ora.size else 0.0
    atol_frac = rtol if atol_frac is None else atol_frac
    diff = np.abs(gpu - ora)
    nrm = np.linalg.norm(gpu - ora)
    ref = np.linalg.norm(ora)
    bad = diff > rtol * np.abs(ora) + atol_frac * scale
    info = (f"{name}: norm err {nrm / max(ref, 1e-300):.3e}, max abs {diff.max() if diff.size else 0:.3e}, "
            f"scale {scale:.3e}, bad {int(bad.sum())}/{bad.size}")
    assert nrm <= rtol * ref + 1e-30, info
    assert not bad.any(), info
    return info


def to_dev(a, dtype=None):
    import torch
    t = torch.as_tensor(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.to("cuda").contiguous()


def gpu_params(params, pose):
    import torch
    mean, ls, q, c = params
    return (to_dev(mean, torch.float32), to_dev(ls, torch.float32), to_dev(q, torch.float32),
            to_dev(c, torch.float32), to_dev(pose, torch.float32))


# Launch configurations the benchmark and the full-size parity tests use.  The
# first is bench.py's default (tile 32, record-per-lane forward over fixed
# chunks of the tile-ordered instance list); tests/test_bench_host.py checks
# that bench.py's defaults stay in this list.
BENCH_CONFIGS = [dict(tile=32, batch=128, persistent=0, cutoff=3.0, forward_mode=1),
                 dict(tile=16, batch=128, persistent=0, cutoff=3.0, forward_mode=1),
                 dict(tile=32, batch=128, persistent=1, cutoff=3.0, forward_mode=2),
                 dict(tile=16, batch=128, persistent=1, cutoff=3.0, forward_mode=0)]
BENCH_CONFIG_IDS = ["tile32-rpl-chunked", "tile16-rpl-chunked", "tile32-rol-persistent", "tile16-pixel-persistent"]


BAND = 1e-4  # relative half-width of q around the cut treated as undecided


def check_band(gpu, core, bnd, name, rtol=RTOL):
    """Like check_close, against the oracle's band split: pairs whose q lies
    within BAND*T^2 of the cut may be decided either way by FP32, so their
    absolute contributions ``bnd`` widen the bound element by element."""
    gpu = np.asarray(gpu, np.float64).ravel()
    core = np.asarray(core, np.float64).ravel()
    bnd = np.asarray(bnd, np.float64).ravel()
    assert gpu.shape == core.shape == bnd.shape, name
    assert np.all(np.isfinite(gpu)), f"{name}: non-finite GPU values"
    scale = np.abs(core).max() if core.size else 0.0
    diff = np.abs(gpu - core)
    bad = diff > rtol * np.abs(core) + rtol * scale + bnd
    nrm, ref = np.linalg.norm(gpu - core), np.linalg.norm(core)
    info = (f"{name}: norm err {nrm / max(ref, 1e-300):.3e}, max abs {diff.max() if diff.size else 0:.3e}, "
            f"scale {scale:.3e}, band-bounded {int((bnd > 0).sum())}, bad {int(bad.sum())}/{bad.size}")
    assert nrm <= rtol * ref + np.linalg.norm(bnd) + 1e-30, info
    assert not bad.any(), info
    return info
