"""GPU tests of the reconstruction driver: the volume read-out against the
oracle (zero PSF = point sampling of V), PSNR, and a short fit."""
import math

import numpy as np
import pytest

from helpers import BAND, check_band
from paper_2512_11624_amd import synth

pytestmark = pytest.mark.gpu
torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

import oracle  # noqa: E402
from paper_2512_11624_amd import recon, svr  # noqa: E402


def _grid_problem(prob, shape, h):
    g = recon.volume_grid(shape, h)
    return synth.Problem(prob.mean, prob.log_scale, prob.quat, prob.amp, prob.gauss_offsets, g.slice_subject,
                         g.height, g.width, g.spacing, g.psf_fwhm, g.rot0, g.trans0, g.pose, g.mask)


def test_volume_readout_matches_oracle():
    """The read-out is the forward model with zero PSF on grid planes; the
    oracle's zero-PSF forward is pinned to point sampling of V (P4)."""
    prob = synth.config1(0, n_gauss=700)
    shape, h = (24, 20, 22), 0.5
    gp = _grid_problem(prob, shape, h)
    core, bnd = oracle.forward_band(gp, 3.0, BAND)
    probe = recon.VolumeProbe(prob.n_gauss, shape, h, (0, 0, 0), np.zeros(gp.n_pixels), np.ones(gp.n_pixels))
    dev = [torch.as_tensor(a).cuda() for a in prob.params()]
    vol = probe.render(*dev).cpu().numpy()
    print(check_band(vol, core, bnd, "volume"))
    probe.close()


def test_psnr_against_oracle_definition():
    prob = synth.config1(0, n_gauss=500)
    shape, h = (16, 16, 16), 0.5
    gp = _grid_problem(prob, shape, h)
    gt = oracle.forward(gp, np.inf)
    mask = (np.random.default_rng(0).uniform(size=gt.size) < 0.8).astype(np.float32)
    params = synth.perturb_params(prob, 1, d_mu=0.1, d_ls=0.05, d_q=0.05, d_c=0.05)
    y = oracle.forward(gp, 3.0, params=params)
    mse = np.sum(mask * (y - gt) ** 2) / mask.sum()
    ref = 10 * math.log10(gt[mask > 0].max() ** 2 / mse)
    probe = recon.VolumeProbe(prob.n_gauss, shape, h, (0, 0, 0), gt, mask)
    got = probe.psnr(*[torch.as_tensor(a).cuda() for a in params])
    assert abs(got - ref) < 1e-3, (got, ref)   # 1e-4 relative on the MSE is ~4e-4 dB
    probe.close()


def test_short_fit_improves_psnr():
    """A short fit from perturbed Gaussians and identity poses raises the
    cube's PSNR and lowers the loss."""
    prob = synth.config1(0)
    target = (oracle.forward(prob, np.inf) + synth.gaussian_noise(1, prob.n_pixels, 0.01)).astype(np.float32)
    shape, h = (64, 64, 64), 0.5
    gp = _grid_problem(prob, shape, h)
    gt = oracle.forward(gp, np.inf)
    c = recon.voxel_centres(shape, h)
    vmask = np.all(np.abs(c) <= 16.0, axis=1).astype(np.float32)
    probe = recon.VolumeProbe(prob.n_gauss, shape, h, (0, 0, 0), gt, vmask)
    ctx = svr.Context(0)
    ctx.svr_set_config(tile=16, batch=128, persistent=0, cutoff=3.0, forward_mode=2)
    ctx.svr_set_geometry(prob)
    init = synth.perturb_params(prob, 3, d_mu=0.5, d_ls=0.2, d_q=0.2, d_c=0.2)
    params = svr.Params.from_arrays(*init, np.zeros((prob.n_slices, 6), np.float32))
    p0 = probe.psnr(*params.views()[:4])
    res = recon.fit(ctx, params, torch.as_tensor(target).cuda(), torch.as_tensor(prob.mask).cuda(), 150,
                    probe=probe, psnr_every=50)
    print("psnr", p0, res.psnr, "loss", res.loss, "seconds", res.seconds)
    assert res.final_psnr > p0 + 1.0
    assert res.loss[-1] < res.loss[0]
    probe.close()
    ctx.close()
