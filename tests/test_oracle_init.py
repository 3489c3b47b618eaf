"""Pins of the content-adaptive initialisation oracle (Sec. 2.5, Eq. 6)
against closed forms, a library routine, brute force and the sampling law."""
import numpy as np
import pytest
from scipy import stats

import oracle
from paper_2512_11624_amd import synth


def _ramp_problem(alpha, beta):
    p = synth.tiny(3, n_slices=3, size=(7, 9), spacing=(0.8, 1.3))
    img = np.empty(p.n_pixels)
    po = p.pix_offset
    for i in range(p.n_slices):
        h, w = int(p.height[i]), int(p.width[i])
        rr, cc = np.mgrid[0:h, 0:w]
        img[po[i]:po[i + 1]] = (alpha * cc * p.spacing[i, 0] + beta * rr * p.spacing[i, 1] + 0.5).ravel()
    return p, img


def test_gradient_of_a_ramp_is_its_slope():
    # I = alpha x + beta y (x, y in mm): ||grad I|| = sqrt(alpha^2 + beta^2)
    # everywhere, border pixels included.
    p, img = _ramp_problem(0.3, -0.7)
    g = oracle.gradient_magnitude(img, p.height, p.width, p.spacing, p.pix_offset)
    assert np.allclose(g, np.hypot(0.3, 0.7), rtol=1e-12)


def test_gradient_matches_numpy_gradient():
    rng = np.random.default_rng(0)
    p = synth.tiny(4, n_slices=3, size=(6, 10), spacing=(0.7, 1.9))
    img = rng.standard_normal(p.n_pixels)
    g = oracle.gradient_magnitude(img, p.height, p.width, p.spacing, p.pix_offset)
    po = p.pix_offset
    for i in range(p.n_slices):
        sl = img[po[i]:po[i + 1]].reshape(int(p.height[i]), int(p.width[i]))
        gy, gx = np.gradient(sl, float(p.spacing[i, 1]), float(p.spacing[i, 0]), edge_order=1)
        assert np.allclose(g[po[i]:po[i + 1]], np.hypot(gx, gy).ravel(), rtol=1e-13, atol=0)


def test_gradient_of_a_single_row_or_column():
    p = synth.tiny(5, n_slices=2, size=(1, 8), spacing=(0.5, 1.0))
    img = np.tile(np.arange(8.0) ** 2, 2)
    g = oracle.gradient_magnitude(img, p.height, p.width, p.spacing, p.pix_offset)
    ref = np.abs(np.gradient(np.arange(8.0) ** 2, 0.5))
    assert np.allclose(g, np.tile(ref, 2), rtol=1e-14)


def test_weights_uniform_and_gradient_limits():
    p = synth.config1(0, n_gauss=100, size=16, n_per_stack=4)
    img = synth.textured_image(p, 1)
    p.mask[: 300] = 0.0
    w1 = oracle.sampling_weights(p, img, 1.0)
    assert np.array_equal(w1, np.where(p.mask > 0, 2 ** 20, 0))
    w0 = oracle.sampling_weights(p, img, 0.0)
    g = oracle.gradient_magnitude(img, p.height, p.width, p.spacing, p.pix_offset)
    m = p.mask > 0
    assert w0[m].max() == 2 ** 20 and w0[~m].max() == 0
    assert np.argmax(np.where(m, g, -1)) == np.argmax(w0)
    # mixture is monotone in the gradient and floored at lambda
    wh = oracle.sampling_weights(p, img, 0.25)
    assert wh[m].min() >= int(0.25 * 2 ** 20)
    order = np.argsort(g[m], kind="stable")
    assert np.all(np.diff(wh[m][order]) >= 0)


def test_constant_subject_falls_back_to_uniform():
    p = synth.tiny(6, n_slices=2)
    w = oracle.sampling_weights(p, np.full(p.n_pixels, 0.4), 0.0)
    assert np.all(w == 0)
    w = oracle.sampling_weights(p, np.full(p.n_pixels, 0.4), 0.5)
    assert np.array_equal(w, np.where(p.mask > 0, 2 ** 19, 0))


def test_cdf_restarts_per_subject():
    a, b = synth.tiny(1, n_slices=2), synth.tiny(2, n_slices=3)
    p = synth.concat([a, b])
    img = synth.textured_image(p, 3)
    c = oracle.sampling_cdf(p, img, 0.1)
    ca = oracle.sampling_cdf(a, img[: a.n_pixels], 0.1)
    cb = oracle.sampling_cdf(b, img[a.n_pixels:], 0.1)
    assert np.array_equal(c, np.concatenate([ca, cb]))


def test_draw_is_the_brute_force_inverse_cdf():
    # first pixel whose cumulative weight exceeds floor(u0 W), by a scan
    p = synth.tiny(7, n_gauss=200, n_slices=3)
    img = synth.textured_image(p, 4)
    u = synth.init_uniforms(5, p.n_gauss)
    _, pix, val = oracle.adaptive_means(p, img, p.pose, u, 0.2)
    w = oracle.sampling_weights(p, img, 0.2)
    W = int(w.sum())
    for j in range(p.n_gauss):
        t = int(np.floor(float(u[j, 0]) * W))
        run, k = 0, 0
        while run + w[k] <= t:
            run += w[k]
            k += 1
        assert pix[j] == k and w[k] > 0
    assert np.array_equal(val, img[pix])


def test_draw_frequencies_follow_the_weights():
    p = synth.tiny(8, n_gauss=40000, n_slices=1, size=(4, 5))
    img = synth.textured_image(p, 6)
    p.mask[[3, 11]] = 0.0
    u = synth.init_uniforms(9, p.n_gauss)
    _, pix, _ = oracle.adaptive_means(p, img, p.pose, u, 0.3)
    w = oracle.sampling_weights(p, img, 0.3).astype(np.float64)
    counts = np.bincount(pix, minlength=p.n_pixels)
    assert counts[3] == 0 and counts[11] == 0
    keep = w > 0
    chi2 = stats.chisquare(counts[keep], w[keep] / w.sum() * p.n_gauss)
    assert chi2.pvalue > 1e-3


def test_centre_offsets_land_on_pixel_centres():
    # u1 = u2 = u3 = 1/2: the mean is the pixel centre under the pose
    p = synth.tiny(10, n_gauss=50, n_slices=3, max_deg=20.0, max_mm=2.0)
    img = synth.textured_image(p, 7)
    u = synth.init_uniforms(11, p.n_gauss)
    u[:, 1:] = 0.5
    mean, pix, _ = oracle.adaptive_means(p, img, p.pose, u, 0.0)
    centres = np.concatenate(synth.pixel_world_positions(p.rot0, p.trans0, p.pose.astype(np.float64),
                                                         p.height, p.width, p.spacing))
    assert np.allclose(mean, centres[pix], atol=1e-12)


def test_offsets_stay_inside_the_pixel_and_slab():
    p = synth.tiny(12, n_gauss=300, n_slices=2, max_deg=20.0)
    img = synth.textured_image(p, 8)
    u = synth.init_uniforms(13, p.n_gauss)
    mean, pix, _ = oracle.adaptive_means(p, img, p.pose, u, 0.0)
    centres = np.concatenate(synth.pixel_world_positions(p.rot0, p.trans0, p.pose.astype(np.float64),
                                                         p.height, p.width, p.spacing))
    sl = np.searchsorted(p.pix_offset, pix, side="right") - 1
    from scipy.spatial.transform import Rotation
    for j in range(p.n_gauss):
        i = sl[j]
        R = Rotation.from_rotvec(p.pose[i, :3].astype(np.float64)).as_matrix() @ p.rot0[i].reshape(3, 3)
        d = np.linalg.solve(R, mean[j] - centres[pix[j]])   # R0 is float32: not exactly orthonormal
        half = np.array([p.spacing[i, 0], p.spacing[i, 1], p.psf_fwhm[i, 2]], np.float64) / 2
        assert np.all(np.abs(d) <= half + 1e-12)
        assert np.allclose(d, (u[j, 1:].astype(np.float64) - 0.5) * 2 * half, rtol=0, atol=1e-12)


def test_subjects_draw_from_their_own_slices():
    a, b = synth.tiny(14, n_gauss=30, n_slices=2), synth.tiny(15, n_gauss=50, n_slices=2)
    p = synth.concat([a, b])
    img = synth.textured_image(p, 9)
    u = synth.init_uniforms(16, p.n_gauss)
    _, pix, _ = oracle.adaptive_means(p, img, p.pose, u, 0.0)
    assert np.all(pix[:30] < a.n_pixels) and np.all(pix[30:] >= a.n_pixels)


def test_subject_without_weight_is_rejected():
    p = synth.tiny(17, n_slices=2)
    p.mask[:] = 0.0
    with pytest.raises(ValueError):
        oracle.adaptive_means(p, synth.textured_image(p, 1), p.pose, synth.init_uniforms(1, p.n_gauss), 0.5)
