"""Pins of the FP64 oracle against what the paper and the mathematics fix.

Each test names the passage it follows.  None of them re-types the oracle's
own formulas: expectations come from quadrature of the acquisition integral
(Eq. 1), scipy's multivariate normal density, closed forms of special cases,
conservation laws, symmetries and finite differences.
"""
import math

import numpy as np
import pytest
from numpy.polynomial.hermite_e import hermegauss
from scipy.spatial.transform import Rotation
from scipy.stats import multivariate_normal

from paper_2512_11624_amd import synth


def _cov(quat_wxyz, log_scale):
    R = Rotation.from_quat(np.asarray(quat_wxyz, float)[[1, 2, 3, 0]]).as_matrix()
    return R @ np.diag(np.exp(2 * np.asarray(log_scale, float))) @ R.T


def _slice_frame(p, i, pose=None):
    pose = p.pose if pose is None else pose
    R = Rotation.from_rotvec(pose[i, :3].astype(float)).as_matrix() @ p.rot0[i].reshape(3, 3).astype(float)
    t = p.trans0[i].astype(float) + pose[i, 3:].astype(float)
    return R, t


def _pixel_world(p, i, r, k, pose=None):
    R, t = _slice_frame(p, i, pose)
    u = np.array([(k - (p.width[i] - 1) / 2) * p.spacing[i, 0], (r - (p.height[i] - 1) / 2) * p.spacing[i, 1], 0.0])
    return R @ u + t


def _psf_cov(p, i, pose=None):
    R, _ = _slice_frame(p, i, pose)
    sig = p.psf_fwhm[i].astype(float) / 2.355
    return R @ np.diag(sig ** 2) @ R.T


def _single(p, j):
    """Problem restricted to Gaussian j."""
    q = synth.Problem(p.mean[j:j + 1].copy(), p.log_scale[j:j + 1].copy(), p.quat[j:j + 1].copy(),
                      p.amp[j:j + 1].copy(), np.array([0, 1], np.int64), p.slice_subject, p.height,
                      p.width, p.spacing, p.psf_fwhm, p.rot0, p.trans0, p.pose, p.mask)
    return q


# ---------------------------------------------------------------- P1 -------
def test_p1_quadrature_of_acquisition_integral(oracle_lib):
    """Eq. 1 / Eq. 3: y(u) = int V(x) phi(x - T(u)) dx by tensor Gauss-Hermite
    quadrature in the PSF's Cholesky frame equals the oracle's exact model."""
    p = synth.tiny(3, n_gauss=3, n_slices=2, size=(5, 6))
    y = oracle_lib.forward(p, tau=np.inf)
    z, w = hermegauss(48)
    w = w / math.sqrt(2 * math.pi)
    Z = np.stack(np.meshgrid(z, z, z, indexing="ij"), -1).reshape(-1, 3)
    W = np.einsum("a,b,c->abc", w, w, w).ravel()
    po = p.pix_offset
    checked = 0
    for i in range(p.n_slices):
        L = np.linalg.cholesky(_psf_cov(p, i))
        for (r, k) in [(0, 0), (2, 3), (4, 5), (1, 4)]:
            x = _pixel_world(p, i, r, k)
            pts = x[None, :] + Z @ L.T
            val = 0.0
            for j in range(p.n_gauss):
                S = _cov(p.quat[j], p.log_scale[j])
                d = pts - p.mean[j].astype(float)
                val += float(p.amp[j]) * np.sum(W * np.exp(-0.5 * np.einsum("pa,ab,pb->p", d, np.linalg.inv(S), d)))
            got = y[po[i] + r * p.width[i] + k]
            assert abs(got - val) <= 1e-12 * max(1.0, abs(val)), (i, r, k, got, val)
            checked += 1
    assert checked == 8


# ---------------------------------------------------------------- P2 -------
def test_p2_covariance_addition_closed_form(oracle_lib):
    """Eq. 4 via a library density: c (2 pi)^(3/2) sqrt(det Sigma_j) N(x; mu, Sigma_j + R Sigma_PSF R^T)."""
    p = synth.tiny(11, n_gauss=5, n_slices=3, size=(7, 8))
    y = oracle_lib.forward(p, tau=np.inf)
    po = p.pix_offset
    for i in range(p.n_slices):
        P = _psf_cov(p, i)
        for pix in range(0, int(p.height[i] * p.width[i]), 5):
            r, k = divmod(pix, int(p.width[i]))
            x = _pixel_world(p, i, r, k)
            ref = 0.0
            for j in range(p.n_gauss):
                S = _cov(p.quat[j], p.log_scale[j])
                ref += float(p.amp[j]) * (2 * math.pi) ** 1.5 * math.sqrt(np.linalg.det(S)) * \
                    multivariate_normal.pdf(x, mean=p.mean[j].astype(float), cov=S + P)
            assert abs(y[po[i] + pix] - ref) <= 1e-12 * max(1.0, abs(ref))


# ---------------------------------------------------------------- P3 -------
def test_p3_isotropic_gaussian_radial_profile(oracle_lib):
    """A slice through one isotropic Gaussian with an in-plane isotropic PSF
    gives the closed radial profile c s^3/((s^2+a^2) sqrt(s^2+b^2)) exp(...)
    (Gaussian closure under convolution, Sec. 2.3) -- radially symmetric."""
    p = synth.tiny(5, n_gauss=1, n_slices=2, size=(21, 21), spacing=(0.5, 0.5))
    s = 1.3
    p.log_scale[:] = math.log(s)
    p.psf_fwhm[:] = np.array([1.1, 1.1, 3.0], np.float32)
    # exactly orthogonal (float64) slice rotations: the closed form assumes R^T R = I
    p.rot0 = Rotation.from_rotvec([[0.3, -0.5, 0.2], [-1.0, 0.4, 0.7]]).as_matrix().reshape(2, 9)
    p.pose = p.pose.astype(np.float64)
    y = oracle_lib.forward(p, tau=np.inf)
    po = p.pix_offset
    s = math.exp(float(p.log_scale[0, 0]))            # the stored (float32) value
    a, b = float(p.psf_fwhm[0, 0]) / 2.355, float(p.psf_fwhm[0, 2]) / 2.355
    for i in range(p.n_slices):
        R, t = _slice_frame(p, i)
        m = R.T @ (p.mean[0].astype(float) - t)          # Gaussian centre in slice frame
        vals, radii = [], []
        for r in range(21):
            for k in range(21):
                u = np.array([(k - 10) * 0.5, (r - 10) * 0.5])
                ref = float(p.amp[0]) * s ** 3 / ((s * s + a * a) * math.sqrt(s * s + b * b)) * math.exp(
                    -0.5 * (np.sum((u - m[:2]) ** 2) / (s * s + a * a) + m[2] ** 2 / (s * s + b * b)))
                got = y[po[i] + r * 21 + k]
                assert abs(got - ref) <= 1e-13 * max(1.0, abs(ref))
                vals.append(got); radii.append(np.linalg.norm(u - m[:2]))
        # symmetry: equal radii give equal values
        order = np.argsort(radii)
        rv, vv = np.array(radii)[order], np.array(vals)[order]
        close = np.abs(np.diff(rv)) < 1e-12
        assert np.all(np.abs(np.diff(vv)[close]) < 1e-13)


# ---------------------------------------------------------------- P4 -------
def test_p4_zero_psf_is_point_sampling(oracle_lib):
    """PSF -> 0: the slice samples V(x) = sum c exp(-1/2 d^T Sigma_j^-1 d) (Eq. 2 numerator)."""
    p = synth.tiny(7, n_gauss=4, n_slices=2, size=(6, 7))
    p.psf_fwhm[:] = 0.0
    y = oracle_lib.forward(p, tau=np.inf)
    po = p.pix_offset
    for i in range(p.n_slices):
        for pix in range(int(p.height[i] * p.width[i])):
            r, k = divmod(pix, int(p.width[i]))
            x = _pixel_world(p, i, r, k)
            ref = sum(float(p.amp[j]) * math.exp(-0.5 * (x - p.mean[j]) @ np.linalg.inv(_cov(p.quat[j], p.log_scale[j])) @ (x - p.mean[j]))
                      for j in range(p.n_gauss))
            assert abs(y[po[i] + pix] - ref) <= 1e-13 * max(1.0, abs(ref))


# ---------------------------------------------------------------- P5 -------
def test_p5_mass_conservation(oracle_lib):
    """The PSF is a normalised density (Sec. 2.3): summing slice signals over a
    fine stack recovers int V = c (2 pi)^(3/2) prod s for any PSF.  Eq. 5 as
    printed (no sqrt(det) factor) would not conserve mass."""
    base = synth.tiny(2, n_gauss=1, n_slices=1)
    h, n, w = 0.25, 128, 128
    orient = Rotation.from_rotvec([0.3, -0.2, 0.4]).as_matrix()
    normal = orient[:, 2]
    offs = (np.arange(n) - (n - 1) / 2) * h
    M = n
    p = synth.Problem(np.zeros((1, 3)), np.log(np.array([[0.9, 1.4, 2.0]])),
                      np.array([[0.8, 0.3, -0.4, 0.2]]), np.array([0.7]),
                      np.array([0, 1], np.int64), np.zeros(M, np.int32), np.full(M, w, np.int32),
                      np.full(M, w, np.int32), np.full((M, 2), h),
                      np.tile(np.array([1.0, 1.0, 3.0]), (M, 1)),
                      np.repeat(orient.reshape(1, 9), M, 0),
                      offs[:, None] * normal[None], np.zeros((M, 6)), np.ones(M * w * w))
    y = oracle_lib.forward(p, tau=np.inf)
    mass = y.sum() * h ** 3
    ref = 0.7 * (2 * math.pi) ** 1.5 * 0.9 * 1.4 * 2.0
    assert abs(mass - ref) <= 1e-9 * ref, (mass, ref)


# ---------------------------------------------------------------- P6 -------
def test_p6_linearity_in_amplitude(oracle_lib):
    """The model is linear in c_j (Eq. 5 numerator); dL/dc_j = <g, y^(j)>."""
    p = synth.tiny(13, n_gauss=5, n_slices=2)
    c1 = p.amp.copy()
    c2 = np.random.default_rng(1).uniform(-1, 1, p.n_gauss).astype(np.float32)
    y1 = oracle_lib.forward(p, 3.0, params=(p.mean, p.log_scale, p.quat, c1))
    y2 = oracle_lib.forward(p, 3.0, params=(p.mean, p.log_scale, p.quat, c2))
    yc = oracle_lib.forward(p, 3.0, params=(p.mean, p.log_scale, p.quat, 2.0 * c1.astype(np.float64) - 3.0 * c2.astype(np.float64)))
    assert np.abs(yc - (2 * y1 - 3 * y2)).max() <= 1e-12
    g = np.random.default_rng(2).standard_normal(p.n_pixels)
    grad = oracle_lib.backward(p, g, 3.0)
    for j in range(p.n_gauss):
        e = np.zeros(p.n_gauss, np.float32)
        e[j] = 1.0
        yj = oracle_lib.forward(p, 3.0, params=(p.mean, p.log_scale, p.quat, e))
        assert abs(grad["amp"][j] - g @ yj) <= 1e-12 * max(1.0, abs(g @ yj))


# ---------------------------------------------------------------- P7 -------
def test_p7_rigid_invariance_and_gradient_balance(oracle_lib):
    """Moving every Gaussian and every slice by one rigid transform leaves every
    pixel unchanged (T_i, Eq. 4); hence sum_j dL/dmu_j + sum_i dL/dtau_i = 0."""
    p = synth.tiny(17, n_gauss=6, n_slices=3)
    y = oracle_lib.forward(p, 3.0)
    Q = Rotation.from_rotvec([0.4, -0.7, 0.25])
    b = np.array([3.0, -1.5, 2.0])
    Qm = Q.as_matrix()
    mu = (p.mean.astype(float) @ Qm.T + b)
    qg = (Q * Rotation.from_quat(p.quat.astype(float)[:, [1, 2, 3, 0]])).as_quat()[:, [3, 0, 1, 2]]
    qg *= np.linalg.norm(p.quat.astype(float), axis=1, keepdims=True)
    rot0 = np.einsum("ab,nbc->nac", Qm, p.rot0.reshape(-1, 3, 3).astype(float)).reshape(-1, 9)
    trans0 = p.trans0.astype(float) @ Qm.T + b
    pose = np.concatenate([p.pose[:, :3].astype(float) @ Qm.T, p.pose[:, 3:].astype(float) @ Qm.T], 1)
    q = synth.Problem(mu, p.log_scale, qg, p.amp, p.gauss_offsets, p.slice_subject, p.height, p.width,
                      p.spacing, p.psf_fwhm, rot0, trans0, pose, p.mask)
    y2 = oracle_lib.forward(q, 3.0)
    assert np.abs(y - y2).max() <= 1e-12
    g = np.random.default_rng(3).standard_normal(p.n_pixels)
    gr = oracle_lib.backward(p, g, 3.0)
    bal = gr["mean"].sum(0) + gr["pose"][:, 3:].sum(0)
    assert np.abs(bal).max() <= 1e-12 * max(1.0, np.abs(gr["mean"]).max())


# ---------------------------------------------------------------- P8 -------
def _fd_check(oracle_lib, p, tau, seed):
    rng = np.random.default_rng(seed)
    g = rng.standard_normal(p.n_pixels)
    an = oracle_lib.backward(p, g, tau)
    base = dict(mean=p.mean.astype(np.float64), log_scale=p.log_scale.astype(np.float64),
                quat=p.quat.astype(np.float64), amp=p.amp.astype(np.float64), pose=p.pose.astype(np.float64))

    def loss(vals):
        y = oracle_lib.forward(p, tau, params=(vals["mean"], vals["log_scale"], vals["quat"], vals["amp"]),
                               pose=vals["pose"])
        return g @ y

    for name in ("mean", "log_scale", "quat", "amp", "pose"):
        arr = base[name]
        fd = np.zeros_like(arr)
        for idx in np.ndindex(arr.shape):
            hstep = 1e-6 * max(1.0, abs(arr[idx]))
            vp = {k: v.copy() for k, v in base.items()}
            vm = {k: v.copy() for k, v in base.items()}
            vp[name][idx] += hstep
            vm[name][idx] -= hstep
            fd[idx] = (loss(vp) - loss(vm)) / (2 * hstep)
        scale = max(np.abs(fd).max(), 1e-12)
        err = np.abs(fd - an[name]).max()
        assert err <= 1e-6 * scale, (name, err, scale)


def test_p8_finite_differences_exact_model(oracle_lib):
    """Analytic gradients of the exact model (tau = inf) vs central differences in FP64."""
    _fd_check(oracle_lib, synth.tiny(21, n_gauss=4, n_slices=2, size=(8, 9)), np.inf, 0)


def test_p8_finite_differences_windowed_model(oracle_lib):
    """Same at the 3-sigma window; this seed keeps every pair away from the cut."""
    p = synth.tiny(23, n_gauss=4, n_slices=2, size=(8, 9))
    # guard: no pixel-Gaussian pair within 1e-4 of q = 9 (kink of the window)
    from oracle import brute
    R = [None]
    for i in range(p.n_slices):
        Rm, t = _slice_frame(p, i)
        P = _psf_cov(p, i)
        for j in range(p.n_gauss):
            L = np.linalg.inv(_cov(p.quat[j], p.log_scale[j]) + P)
            for pix in range(int(p.height[i] * p.width[i])):
                r, k = divmod(pix, int(p.width[i]))
                d = _pixel_world(p, i, r, k) - p.mean[j]
                assert abs(d @ L @ d - 9.0) > 1e-4
    _fd_check(oracle_lib, p, 3.0, 1)


def test_p8_fd_large_rotation_pose(oracle_lib):
    """Left-Jacobian chain at a large rotation (|omega| ~ 1 rad) and non-unit quaternions."""
    p = synth.tiny(29, n_gauss=3, n_slices=2, size=(7, 7), max_deg=60.0)
    _fd_check(oracle_lib, p, np.inf, 2)


# ---------------------------------------------------------------- P9 -------
def test_p9_pruned_oracle_equals_brute_force_tiny(oracle_lib):
    """The oracle's plane/disc pruning is exact: it equals the brute force over
    every (slice, pixel, Gaussian) triple at the same window."""
    from oracle import brute
    for seed in range(4):
        p = synth.tiny(40 + seed, n_gauss=8, n_slices=3, size=(10, 13))
        for tau in (np.inf, 3.0, 1.5):
            a = oracle_lib.forward(p, tau)
            b = brute.forward(p, tau)
            assert np.abs(a - b).max() <= 1e-13 * max(1.0, np.abs(b).max())


def test_p9_pruned_oracle_equals_brute_force_cube(oracle_lib):
    """Same on a slice subset of the 2,000-Gaussian cube problem."""
    from oracle import brute
    p = synth.config1(0)
    sel = np.array([0, 7, 15, 16, 23, 31, 32, 40, 47])
    sub = synth.Problem(p.mean, p.log_scale, p.quat, p.amp, p.gauss_offsets, p.slice_subject[sel],
                        p.height[sel], p.width[sel], p.spacing[sel], p.psf_fwhm[sel], p.rot0[sel],
                        p.trans0[sel], p.pose[sel], np.ones(len(sel) * 1024, np.float32))
    a, n_in, n_pairs = oracle_lib.forward(sub, 3.0, counts=True)
    b = brute.forward(sub, 3.0)
    assert np.abs(a - b).max() <= 1e-12 * np.abs(b).max()
    assert n_in > 0 and n_pairs > 0


# ------------------------------------------------------------ geometry -----
def test_pixel_embedding_and_pose_convention(oracle_lib):
    """Reading of Eq. 1's T_i(u) = R_i u + t_i with u = (u, 0) in the slice frame,
    pixel centres at ((k-(W-1)/2) dx, (r-(H-1)/2) dy), R = Exp(omega) R0,
    t = t0 + tau: a narrow Gaussian placed at a chosen pixel's world position
    peaks exactly there."""
    p = synth.tiny(31, n_gauss=1, n_slices=2, size=(9, 12), spacing=(0.7, 1.1))
    p.psf_fwhm[:] = 0.0
    p.log_scale[:] = math.log(0.2)
    for i, (r, k) in enumerate([(2, 9), (7, 1)]):
        x = _pixel_world(p, i, r, k)
        p.mean[0] = x
        y = oracle_lib.forward(p, np.inf)
        po = p.pix_offset
        seg = y[po[i]:po[i + 1]]
        assert int(np.argmax(seg)) == r * int(p.width[i]) + k
        assert abs(seg.max() - p.amp[0]) < 1e-5 * abs(p.amp[0]) + 1e-6


def test_forward_pixels_matches_forward(oracle_lib):
    p = synth.config1(0, n_gauss=300)
    y = oracle_lib.forward(p, 3.0)
    sel = np.random.default_rng(0).choice(p.n_pixels, 200, replace=False)
    ys = oracle_lib.forward_pixels(p, sel, 3.0)
    assert np.abs(ys - y[sel]).max() <= 1e-13


def test_backward_subset_matches_backward(oracle_lib):
    p = synth.config1(0, n_gauss=300)
    g = np.random.default_rng(0).standard_normal(p.n_pixels)
    full = oracle_lib.backward(p, g, 3.0)
    idx = np.array([0, 5, 17, 299])
    sub = oracle_lib.backward_subset(p, g, idx, 3.0)
    for k in ("mean", "log_scale", "quat", "amp"):
        assert np.abs(sub[k] - full[k][idx]).max() <= 1e-13 * max(1.0, np.abs(full[k]).max())


def test_batched_subjects_are_independent(oracle_lib):
    """Gaussians of one subject never reach another subject's slices."""
    a, b = synth.tiny(50, n_gauss=4), synth.tiny(51, n_gauss=5)
    cat = synth.concat([a, b])
    y = oracle_lib.forward(cat, 3.0)
    ya, yb = oracle_lib.forward(a, 3.0), oracle_lib.forward(b, 3.0)
    assert np.array_equal(y, np.concatenate([ya, yb]))
    g = np.random.default_rng(0).standard_normal(cat.n_pixels)
    gc = oracle_lib.backward(cat, g, 3.0)
    ga = oracle_lib.backward(a, g[:a.n_pixels], 3.0)
    assert np.abs(gc["mean"][:4] - ga["mean"]).max() <= 1e-14
    assert np.abs(gc["pose"][:a.n_slices] - ga["pose"]).max() <= 1e-14


# ------------------------------------------------------------ band split ---
def test_band_split_bounds_the_standard_evaluation(oracle_lib):
    """Pairs within band*tau^2 of the cut are reported apart: the standard
    gradient (which decides them by q <= tau^2) must lie within core +- bound,
    the bound must vanish for a zero band, and with a wide band it must be
    active (the test exercises the split)."""
    p = synth.tiny(60, n_gauss=8, n_slices=3, size=(12, 14))
    g = np.random.default_rng(0).standard_normal(p.n_pixels)
    std = oracle_lib.backward(p, g, 3.0)
    core0, b0 = oracle_lib.backward_band(p, g, 3.0, 0.0)
    for k in std:
        assert np.allclose(core0[k], std[k], rtol=1e-12, atol=1e-14)
        assert np.all(b0[k] == 0.0)
    core, b = oracle_lib.backward_band(p, g, 3.0, 0.3)
    active = 0
    for k in std:
        assert np.all(np.abs(std[k] - core[k]) <= b[k] * (1 + 1e-12) + 1e-15), k
        active += int((b[k] > 0).sum())
    assert active > 0
    y = oracle_lib.forward(p, 3.0)
    yc, yb = oracle_lib.forward_band(p, 3.0, 0.3)
    assert np.all(np.abs(y - yc) <= yb * (1 + 1e-12) + 1e-15) and yb.max() > 0
    yc0, yb0 = oracle_lib.forward_band(p, 3.0, 0.0)
    assert np.allclose(yc0, y, rtol=1e-13, atol=1e-15) and np.all(yb0 == 0)


def test_p8_fd_stress_subproblem(oracle_lib):
    """Central differences on the differentiation-stress geometry: the 500
    Gaussians nearest the head centre, crops of a few slices through them,
    interleaved-segment motion; a sample of parameters of every block and all
    six pose coordinates of every cropped slice."""
    W = 48   # the central 48x48 pixels of 320x320 slices: same centres and spacing
    full = synth.config3(0, n_gauss=60000, n_per_stack=40, size=W)
    d = np.linalg.norm(full.mean, axis=1)
    near = np.argsort(d)[:500]
    sel = np.array([19, 20, 60, 100, 139, 180, 221])      # slices through the centre of several stacks
    sub = synth.Problem(full.mean[near], full.log_scale[near], full.quat[near], full.amp[near],
                        np.array([0, 500], np.int64), np.zeros(len(sel), np.int32), np.full(len(sel), W, np.int32),
                        np.full(len(sel), W, np.int32), full.spacing[sel], full.psf_fwhm[sel], full.rot0[sel],
                        full.trans0[sel], full.pose[sel], np.ones(len(sel) * W * W, np.float32))
    rng = np.random.default_rng(5)
    g = rng.standard_normal(sub.n_pixels)
    tau = np.inf
    an = oracle_lib.backward(sub, g, tau)
    base = dict(mean=sub.mean.astype(np.float64), log_scale=sub.log_scale.astype(np.float64),
                quat=sub.quat.astype(np.float64), amp=sub.amp.astype(np.float64), pose=sub.pose.astype(np.float64))

    def loss(vals):
        y = oracle_lib.forward(sub, tau, params=(vals["mean"], vals["log_scale"], vals["quat"], vals["amp"]),
                               pose=vals["pose"])
        return g @ y

    picks = {k: [tuple(rng.integers(0, s) for s in base[k].shape) for _ in range(12)] for k in
             ("mean", "log_scale", "quat", "amp")}
    picks["pose"] = [(i, c) for i in range(len(sel)) for c in range(6)]
    for name, idxs in picks.items():
        scale = max(np.abs(an[name]).max(), 1e-12)
        for idx in idxs:
            h = 1e-6 * max(1.0, abs(base[name][idx]))
            vp = {k: v.copy() for k, v in base.items()}
            vm = {k: v.copy() for k, v in base.items()}
            vp[name][idx] += h
            vm[name][idx] -= h
            fd = (loss(vp) - loss(vm)) / (2 * h)
            assert abs(fd - an[name][idx]) <= 1e-6 * scale, (name, idx, fd, an[name][idx], scale)
