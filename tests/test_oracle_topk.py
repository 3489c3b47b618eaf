"""Pins of the normalised Top-K oracle (Eqs. 2 and 5, Top-K of Sec. 2.5)
against scipy's rotations and Gaussian density, brute-force neighbour
search, closed special cases and central finite differences."""
import numpy as np
import pytest
import torch
from scipy.spatial.transform import Rotation
from scipy.stats import multivariate_normal

from oracle import topk
from paper_2512_11624_amd import synth


def test_rotations_match_scipy():
    rng = np.random.default_rng(0)
    w = np.concatenate([rng.normal(0, 1.0, (6, 3)), rng.normal(0, 1e-8, (2, 3)), np.zeros((1, 3))])
    R = topk.rotvec_matrix(torch.tensor(w)).numpy()
    assert np.abs(R - Rotation.from_rotvec(w).as_matrix()).max() < 1e-14
    q = rng.normal(size=(8, 4)) * rng.uniform(0.5, 2.0, (8, 1))
    Rq = topk.quat_matrix(torch.tensor(q)).numpy()
    assert np.abs(Rq - Rotation.from_quat(q[:, [1, 2, 3, 0]]).as_matrix()).max() < 1e-14


def _prob(seed=0, n=40, **kw):
    return synth.tiny(seed, n_gauss=n, **kw)


def test_pixel_positions_match_generator():
    p = _prob(1, n_slices=3)
    x = topk.pixel_positions(p, torch.tensor(p.pose, dtype=torch.float64)).numpy()
    ref = np.concatenate(synth.pixel_world_positions(p.rot0, p.trans0, p.pose.astype(np.float64), p.height,
                                                     p.width, p.spacing))
    assert np.abs(x - ref).max() < 1e-12


def test_knn_matches_brute_force():
    a, b = _prob(2, n=60, n_slices=2), _prob(3, n=80, n_slices=2)
    p = synth.concat([a, b])
    K = 7
    idx, d2 = topk.knn(p, p.mean, p.pose, K)
    x = topk.pixel_positions(p, torch.tensor(p.pose, dtype=torch.float64)).numpy()
    go = p.gauss_offsets
    sl, _ = topk.pixel_slices(p)
    for r in range(len(x)):
        s = p.slice_subject[sl[r]]
        m = p.mean[go[s]:go[s + 1]].astype(np.float64)
        d = ((x[r] - m) ** 2).sum(1)
        order = np.argsort(d, kind="stable")
        assert np.allclose(np.sort(d)[:K + 1], d2[r], rtol=1e-12)
        assert set(idx[r]) == set(go[s] + order[:K]) or np.isclose(d[order[K - 1]], d[order[K]], rtol=1e-12)


def _params(p):
    return p.mean, p.log_scale, p.quat, p.amp


def test_single_neighbour_closed_form():
    # K = 1: y = c e / (e + delta), e = (2 pi)^{3/2} sqrt(det S_obs) N(x; mu, S_obs)
    p = _prob(4, n=30, n_slices=2)
    nbr, _ = topk.knn(p, p.mean, p.pose, 1)
    delta = 0.05
    y, num, den = topk.forward_np(p, _params(p), p.pose, nbr, delta)
    x = topk.pixel_positions(p, torch.tensor(p.pose, dtype=torch.float64)).numpy()
    sl, _ = topk.pixel_slices(p)
    for r in range(0, len(x), 7):
        j = nbr[r, 0]
        Rg = Rotation.from_quat(p.quat[j, [1, 2, 3, 0]].astype(np.float64)).as_matrix()
        Sg = Rg @ np.diag(np.exp(2 * p.log_scale[j].astype(np.float64))) @ Rg.T
        Ri = Rotation.from_rotvec(p.pose[sl[r], :3].astype(np.float64)).as_matrix() @ \
            p.rot0[sl[r]].reshape(3, 3).astype(np.float64)
        Sp = Ri @ np.diag((p.psf_fwhm[sl[r]].astype(np.float64) / 2.355) ** 2) @ Ri.T
        So = Sg + Sp
        e = multivariate_normal(p.mean[j].astype(np.float64), So).pdf(x[r]) * (2 * np.pi) ** 1.5 * np.sqrt(np.linalg.det(So))
        assert abs(den[r] - e) < 1e-12 * max(1.0, e)
        assert abs(y[r] - p.amp[j] * e / (e + delta)) < 1e-12


def test_all_neighbours_is_the_normalised_mixture():
    # K = N, delta = 0: y = sum c e / sum e over every Gaussian
    p = _prob(5, n=12, n_slices=2)
    nbr, _ = topk.knn(p, p.mean, p.pose, p.n_gauss)
    y, _, _ = topk.forward_np(p, _params(p), p.pose, nbr, 0.0)
    x = topk.pixel_positions(p, torch.tensor(p.pose, dtype=torch.float64)).numpy()
    sl, _ = topk.pixel_slices(p)
    for r in range(0, len(x), 11):
        Ri = Rotation.from_rotvec(p.pose[sl[r], :3].astype(np.float64)).as_matrix() @ \
            p.rot0[sl[r]].reshape(3, 3).astype(np.float64)
        Sp = Ri @ np.diag((p.psf_fwhm[sl[r]].astype(np.float64) / 2.355) ** 2) @ Ri.T
        es = []
        for j in range(p.n_gauss):
            Rg = Rotation.from_quat(p.quat[j, [1, 2, 3, 0]].astype(np.float64)).as_matrix()
            So = Rg @ np.diag(np.exp(2 * p.log_scale[j].astype(np.float64))) @ Rg.T + Sp
            es.append(multivariate_normal(p.mean[j].astype(np.float64), So).pdf(x[r]) * (2 * np.pi) ** 1.5
                      * np.sqrt(np.linalg.det(So)))
        es = np.array(es)
        assert abs(y[r] - (p.amp.astype(np.float64) * es).sum() / es.sum()) < 1e-10


def test_convex_combination_and_intensity_scalar():
    p = _prob(6, n=50, n_slices=3)
    nbr, _ = topk.knn(p, p.mean, p.pose, 8)
    delta = 1e-3
    y, num, den = topk.forward_np(p, _params(p), p.pose, nbr, delta)
    ratio = y * (den + delta) / den
    c = p.amp.astype(np.float64)[nbr]
    assert np.all(ratio >= c.min(1) - 1e-12) and np.all(ratio <= c.max(1) + 1e-12)
    sigma = np.random.default_rng(1).uniform(0.5, 2.0, p.n_slices)
    ys, _, _ = topk.forward_np(p, _params(p), p.pose, nbr, delta, sigma)
    sl, _ = topk.pixel_slices(p)
    assert np.allclose(ys, sigma[sl] * y, rtol=1e-14)


def test_gradients_match_central_differences():
    p = _prob(7, n=25, n_slices=2, size=(5, 6))
    nbr, _ = topk.knn(p, p.mean, p.pose, 6)
    delta = 1e-2
    rng = np.random.default_rng(2)
    g = rng.normal(size=p.n_pixels)
    sigma = rng.uniform(0.5, 1.5, p.n_slices)
    params = [a.astype(np.float64) for a in _params(p)]
    pose = p.pose.astype(np.float64)
    grads = topk.gradients(p, params, pose, nbr, delta, g, sigma)
    blocks = params + [pose, sigma]

    def f(bl):
        y, _, _ = topk.forward_np(p, bl[:4], bl[4], nbr, delta, bl[5])
        return float((g * y).sum())

    for b, (blk, gr) in enumerate(zip(blocks, grads)):
        flat = blk.ravel()
        picks = rng.choice(flat.size, min(12, flat.size), replace=False)
        for k in picks:
            h = 1e-6 * max(1.0, abs(flat[k]))
            up = [x.copy() for x in blocks]
            dn = [x.copy() for x in blocks]
            up[b].ravel()[k] += h
            dn[b].ravel()[k] -= h
            fd = (f(up) - f(dn)) / (2 * h)
            assert abs(fd - gr.ravel()[k]) <= 1e-6 * max(1.0, np.abs(gr).max()), (b, k, fd, gr.ravel()[k])
