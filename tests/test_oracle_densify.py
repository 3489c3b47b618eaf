"""Pins of the densification oracle (oracle/densify.py) against facts that do
not come from its own formulas: grid quadrature of the parent and children
volumes (integral, mean, covariance), the eigenvectors of the covariance,
hand-computed decisions at the thresholds and a hand-worked layout."""
import numpy as np
import pytest

from oracle import densify as od


def _rot(q):
    """Rotation of a (w, x, y, z) quaternion of any norm, the textbook formula."""
    w, x, y, z = np.asarray(q, np.float64) / np.linalg.norm(q)
    return np.array([[1 - 2 * (y * y + z * z), 2 * (x * y - w * z), 2 * (x * z + w * y)],
                     [2 * (x * y + w * z), 1 - 2 * (x * x + z * z), 2 * (y * z - w * x)],
                     [2 * (x * z - w * y), 2 * (y * z + w * x), 1 - 2 * (x * x + y * y)]])


def _cov(ls, q):
    R = _rot(q)
    return R @ np.diag(np.exp(2.0 * np.asarray(ls, np.float64))) @ R.T


def _grid_moments(mu, cov, amp, n=88, half=None):
    """Integral, mean and covariance of sum_k c_k exp(-1/2 (x-mu_k)^T S_k^-1 (x-mu_k)) by the
    trapezoidal rule on a box grid (spectrally accurate for Gaussians well inside the box)."""
    centre = np.mean(mu, 0)
    half = half or 7.0 * np.sqrt(max(np.linalg.eigvalsh(c).max() for c in cov)) + np.abs(mu - centre).max()
    ax = np.linspace(-half, half, n)
    h = ax[1] - ax[0]
    X = np.stack(np.meshgrid(ax, ax, ax, indexing="ij"), -1).reshape(-1, 3) + centre
    V = np.zeros(len(X))
    for m, S, c in zip(mu, cov, amp):
        d = X - m
        V += c * np.exp(-0.5 * np.einsum("ni,ij,nj->n", d, np.linalg.inv(S), d))
    mass = V.sum() * h ** 3
    mean = (V[:, None] * X).sum(0) * h ** 3 / mass
    d = X - mean
    cov_ = (V[:, None, None] * d[:, :, None] * d[:, None, :]).sum(0) * h ** 3 / mass
    return mass, mean, cov_


def _parents(seed, n):
    rng = np.random.default_rng(seed)
    mean = rng.uniform(-3, 3, (n, 3))
    ls = np.log(rng.uniform(0.6, 2.0, (n, 3)))
    q = rng.normal(size=(n, 4)) * rng.uniform(0.5, 2.0, (n, 1))   # storage of any norm
    amp = rng.uniform(-1.0, 2.0, n)
    return mean, ls, q, amp


@pytest.mark.parametrize("a", [np.sqrt(3.0) / 2.0, 0.6])
def test_split_keeps_integral_and_two_moments(a):
    mean, ls, q, amp = _parents(1, 3)
    (cm, cp), cls, cq, ca = od.children(mean, ls, q, amp, np.ones(3, bool), split_offset=a, clone_offset=0.5)
    for j in range(3):
        m0, mu0, c0 = _grid_moments([mean[j]], [_cov(ls[j], q[j])], [amp[j]])
        m1, mu1, c1 = _grid_moments([cm[j], cp[j]], [_cov(cls[j], cq[j])] * 2, [ca[j]] * 2)
        assert abs(m1 - m0) <= 1e-9 * abs(m0)
        np.testing.assert_allclose(mu1, mu0, atol=1e-9)
        np.testing.assert_allclose(c1, c0, atol=1e-8 * np.abs(c0).max())


def test_split_at_sqrt3_over_2_halves_the_long_axis_and_keeps_the_amplitude():
    mean, ls, q, amp = _parents(2, 5)
    (cm, cp), cls, cq, ca = od.children(mean, ls, q, amp, np.ones(5, bool), split_offset=np.sqrt(3) / 2,
                                        clone_offset=0.5)
    np.testing.assert_allclose(ca, amp, rtol=1e-14)
    for j in range(5):
        w, V = np.linalg.eigh(_cov(ls[j], q[j]))
        e = V[:, -1]                                 # eigenvector of the largest eigenvalue
        d = cp[j] - mean[j]
        assert abs(abs(d @ e) - np.linalg.norm(d)) < 1e-12 * np.linalg.norm(d)    # along the long axis
        np.testing.assert_allclose(cm[j] - mean[j], -d, atol=1e-14)
        np.testing.assert_allclose(np.linalg.norm(d), np.sqrt(3) / 2 * np.sqrt(w[-1]), rtol=1e-12)
        wc = np.linalg.eigvalsh(_cov(cls[j], cq[j]))
        np.testing.assert_allclose(sorted(wc), sorted([w[-1] / 4, w[0], w[1]]), rtol=1e-12)


def test_clone_keeps_integral_and_mean_and_widens_along_the_long_axis():
    mean, ls, q, amp = _parents(3, 2)
    b = 0.5
    (cm, cp), cls, cq, ca = od.children(mean, ls, q, amp, np.zeros(2, bool), split_offset=0.8, clone_offset=b)
    for j in range(2):
        S = _cov(ls[j], q[j])
        m0, mu0, _ = _grid_moments([mean[j]], [S], [amp[j]])
        m1, mu1, c1 = _grid_moments([cm[j], cp[j]], [_cov(cls[j], cq[j])] * 2, [ca[j]] * 2)
        assert abs(m1 - m0) <= 1e-9 * abs(m0)
        np.testing.assert_allclose(mu1, mu0, atol=1e-9)
        w, V = np.linalg.eigh(S)
        np.testing.assert_allclose(c1, S + b * b * w[-1] * np.outer(V[:, -1], V[:, -1]), atol=1e-8 * w[-1])


def test_decisions_at_the_thresholds():
    f = np.float32
    acc = np.array([2.0, np.nextafter(f(2.0), f(3.0)), 5.0, 0.0, 9.0, 9.0, 9.0, 0.1], np.float32)
    cnt = np.array([4, 4, 0, 3, 1, 1, 1, 1], np.int32)
    ls = np.zeros((8, 3), np.float32)
    ls[5, 1] = f(0.25)                                # exactly at the scale threshold: clone
    ls[6, 2] = np.nextafter(f(0.25), f(1.0))           # just above: split
    amp = np.array([1, 1, 1, 1, 1, 1, 1, 0.01], np.float32)
    n_out, split = od.decide(acc, cnt, ls, amp, grad_threshold=0.5, log_scale_threshold=0.25, prune_amp=0.05)
    # mean norm 0.5 == threshold: kept; one ulp above: densified; unseen: kept; pruned beats densify
    assert n_out.tolist() == [1, 2, 1, 1, 2, 2, 2, 0]
    assert split.tolist() == [False, False, False, False, False, False, True, False]


def test_decision_matches_the_mean_gradient_away_from_ties():
    rng = np.random.default_rng(4)
    acc = rng.exponential(1e-3, 10000).astype(np.float32)
    cnt = rng.integers(0, 50, 10000).astype(np.int32)
    n_out, _ = od.decide(acc, cnt, np.zeros((10000, 3)), np.ones(10000), grad_threshold=2e-5,
                         log_scale_threshold=1.0)
    with np.errstate(divide="ignore", invalid="ignore"):
        mean = acc.astype(np.float64) / cnt
    far = (cnt == 0) | (np.abs(mean / 2e-5 - 1) > 1e-5)
    expect = np.where((cnt > 0) & (mean > 2e-5), 2, 1)
    assert far.sum() > 9900
    assert np.array_equal(n_out[far], expect[far])


def test_layout_offsets_and_sources_by_hand():
    # two subjects of 3 and 2 Gaussians: keep, densify, prune | densify, keep
    go = np.array([0, 3, 5])
    mean, ls, q, _ = _parents(5, 5)
    amp = np.array([1.0, 1.0, 0.0, 1.0, 1.0])
    acc = np.array([0, 1, 1, 1, 0], np.float32)
    cnt = np.array([1, 1, 1, 1, 1], np.int32)
    out = od.densify(go, mean, ls, q, amp, acc, cnt, dict(grad_threshold=0.5, prune_amp=0.5))
    assert out["offsets"].tolist() == [0, 3, 6]
    assert out["src"].tolist() == [0, -2, -2, -4, -4, 4]
    np.testing.assert_array_equal(out["mean"][0], mean[0])
    np.testing.assert_array_equal(out["mean"][5], mean[4])
    np.testing.assert_allclose(out["mean"][1] + out["mean"][2], 2 * mean[1], atol=1e-12)


def test_moments_follow_the_sources():
    N, M = 3, 2
    mom = np.arange(11 * N + 6 * M, dtype=np.float64)
    src = np.array([0, -2, -2, 2])
    new = od.remap_moments(mom, src, N)
    K = 4
    assert len(new) == 11 * K + 6 * M
    np.testing.assert_array_equal(new[:3 * K].reshape(K, 3), [[0, 1, 2], [0, 0, 0], [0, 0, 0], [6, 7, 8]])
    np.testing.assert_array_equal(new[10 * K:11 * K], [30, 0, 0, 32])    # amp block starts at 10N
    np.testing.assert_array_equal(new[11 * K:], mom[11 * N:])


def test_accumulate_by_hand():
    acc, cnt = od.accumulate(np.zeros(3, np.float32), np.zeros(3, np.int32),
                             np.array([[3, 4, 0], [0, 0, 0], [0, -1e-30, 0]], np.float32))
    assert acc.tolist() == [5.0, 0.0, np.float32(1e-30)]
    assert cnt.tolist() == [1, 0, 1]
