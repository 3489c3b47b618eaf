"""Pins of the bias-field oracle (oracle/bias.py): a zero field, a constant
field, central finite differences of every gradient block, linearity of
log b in beta and invariance under a rigid motion of the whole scene."""
import numpy as np
from scipy.spatial.transform import Rotation

from oracle import bias
from paper_2512_11624_amd import synth


def _setup(seed=0, K=5, width=6.0):
    prob = synth.tiny(seed, n_gauss=4, n_slices=3)
    rng = np.random.default_rng(seed + 10)
    S = prob.n_subjects
    centres = rng.uniform(-6.0, 6.0, (S, K, 3))
    beta = rng.normal(0.0, 0.3, (S, K))
    y = rng.uniform(0.1, 1.0, prob.n_pixels)
    return prob, centres, width, beta, y


def test_zero_field_leaves_pixels_unchanged():
    prob, c, w, beta, y = _setup()
    yb, b = bias.apply(prob, y, c, w, np.zeros_like(beta))
    assert np.array_equal(b, np.ones_like(y))
    assert np.array_equal(yb, y)


def test_constant_field_of_one_wide_basis():
    prob, c, w, beta, y = _setup(K=1)
    yb, b = bias.apply(prob, y, c, 1e7, beta)
    np.testing.assert_allclose(b, np.exp(beta[0, 0]), rtol=1e-12)
    np.testing.assert_allclose(yb, np.exp(beta[0, 0]) * y, rtol=1e-12)


def test_log_field_is_linear_in_beta():
    prob, c, w, beta, y = _setup()
    beta2 = np.random.default_rng(3).normal(0.0, 0.2, beta.shape)
    b1 = bias.field(prob, c, w, beta)
    b2 = bias.field(prob, c, w, beta2)
    b12 = bias.field(prob, c, w, beta + beta2)
    np.testing.assert_allclose(np.log(b12), np.log(b1) + np.log(b2), atol=1e-12)


def test_rigid_motion_of_the_scene_leaves_the_field_unchanged():
    prob, c, w, beta, y = _setup(seed=2)
    Q = Rotation.from_rotvec([0.3, -0.5, 0.7]).as_matrix()
    v = np.array([4.0, -2.0, 1.5])
    moved = synth.tiny(2, n_gauss=4, n_slices=3)
    moved.rot0 = np.stack([(Q @ r.reshape(3, 3)).ravel() for r in prob.rot0.astype(np.float64)])
    moved.trans0 = prob.trans0.astype(np.float64) @ Q.T + v
    pose = prob.pose.astype(np.float64).copy()
    mp = pose.copy()
    mp[:, :3] = pose[:, :3] @ Q.T   # Exp(Q w) Q R0 = Q Exp(w) R0
    mp[:, 3:] = pose[:, 3:] @ Q.T
    b0 = bias.field(prob, c, w, beta, pose)
    b1 = bias.field(moved, c @ Q.T + v, w, beta, mp)
    np.testing.assert_allclose(b1, b0, rtol=1e-12)


def test_gradients_match_central_differences():
    prob, c, w, beta, y = _setup(seed=1)
    g = np.random.default_rng(7).normal(0.0, 1.0, prob.n_pixels)
    pose = prob.pose.astype(np.float64)
    gr = bias.gradients(prob, y, g, c, w, beta, pose)
    L = lambda bt, ps, yy=y: float(g @ bias.apply(prob, yy, c, w, bt, ps)[0])
    h = 1e-6
    fd_beta = np.zeros_like(beta)
    for idx in np.ndindex(beta.shape):
        e = np.zeros_like(beta)
        e[idx] = h
        fd_beta[idx] = (L(beta + e, pose) - L(beta - e, pose)) / (2 * h)
    fd_pose = np.zeros_like(pose)
    for idx in np.ndindex(pose.shape):
        e = np.zeros_like(pose)
        e[idx] = h
        fd_pose[idx] = (L(beta, pose + e) - L(beta, pose - e)) / (2 * h)
    for name, fd in (("beta", fd_beta), ("pose", fd_pose)):
        scale = np.abs(fd).max()
        assert np.abs(gr[name] - fd).max() <= 1e-6 * scale, (name, np.abs(gr[name] - fd).max(), scale)
    # dL/dy: the loss is linear in y with coefficient g b
    b = bias.field(prob, c, w, beta, pose)
    np.testing.assert_allclose(gr["pred"], g * b, rtol=1e-12)
