"""Seeded synthetic inputs for the Gaussian-primitive slice-to-volume problem.

This module only *draws* inputs: Gaussian parameters, stack geometry, slice
motion, masks and noise.  It holds none of the forward model's arithmetic
(no covariance addition, no Gaussian evaluation) so that it can feed both the
FP64 oracle and the HIP path without coupling them.  Random numbers come from
``numpy.random.default_rng(SeedSequence(seed).spawn(k))`` streams, one stream
per quantity, so that changing one size does not reshuffle the others.

Conventions shared by every consumer (they are *inputs*, not arithmetic):

* Gaussian ``j``: mean ``mu`` [mm], log-scale ``log_scale`` (s = exp), quaternion
  ``quat`` stored (w, x, y, z) and not necessarily unit length, amplitude ``amp``
  (Sec. 2.2 and the nomenclature table of the paper).
* Slice ``i``: nominal rotation ``rot0`` (row-major 3x3, columns = slice x axis,
  slice y axis, slice normal), nominal centre ``trans0`` [mm], rigid pose delta
  ``pose`` = (omega [rad], tau [mm]) with R = Exp(omega) R0 and t = t0 + tau
  (Sec. 2.1 and 2.4), pixel spacing (dx along columns, dy along rows) and PSF
  full width at half maximum along the slice frame axes (Sec. 2.3).
* Pixels of slice ``i`` are stored row-major and contiguously; slice ``i``
  starts at ``pix_offset[i]``.
"""
from __future__ import annotations

from dataclasses import dataclass, field
import math

import numpy as np
from scipy.spatial.transform import Rotation

DEG = math.pi / 180.0


@dataclass
class Problem:
    """A complete seeded problem instance (all float arrays are float32)."""

    mean: np.ndarray          # [N,3]
    log_scale: np.ndarray     # [N,3]
    quat: np.ndarray          # [N,4] (w,x,y,z)
    amp: np.ndarray           # [N]
    gauss_offsets: np.ndarray  # [S+1] int64
    slice_subject: np.ndarray  # [M] int32
    height: np.ndarray        # [M] int32
    width: np.ndarray         # [M] int32
    spacing: np.ndarray       # [M,2]
    psf_fwhm: np.ndarray      # [M,3]
    rot0: np.ndarray          # [M,9]
    trans0: np.ndarray        # [M,3]
    pose: np.ndarray          # [M,6] acquisition motion (omega, tau)
    mask: np.ndarray          # [P]
    name: str = ""
    extra: dict = field(default_factory=dict)

    @property
    def n_gauss(self) -> int:
        return int(self.mean.shape[0])

    @property
    def n_slices(self) -> int:
        return int(self.height.shape[0])

    @property
    def n_subjects(self) -> int:
        return int(self.gauss_offsets.shape[0] - 1)

    @property
    def pix_offset(self) -> np.ndarray:
        npx = self.height.astype(np.int64) * self.width.astype(np.int64)
        return np.concatenate([[0], np.cumsum(npx)]).astype(np.int64)

    @property
    def n_pixels(self) -> int:
        return int(self.pix_offset[-1])

    def params(self):
        return self.mean, self.log_scale, self.quat, self.amp


def _streams(seed: int, k: int):
    return [np.random.default_rng(s) for s in np.random.SeedSequence(seed).spawn(k)]


def _random_quats(rng, n):
    q = rng.standard_normal((n, 4))
    q /= np.linalg.norm(q, axis=1, keepdims=True)
    return q


# Stack orientations: columns are (slice x, slice y, normal), right handed.
AXIAL = np.eye(3)
CORONAL = np.stack([[1, 0, 0], [0, 0, 1], [0, -1, 0]], axis=1).astype(float)
SAGITTAL = np.stack([[0, 1, 0], [0, 0, 1], [1, 0, 0]], axis=1).astype(float)


def oblique(rx_deg, ry_deg, rz_deg=0.0):
    return Rotation.from_rotvec(np.array([rx_deg, ry_deg, rz_deg]) * DEG).as_matrix() @ AXIAL


def _stack(orient, n_slices, thickness, centre):
    """Nominal rotations / centres of one stack: slices tile the normal axis
    with no gap, centred on ``centre``."""
    normal = orient[:, 2]
    offs = (np.arange(n_slices) - (n_slices - 1) / 2.0) * thickness
    rot = np.repeat(orient.reshape(1, 9), n_slices, axis=0)
    trans = centre[None, :] + offs[:, None] * normal[None, :]
    return rot, trans


def _assemble_slices(stacks):
    """stacks: list of dicts(orient, n, H, W, dx, dy, thick, fwhm, centre, subject)."""
    rot, trans, H, W, sp, fw, subj = [], [], [], [], [], [], []
    for s in stacks:
        r, t = _stack(s["orient"], s["n"], s["thick"], s["centre"])
        rot.append(r)
        trans.append(t)
        H.append(np.full(s["n"], s["H"], np.int32))
        W.append(np.full(s["n"], s["W"], np.int32))
        sp.append(np.tile([s["dx"], s["dy"]], (s["n"], 1)))
        fw.append(np.tile(s["fwhm"], (s["n"], 1)))
        subj.append(np.full(s["n"], s.get("subject", 0), np.int32))
    return (np.concatenate(rot), np.concatenate(trans), np.concatenate(H),
            np.concatenate(W), np.concatenate(sp), np.concatenate(fw), np.concatenate(subj))


def pixel_world_positions(rot0, trans0, pose, height, width, spacing, slice_ids=None):
    """World position of every pixel centre under pose (scipy rotations; used
    for masks only).  Returns a list of [H*W,3] float64 arrays."""
    out = []
    ids = range(len(height)) if slice_ids is None else slice_ids
    for i in ids:
        R = Rotation.from_rotvec(pose[i, :3].astype(np.float64)).as_matrix() @ rot0[i].reshape(3, 3)
        t = trans0[i].astype(np.float64) + pose[i, 3:].astype(np.float64)
        h, w = int(height[i]), int(width[i])
        cols = (np.arange(w) - (w - 1) / 2.0) * float(spacing[i, 0])
        rows = (np.arange(h) - (h - 1) / 2.0) * float(spacing[i, 1])
        uu, vv = np.meshgrid(cols, rows)
        u = np.stack([uu.ravel(), vv.ravel(), np.zeros(h * w)], axis=1)
        out.append(u @ R.T + t[None, :])
    return out


def _motion_uniform(rng, m, max_deg, max_mm):
    axis = rng.standard_normal((m, 3))
    axis /= np.linalg.norm(axis, axis=1, keepdims=True)
    ang = rng.uniform(0.0, max_deg * DEG, size=(m, 1))
    tau = rng.uniform(-max_mm, max_mm, size=(m, 3))
    return np.concatenate([axis * ang, tau], axis=1)


def _motion_normal(rng, m, sd_deg, sd_mm):
    om = rng.normal(0.0, sd_deg * DEG, size=(m, 3))
    tau = rng.normal(0.0, sd_mm, size=(m, 3))
    return np.concatenate([om, tau], axis=1)


def _f32(*arrs):
    return [np.ascontiguousarray(a, dtype=np.float32) for a in arrs]


def cube_gaussians(rng_mu, rng_s, rng_q, rng_c, n, half, s_lo=0.5, s_hi=2.0):
    mu = rng_mu.uniform(-half, half, size=(n, 3))
    ls = rng_s.uniform(math.log(s_lo), math.log(s_hi), size=(n, 3))
    q = _random_quats(rng_q, n)
    c = rng_c.uniform(0.0, 1.0, size=n)
    return mu, ls, q, c


def config1(seed: int = 0, n_gauss: int = 2000, side: float = 32.0, n_per_stack: int = 16,
            size: int = 32, spacing: float = 1.0, thickness: float = 3.0,
            max_deg: float = 5.0, max_mm: float = 2.0, n_stacks: int = 3) -> Problem:
    """Cube phantom: 2,000 Gaussians in a 32 mm cube, three orthogonal stacks of
    16 slices of 32x32 px at 1x1x3 mm, PSF FWHM (1,1,3) mm, motion <=5 deg and
    <=2 mm.  Smaller/larger variants keep the same distributions."""
    r_mu, r_s, r_q, r_c, r_mot = _streams(seed, 5)
    half = side / 2.0
    mu, ls, q, c = cube_gaussians(r_mu, r_s, r_q, r_c, n_gauss, half)
    orients = [AXIAL, CORONAL, SAGITTAL][:n_stacks]
    stacks = [dict(orient=o, n=n_per_stack, H=size, W=size, dx=spacing, dy=spacing,
                   thick=thickness, fwhm=[spacing, spacing, thickness], centre=np.zeros(3))
              for o in orients]
    rot, trans, H, W, sp, fw, subj = _assemble_slices(stacks)
    pose = _motion_uniform(r_mot, len(H), max_deg, max_mm)
    pos = pixel_world_positions(rot, trans, pose, H, W, sp)
    mask = np.concatenate([np.all(np.abs(p) <= half, axis=1) for p in pos]).astype(np.float32)
    mu, ls, q, c, sp, fw, rot, trans, pose = _f32(mu, ls, q, c, sp, fw, rot, trans, pose)
    return Problem(mu, ls, q, c, np.array([0, n_gauss], np.int64), subj, H, W, sp, fw,
                   rot, trans, pose, mask, name="cube", extra=dict(side=side))


# ---------------------------------------------------------------------------
# Head phantom (nested ellipsoid shells, intensities in [0,1], smooth bias)
# ---------------------------------------------------------------------------

HEAD_AXES = np.array([40.0, 50.0, 42.0])


def head_intensity(x, axes=HEAD_AXES):
    """Piecewise-constant tissue intensity of the synthetic head at points x [K,3]."""
    r = np.linalg.norm(x / axes[None, :], axis=1)
    val = np.zeros(len(x))
    val[r < 1.0] = 0.2                      # scalp / skull
    val[r < 0.92] = 1.0                     # CSF
    val[r < 0.85] = 0.6                     # cortex
    val[r < 0.75] = 0.8                     # white matter
    for c, a in (((12.0, 5.0, 4.0), (6.0, 16.0, 7.0)), ((-12.0, 5.0, 4.0), (6.0, 16.0, 7.0))):
        rv = np.linalg.norm((x - np.array(c)) / np.array(a), axis=1)
        val[rv < 1.0] = 1.0                 # ventricles
    return val


def head_bias(x, rng_params, axes=HEAD_AXES):
    """Smooth multiplicative bias field in [0.85, 1.15] from three broad bumps."""
    p = rng_params
    f = np.zeros(len(x))
    for k in range(3):
        c = p["centres"][k]
        w = p["widths"][k]
        f += p["weights"][k] * np.exp(-0.5 * np.sum(((x - c) / w) ** 2, axis=1))
    lo, hi = p["range"]
    return 0.85 + 0.30 * (f - lo) / max(hi - lo, 1e-12)


def _bias_params(rng, axes=HEAD_AXES):
    centres = rng.uniform(-1.0, 1.0, size=(3, 3)) * axes[None, :]
    widths = rng.uniform(0.6, 1.2, size=(3, 1)) * axes[None, :]
    weights = rng.uniform(-1.0, 1.0, size=3)
    p = dict(centres=centres, widths=widths, weights=weights)
    # normalisation range estimated on a fixed coarse grid inside the head
    g = np.stack(np.meshgrid(*[np.linspace(-1, 1, 13)] * 3, indexing="ij"), -1).reshape(-1, 3)
    g = g[np.linalg.norm(g, axis=1) <= 1.0] * axes[None, :]
    f = np.zeros(len(g))
    for k in range(3):
        f += weights[k] * np.exp(-0.5 * np.sum(((g - centres[k]) / widths[k]) ** 2, axis=1))
    p["range"] = (float(f.min()), float(f.max()))
    return p


def head_gaussians(rng_mu, rng_s, rng_q, rng_b, n, axes=HEAD_AXES):
    """n Gaussians with means uniform in the head ellipsoid, log-uniform scales on
    [0.5h, 1.5h] (h = (V/n)^(1/3)), random rotations and amplitudes
    c = p(mu) b(mu) kappa, kappa making the mixture's mean density match p."""
    vol = 4.0 / 3.0 * math.pi * float(np.prod(axes))
    h = (vol / n) ** (1.0 / 3.0)
    pts = []
    need = n
    while need > 0:
        x = rng_mu.uniform(-1.0, 1.0, size=(int(need * 2.1) + 16, 3))
        x = x[np.linalg.norm(x, axis=1) <= 1.0][:need]
        pts.append(x)
        need -= len(x)
    mu = np.concatenate(pts)[:n] * axes[None, :]
    ls = rng_s.uniform(math.log(0.5 * h), math.log(1.5 * h), size=(n, 3))
    q = _random_quats(rng_q, n)
    bp = _bias_params(rng_b, axes)
    es = (h / math.log(3.0))      # E[s] for log-uniform on [0.5h, 1.5h]
    kappa = 1.0 / ((n / vol) * (2.0 * math.pi) ** 1.5 * es ** 3)
    c = head_intensity(mu, axes) * head_bias(mu, bp, axes) * kappa
    return mu, ls, q, c, h, bp


def config2(seed: int = 0, n_gauss: int = 500_000, n_per_stack: int = 32, size: int = 256,
            spacing: float = 0.8, thickness: float = 3.5, sd_deg: float = 4.0,
            sd_mm: float = 2.0, axes=HEAD_AXES, orients=None) -> Problem:
    """Fetal-scale head phantom: 500k Gaussians, four stacks (axial, coronal,
    sagittal, oblique 30/20 deg) of 32 slices of 256x256 px at 0.8x0.8x3.5 mm,
    PSF FWHM = (spacing, spacing, thickness), motion ~N(0,4 deg), ~N(0,2 mm)."""
    r_mu, r_s, r_q, r_b, r_mot = _streams(seed, 5)
    axes = np.asarray(axes, float)
    mu, ls, q, c, h, bp = head_gaussians(r_mu, r_s, r_q, r_b, n_gauss, axes)
    if orients is None:
        orients = [AXIAL, CORONAL, SAGITTAL, oblique(30.0, 20.0)]
    stacks = [dict(orient=o, n=n_per_stack, H=size, W=size, dx=spacing, dy=spacing,
                   thick=thickness, fwhm=[spacing, spacing, thickness], centre=np.zeros(3))
              for o in orients]
    rot, trans, H, W, sp, fw, subj = _assemble_slices(stacks)
    pose = _motion_normal(r_mot, len(H), sd_deg, sd_mm)
    pos = pixel_world_positions(rot, trans, pose, H, W, sp)
    dil = axes + 2.0
    mask = np.concatenate([np.linalg.norm(p / dil[None, :], axis=1) <= 1.0 for p in pos])
    mu, ls, q, c, sp, fw, rot, trans, pose = _f32(mu, ls, q, c, sp, fw, rot, trans, pose)
    return Problem(mu, ls, q, c, np.array([0, n_gauss], np.int64), subj, H, W, sp, fw,
                   rot, trans, pose, mask.astype(np.float32), name="head",
                   extra=dict(h=h, axes=axes, bias=bp))


def config3(seed: int = 0, n_gauss: int = 1_200_000, n_per_stack: int = 40, size: int = 320,
            spacing: float = 0.7, thickness: float = 3.0, n_segments: int = 6,
            axes=HEAD_AXES) -> Problem:
    """Differentiation stress: 1.2M Gaussians, 6 stacks of 40 slices of 320x320 px
    at 0.7x0.7x3 mm.  Motion: each stack's interleaved acquisition order (even
    slices then odd) is cut into 6 contiguous segments with one rigid motion
    each, plus small per-slice jitter."""
    r_mu, r_s, r_q, r_b, r_mot = _streams(seed, 5)
    axes = np.asarray(axes, float)
    mu, ls, q, c, h, bp = head_gaussians(r_mu, r_s, r_q, r_b, n_gauss, axes)
    orients = [AXIAL, CORONAL, SAGITTAL, oblique(30.0, 20.0), oblique(-25.0, 35.0),
               oblique(40.0, -15.0, 20.0)]
    stacks = [dict(orient=o, n=n_per_stack, H=size, W=size, dx=spacing, dy=spacing,
                   thick=thickness, fwhm=[spacing, spacing, thickness], centre=np.zeros(3))
              for o in orients]
    rot, trans, H, W, sp, fw, subj = _assemble_slices(stacks)
    pose = np.zeros((len(H), 6))
    for s in range(len(orients)):
        order = np.concatenate([np.arange(0, n_per_stack, 2), np.arange(1, n_per_stack, 2)])
        segs = np.array_split(order, n_segments)
        for seg in segs:
            base = _motion_normal(r_mot, 1, 4.0, 2.0)[0]
            for k in seg:
                pose[s * n_per_stack + k] = base + _motion_normal(r_mot, 1, 0.5, 0.5)[0]
    pos = pixel_world_positions(rot, trans, pose, H, W, sp)
    dil = axes + 2.0
    mask = np.concatenate([np.linalg.norm(p / dil[None, :], axis=1) <= 1.0 for p in pos])
    mu, ls, q, c, sp, fw, rot, trans, pose = _f32(mu, ls, q, c, sp, fw, rot, trans, pose)
    return Problem(mu, ls, q, c, np.array([0, n_gauss], np.int64), subj, H, W, sp, fw,
                   rot, trans, pose, mask.astype(np.float32), name="head-stress",
                   extra=dict(h=h, axes=axes, bias=bp))


def config4(seed: int = 0, n_subjects: int = 16, n_lo: float = 1.5e5, n_hi: float = 1.5e6,
            scale: float = 1.0) -> Problem:
    """Batched: n_subjects cube subjects with the cube phantom's density (2,000
    Gaussians per 32^3 mm^3).  Gaussian counts log-uniform in [n_lo, n_hi];
    3-9 stacks of 20-48 slices, in-plane size from {192,256,320} (times
    ``scale`` for reduced test variants), thickness U[2.5, 4.5] mm, in-plane
    spacing = cube side / size, motion <=5 deg / <=2 mm.  Subjects are stored
    back to back: Gaussians by ``gauss_offsets``, slices by ``slice_subject``."""
    rng = _streams(seed, 1)[0]
    subj_seeds = rng.integers(0, 2**31 - 1, size=n_subjects)
    mus, lss, qs, cs, offs = [], [], [], [], [0]
    rots, transs, Hs, Ws, sps, fws, subjs, poses, masks = [], [], [], [], [], [], [], [], []
    sizes = [max(8, int(round(s * scale))) for s in (192, 256, 320)]
    for k in range(n_subjects):
        r_n, r_mu, r_s, r_q, r_c, r_geo, r_mot = _streams(int(subj_seeds[k]), 7)
        n = int(round(math.exp(r_n.uniform(math.log(n_lo), math.log(n_hi)))))
        side = 32.0 * (n / 2000.0) ** (1.0 / 3.0)
        mu, ls, q, c = cube_gaussians(r_mu, r_s, r_q, r_c, n, side / 2.0)
        n_st = int(r_geo.integers(3, 10))
        stacks = []
        for s in range(n_st):
            if s < 3:
                o = [AXIAL, CORONAL, SAGITTAL][s]
            else:
                o = Rotation.from_rotvec(r_geo.normal(0, 0.6, 3)).as_matrix()
            ns = int(r_geo.integers(20, 49))
            w = int(sizes[int(r_geo.integers(0, 3))])
            th = float(r_geo.uniform(2.5, 4.5))
            dx = side / w
            stacks.append(dict(orient=o, n=ns, H=w, W=w, dx=dx, dy=dx, thick=th,
                               fwhm=[dx, dx, th], centre=np.zeros(3), subject=k))
        rot, trans, H, W, sp, fw, subj = _assemble_slices(stacks)
        pose = _motion_uniform(r_mot, len(H), 5.0, 2.0)
        pos = pixel_world_positions(rot, trans, pose, H, W, sp)
        masks.append(np.concatenate([np.all(np.abs(p) <= side / 2, axis=1) for p in pos]))
        mus.append(mu); lss.append(ls); qs.append(q); cs.append(c); offs.append(offs[-1] + n)
        rots.append(rot); transs.append(trans); Hs.append(H); Ws.append(W); sps.append(sp)
        fws.append(fw); subjs.append(subj); poses.append(pose)
    mu, ls, q, c, sp, fw, rot, trans, pose = _f32(
        np.concatenate(mus), np.concatenate(lss), np.concatenate(qs), np.concatenate(cs),
        np.concatenate(sps), np.concatenate(fws), np.concatenate(rots),
        np.concatenate(transs), np.concatenate(poses))
    return Problem(mu, ls, q, c, np.array(offs, np.int64), np.concatenate(subjs).astype(np.int32),
                   np.concatenate(Hs), np.concatenate(Ws), sp, fw, rot, trans, pose,
                   np.concatenate(masks).astype(np.float32), name="batched")


def subject(problem: Problem, k: int) -> Problem:
    """Extract subject k of a batched problem as a stand-alone problem."""
    g0, g1 = int(problem.gauss_offsets[k]), int(problem.gauss_offsets[k + 1])
    sl = np.nonzero(problem.slice_subject == k)[0]
    po = problem.pix_offset
    pix = np.concatenate([np.arange(po[i], po[i + 1]) for i in sl])
    return Problem(problem.mean[g0:g1].copy(), problem.log_scale[g0:g1].copy(),
                   problem.quat[g0:g1].copy(), problem.amp[g0:g1].copy(),
                   np.array([0, g1 - g0], np.int64), np.zeros(len(sl), np.int32),
                   problem.height[sl].copy(), problem.width[sl].copy(), problem.spacing[sl].copy(),
                   problem.psf_fwhm[sl].copy(), problem.rot0[sl].copy(), problem.trans0[sl].copy(),
                   problem.pose[sl].copy(), problem.mask[pix].copy(), name=f"{problem.name}[{k}]")


def concat(problems) -> Problem:
    """Stack independent single-subject problems into one batched problem."""
    offs = [0]
    for p in problems:
        assert p.n_subjects == 1
        offs.append(offs[-1] + p.n_gauss)
    cat = lambda attr: np.concatenate([getattr(p, attr) for p in problems])
    subj = np.concatenate([np.full(p.n_slices, k, np.int32) for k, p in enumerate(problems)])
    return Problem(cat("mean"), cat("log_scale"), cat("quat"), cat("amp"), np.array(offs, np.int64),
                   subj, cat("height"), cat("width"), cat("spacing"), cat("psf_fwhm"),
                   cat("rot0"), cat("trans0"), cat("pose"), cat("mask"), name="concat")


def perturb_params(problem: Problem, seed: int, d_mu=0.3, d_ls=0.1, d_q=0.1, d_c=0.1):
    """A seeded perturbation of the Gaussian parameters (a 'current iterate')."""
    r1, r2, r3, r4 = _streams(seed, 4)
    n = problem.n_gauss
    mu = problem.mean + r1.normal(0, d_mu, (n, 3))
    ls = problem.log_scale + r2.normal(0, d_ls, (n, 3))
    q = problem.quat + r3.normal(0, d_q, (n, 4))
    c = problem.amp + r4.normal(0, d_c, n)
    return _f32(mu, ls, q, c)


def gaussian_noise(seed: int, n: int, sigma: float):
    return (np.random.default_rng(seed).standard_normal(n) * sigma).astype(np.float32)


def rician(clean: np.ndarray, seed: int, sigma: float):
    """Rician magnitude noise: sqrt((y + n1)^2 + n2^2), n1, n2 ~ N(0, sigma^2)."""
    r = np.random.default_rng(seed)
    n1 = r.standard_normal(clean.shape) * sigma
    n2 = r.standard_normal(clean.shape) * sigma
    return np.sqrt((clean.astype(np.float64) + n1) ** 2 + n2 ** 2).astype(np.float32)


def tiny(seed: int, n_gauss: int = 6, n_slices: int = 2, size=(9, 11), spacing=(1.0, 1.2),
         thickness: float = 2.5, half: float = 4.0, max_deg=10.0, max_mm=1.0) -> Problem:
    """A tiny random problem for brute-force and finite-difference pins."""
    r_mu, r_s, r_q, r_c, r_o, r_mot = _streams(seed, 6)
    mu, ls, q, c = cube_gaussians(r_mu, r_s, r_q, r_c, n_gauss, half, 0.6, 2.0)
    q = q * r_q.uniform(0.5, 2.0, size=(n_gauss, 1))        # non-unit storage
    stacks = []
    for k in range(n_slices):
        o = Rotation.from_rotvec(r_o.normal(0, 0.8, 3)).as_matrix()
        stacks.append(dict(orient=o, n=1, H=size[0], W=size[1], dx=spacing[0], dy=spacing[1],
                           thick=thickness, fwhm=[spacing[0], spacing[1], thickness],
                           centre=r_o.uniform(-1.5, 1.5, 3)))
    rot, trans, H, W, sp, fw, subj = _assemble_slices(stacks)
    pose = _motion_uniform(r_mot, len(H), max_deg, max_mm)
    mask = (np.random.default_rng(seed + 7).uniform(size=int((H * W).sum())) < 0.85).astype(np.float32)
    mu, ls, q, c, sp, fw, rot, trans, pose = _f32(mu, ls, q, c, sp, fw, rot, trans, pose)
    return Problem(mu, ls, q, c, np.array([0, n_gauss], np.int64), subj, H, W, sp, fw,
                   rot, trans, pose, mask, name="tiny")


def head_observation(problem: Problem, seed: int, snr: float = 20.0, thickness_samples: int = 5):
    """Synthetic observed slices of the head phantom (not of its Gaussian fit):
    the piecewise-constant phantom times its bias field, averaged over
    ``thickness_samples`` points across the slice thickness at every pixel
    centre of the true pose, with Rician noise at the given SNR.  An input
    only: it involves no Gaussian-model arithmetic."""
    axes = problem.extra["axes"]
    bp = problem.extra["bias"]
    out = []
    offs = (np.arange(thickness_samples) - (thickness_samples - 1) / 2) / thickness_samples
    for i in range(problem.n_slices):
        R = Rotation.from_rotvec(problem.pose[i, :3].astype(np.float64)).as_matrix() @ problem.rot0[i].reshape(3, 3)
        normal = R[:, 2]
        th = float(problem.psf_fwhm[i, 2])
        pos = pixel_world_positions(problem.rot0, problem.trans0, problem.pose, problem.height, problem.width,
                                    problem.spacing, slice_ids=[i])[0]
        acc = np.zeros(len(pos))
        for o in offs:
            x = pos + (o * th) * normal[None, :]
            acc += head_intensity(x, axes) * head_bias(x, bp, axes)
        out.append(acc / thickness_samples)
    clean = np.concatenate(out)
    m = problem.mask > 0
    sigma = float(clean[m].mean()) / snr if m.any() else 0.05
    return rician(clean, seed, sigma)


def init_uniforms(seed: int, n: int) -> np.ndarray:
    """Uniform draws in [0, 1) for the content-adaptive initialisation, [n,4]
    float32: pixel choice, column offset, row offset, through-plane offset."""
    return np.random.default_rng(seed).random((n, 4), dtype=np.float32)


def textured_image(problem: Problem, seed: int) -> np.ndarray:
    """A slice image [P] with homogeneous regions and sharp edges: a few
    random-intensity discs per slice over a constant background, plus weak
    noise (float32)."""
    rng = np.random.default_rng(seed)
    out = np.empty(problem.n_pixels, np.float32)
    po = problem.pix_offset
    for i in range(problem.n_slices):
        h, w = int(problem.height[i]), int(problem.width[i])
        rr, cc = np.mgrid[0:h, 0:w].astype(np.float64)
        img = np.full((h, w), 0.2)
        for _ in range(4):
            r0, c0 = rng.uniform(0, h), rng.uniform(0, w)
            rad = rng.uniform(0.15, 0.4) * min(h, w)
            img[(rr - r0) ** 2 + (cc - c0) ** 2 <= rad * rad] = rng.uniform(0.3, 1.0)
        img += rng.normal(0.0, 0.01, (h, w))
        out[po[i]:po[i + 1]] = img.ravel()
    return out
