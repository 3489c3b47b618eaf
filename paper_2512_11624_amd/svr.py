"""ctypes binding of libsvr (``include/svr.h``): argument marshalling only.

Every computation runs in the HIP kernels of ``libsvr.so``; PyTorch provides
device memory and the stream.  The functions keep the C names
(``svr_project_bin``, ``svr_forward``, ``svr_backward``, ``svr_step``, ...);
:class:`Context` wraps a ``svr_ctx*`` and :class:`SvrRender` exposes the
forward/adjoint pair to ``torch.autograd``.
"""
from __future__ import annotations

import ctypes as C
import os
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsvr.so")
_lib = None
_lock = threading.Lock()

SVR_OK, SVR_ERR_ARG, SVR_ERR_HIP, SVR_ERR_CAPACITY, SVR_ERR_STATE, SVR_ERR_NODEVICE = 0, -1, -2, -3, -4, -5
SVR_ERR_NONFINITE = -6
SVR_CHECK_FINITE = 1
SVR_STATS_SYNC = 1
SVR_SORT_NOALLOC_MAX = 1 << 20
SVR_TUNE_TILE, SVR_TUNE_BATCH, SVR_TUNE_PERSISTENT, SVR_TUNE_MODE, SVR_TUNE_ALL = 1, 2, 4, 8, 15
SVR_LOSS_MSE, SVR_LOSS_L1 = 0, 1

vp = C.c_void_p


class svr_geometry(C.Structure):
    _fields_ = [("n_subjects", C.c_int32), ("gauss_offsets", vp), ("n_slices", C.c_int32),
                ("slice_subject", vp), ("height", vp), ("width", vp), ("spacing", vp),
                ("psf_fwhm", vp), ("rot0", vp), ("trans0", vp)]


class svr_config(C.Structure):
    _fields_ = [("tile", C.c_int32), ("batch", C.c_int32), ("persistent", C.c_int32),
                ("cutoff", C.c_float), ("forward_mode", C.c_int32)]

    def as_dict(self):
        return dict(tile=self.tile, batch=self.batch, persistent=self.persistent, cutoff=self.cutoff,
                    forward_mode=self.forward_mode)


class svr_params(C.Structure):
    _fields_ = [("mean", vp), ("log_scale", vp), ("quat", vp), ("amp", vp), ("pose", vp)]


class svr_grads(C.Structure):
    _fields_ = [("mean", vp), ("log_scale", vp), ("quat", vp), ("amp", vp), ("pose", vp)]


class svr_adam(C.Structure):
    _fields_ = [("lr", C.c_float * 6), ("beta1", C.c_double), ("beta2", C.c_double),
                ("eps", C.c_double), ("weight_decay", C.c_double)]


class svr_densify_cfg(C.Structure):
    _fields_ = [("grad_threshold", C.c_float), ("log_scale_threshold", C.c_float), ("split_offset", C.c_float),
                ("clone_offset", C.c_float), ("prune_amp", C.c_float)]


class svr_timer(C.Structure):
    _fields_ = [("name", C.c_char * 32), ("calls", C.c_int64), ("total_ms", C.c_double)]


class svr_stats(C.Structure):
    _fields_ = [("n_gauss", C.c_int64), ("n_slices", C.c_int64), ("n_pixels", C.c_int64),
                ("n_tiles", C.c_int64), ("n_candidates", C.c_int64), ("n_records", C.c_int64),
                ("n_instances", C.c_int64), ("n_incut", C.c_int64), ("n_evaluated", C.c_int64),
                ("key_bits", C.c_int32), ("sort_passes", C.c_int32), ("n_fallback_blocks", C.c_int64)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


_SIGS = {
    "svr_abi_version": ([], C.c_int),
    "svr_status_string": ([C.c_int], C.c_char_p),
    "svr_ctx_create": ([C.POINTER(vp), C.c_int, vp], C.c_int),
    "svr_ctx_destroy": ([vp], C.c_int),
    "svr_set_stream": ([vp, vp], C.c_int),
    "svr_last_error": ([vp], C.c_char_p),
    "svr_set_geometry": ([vp, C.POINTER(svr_geometry)], C.c_int),
    "svr_num_pixels": ([vp], C.c_int64),
    "svr_set_config": ([vp, C.POINTER(svr_config)], C.c_int),
    "svr_get_config": ([vp, C.POINTER(svr_config)], C.c_int),
    "svr_project_bin": ([vp, C.POINTER(svr_params)], C.c_int),
    "svr_forward": ([vp, vp, vp, vp, vp, vp, vp], C.c_int),
    "svr_backward": ([vp, vp, vp, C.POINTER(svr_grads)], C.c_int),
    "svr_step": ([vp, C.POINTER(svr_grads), C.POINTER(svr_grads), vp, vp, C.POINTER(svr_adam),
                  C.c_int64], C.c_int),
    "svr_set_count_pairs": ([vp, C.c_int], C.c_int),
    "svr_get_stats": ([vp, C.c_int, C.POINTER(svr_stats)], C.c_int),
    "svr_sort_pairs": ([vp, vp, vp, C.c_int64, C.c_int], C.c_int),
    "svr_sort_pairs_noalloc": ([vp, vp, vp, C.c_int64, C.c_int], C.c_int),
    "svr_set_capacity": ([vp, C.c_int64, C.c_int64], C.c_int),
    "svr_set_checks": ([vp, C.c_int], C.c_int),
    "svr_check_status": ([vp, C.POINTER(C.c_int64), C.POINTER(C.c_int64)], C.c_int),
    "svr_set_timing": ([vp, C.c_int], C.c_int),
    "svr_get_timing": ([vp, C.POINTER(svr_timer), C.c_int, C.POINTER(C.c_int)], C.c_int),
    "svr_set_timing_stages": ([vp, C.c_uint32], C.c_int),
    "svr_posenet_create": ([C.POINTER(vp), C.c_int, vp, C.c_uint64, C.c_int], C.c_int),
    "svr_posenet_destroy": ([vp], C.c_int),
    "svr_posenet_num_params": ([vp], C.c_int64),
    "svr_posenet_get_params": ([vp, vp], C.c_int),
    "svr_posenet_set_params": ([vp, vp], C.c_int),
    "svr_posenet_prepare": ([vp, vp, C.c_int, C.c_int, C.c_int, vp], C.c_int),
    "svr_posenet_forward": ([vp, vp, vp, C.c_int, vp], C.c_int),
    "svr_posenet_train_step": ([vp, vp, vp, vp, C.c_int, C.c_float, vp], C.c_int),
    "svr_posenet_grads": ([vp, vp, vp, vp, C.c_int, vp, vp], C.c_int),
    "svr_conv3x3s2_forward": ([vp, vp, vp, vp, vp, C.c_int, C.c_int, C.c_int, C.c_int, C.c_int, C.c_int], C.c_int),
    "svr_conv3x3s2_dgrad": ([vp, vp, vp, vp, vp, C.c_int, C.c_int, C.c_int, C.c_int, C.c_int], C.c_int),
    "svr_conv3x3s2_wgrad": ([vp, vp, vp, vp, vp, vp, C.c_int, C.c_int, C.c_int, C.c_int, C.c_int], C.c_int),
    "svr_linear_forward": ([vp, vp, vp, vp, vp, C.c_int, C.c_int, C.c_int, C.c_int], C.c_int),
    "svr_linear_dgrad": ([vp, vp, vp, vp, vp, C.c_int, C.c_int, C.c_int], C.c_int),
    "svr_linear_wgrad": ([vp, vp, vp, vp, vp, vp, C.c_int, C.c_int, C.c_int], C.c_int),
    "svr_set_loss": ([vp, C.c_int], C.c_int),
    "svr_scale_regularizer": ([vp, vp, C.c_int64, C.c_float, C.c_float, vp, vp], C.c_int),
    "svr_init_cdf": ([vp, vp, vp, C.c_float, vp, C.POINTER(C.c_int64)], C.c_int),
    "svr_init_means": ([vp, vp, vp, vp, C.c_float, vp, vp, vp, vp], C.c_int),
    "svr_slice_loss": ([vp, vp, vp, vp, vp, vp, vp, vp, vp, vp, vp], C.c_int),
    "svr_adam_vector": ([vp, vp, vp, vp, vp, C.c_int64, C.c_float, C.POINTER(svr_adam), C.c_int64], C.c_int),
    "svr_bias_apply": ([vp, vp, C.c_float, vp, C.c_int32, vp, vp], C.c_int),
    "svr_bias_backward": ([vp, vp, C.c_float, vp, C.c_int32, vp, vp, vp, vp, vp], C.c_int),
    "svr_densify_accumulate": ([vp, vp, vp, vp], C.c_int),
    "svr_densify": ([vp, C.POINTER(svr_params), vp, vp, C.POINTER(svr_densify_cfg), C.POINTER(svr_grads), C.c_int64,
                     vp, vp, vp, vp, vp, vp], C.c_int),
    "svr_topk_build": ([vp, vp, vp, vp, C.c_int, vp], C.c_int),
    "svr_topk_forward": ([vp, C.POINTER(svr_params), vp, vp, C.c_int, C.c_float, vp, vp, vp, vp, vp], C.c_int),
    "svr_topk_backward": ([vp, C.POINTER(svr_params), vp, C.c_int, vp, C.POINTER(svr_grads), vp], C.c_int),
    "svr_autotune": ([vp, C.POINTER(svr_params), vp, C.c_int, C.c_char_p, C.POINTER(svr_config),
                      C.POINTER(C.c_float), C.c_int], C.c_int),
}


def load():
    """Load libsvr.so (built in-tree).  Raises if it is missing: there is no
    fallback implementation."""
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(LIB_PATH):
                raise RuntimeError(f"{LIB_PATH} is missing; build it with "
                                   "`python -m paper_2512_11624_amd.build`")
            lib = C.CDLL(LIB_PATH)
            for name, (args, res) in _SIGS.items():
                f = getattr(lib, name)
                f.argtypes = args
                f.restype = res
            _lib = lib
    return _lib


def declared_symbols():
    return sorted(_SIGS)


class SvrError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{load().svr_status_string(status).decode()}: {msg}")
        self.status = status


def _ptr(t):
    if t is None:
        return None
    return C.c_void_p(t.data_ptr())


def _np(a, dt):
    return np.ascontiguousarray(a, dtype=dt)


class Context:
    """One ``svr_ctx``.  device=-1 gives a host-only context (validation only)."""

    def __init__(self, device: int = 0, stream=None):
        lib = load()
        h = vp()
        if stream is None and device >= 0:
            import torch
            stream = torch.cuda.current_stream(device).cuda_stream
        rc = lib.svr_ctx_create(C.byref(h), int(device), C.c_void_p(stream) if stream else None)
        if rc != SVR_OK:
            raise SvrError(rc, f"svr_ctx_create(device={device})")
        self.h = h
        self.device = device
        self._keep = []
        self.n_gauss = 0
        self.n_slices = 0
        self.n_subjects = 0
        self.n_pixels = 0
        self.bin_generation = 0   # svr_project_bin calls made through this object

    def close(self):
        if getattr(self, "h", None) is not None and self.h.value:
            load().svr_ctx_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, rc, what):
        if rc != SVR_OK:
            raise SvrError(rc, f"{what}: {load().svr_last_error(self.h).decode()}")

    # -- configuration ------------------------------------------------------
    def svr_set_stream(self, stream):
        self._check(load().svr_set_stream(self.h, C.c_void_p(stream)), "svr_set_stream")

    def svr_set_geometry(self, prob):
        """prob: any object with the attributes of ``synth.Problem``."""
        arrs = dict(go=_np(prob.gauss_offsets, np.int64), ss=_np(prob.slice_subject, np.int32),
                    h=_np(prob.height, np.int32), w=_np(prob.width, np.int32),
                    sp=_np(prob.spacing, np.float32), fw=_np(prob.psf_fwhm, np.float32),
                    r0=_np(prob.rot0, np.float32), t0=_np(prob.trans0, np.float32))
        g = svr_geometry(len(arrs["go"]) - 1, arrs["go"].ctypes.data, len(arrs["h"]),
                         arrs["ss"].ctypes.data, arrs["h"].ctypes.data, arrs["w"].ctypes.data,
                         arrs["sp"].ctypes.data, arrs["fw"].ctypes.data, arrs["r0"].ctypes.data,
                         arrs["t0"].ctypes.data)
        self._check(load().svr_set_geometry(self.h, C.byref(g)), "svr_set_geometry")
        self.n_gauss = int(arrs["go"][-1])
        self.n_subjects = int(len(arrs["go"]) - 1)
        self.n_slices = int(len(arrs["h"]))
        self.n_pixels = int(load().svr_num_pixels(self.h))

    def svr_set_config(self, tile=None, batch=None, persistent=None, cutoff=None, forward_mode=None):
        cur = self.svr_get_config()
        cfg = svr_config(cur["tile"] if tile is None else tile, cur["batch"] if batch is None else batch,
                         cur["persistent"] if persistent is None else persistent,
                         cur["cutoff"] if cutoff is None else cutoff,
                         cur["forward_mode"] if forward_mode is None else forward_mode)
        self._check(load().svr_set_config(self.h, C.byref(cfg)), "svr_set_config")

    def svr_get_config(self):
        cfg = svr_config()
        self._check(load().svr_get_config(self.h, C.byref(cfg)), "svr_get_config")
        return cfg.as_dict()

    # -- hot path ------------------------------------------------------------
    def svr_project_bin(self, mean, log_scale, quat, amp, pose):
        p = svr_params(_ptr(mean), _ptr(log_scale), _ptr(quat), _ptr(amp), _ptr(pose))
        self.bin_generation += 1
        self._check(load().svr_project_bin(self.h, C.byref(p)), "svr_project_bin")

    def svr_forward(self, pred, target=None, mask=None, loss=None, slice_sse=None, grad_pred=None):
        rc = load().svr_forward(self.h, _ptr(target), _ptr(mask), _ptr(pred), _ptr(loss),
                                _ptr(slice_sse), _ptr(grad_pred))
        self._check(rc, "svr_forward")

    def svr_backward(self, grad_pred, g_mean, g_log_scale, g_quat, g_amp, g_pose, grad_scale=None):
        g = svr_grads(_ptr(g_mean), _ptr(g_log_scale), _ptr(g_quat), _ptr(g_amp), _ptr(g_pose))
        self._check(load().svr_backward(self.h, _ptr(grad_pred), _ptr(grad_scale), C.byref(g)),
                    "svr_backward")

    def svr_step(self, params, grads, exp_avg, exp_avg_sq, lr, step, beta1=0.9, beta2=0.999,
                 eps=1e-8, weight_decay=0.0):
        """params / grads: 5-tuples (mean, log_scale, quat, amp, pose) of tensors."""
        P = svr_grads(*[_ptr(t) for t in params])
        G = svr_grads(*[_ptr(t) for t in grads])
        hp = svr_adam((C.c_float * 6)(*[float(x) for x in lr]), beta1, beta2, eps, weight_decay)
        self._check(load().svr_step(self.h, C.byref(P), C.byref(G), _ptr(exp_avg), _ptr(exp_avg_sq),
                                    C.byref(hp), int(step)), "svr_step")

    def svr_set_loss(self, kind):
        """kind: SVR_LOSS_MSE (0) or SVR_LOSS_L1 (1)."""
        self._check(load().svr_set_loss(self.h, int(kind)), "svr_set_loss")

    def svr_scale_regularizer(self, log_scale, lam, s_target, g_log_scale, loss=None):
        self._check(load().svr_scale_regularizer(self.h, _ptr(log_scale), int(log_scale.shape[0]), float(lam),
                                                 float(s_target), _ptr(g_log_scale), _ptr(loss)),
                    "svr_scale_regularizer")

    def svr_init_cdf(self, image, mask, lambda_init, cdf):
        """Cumulative Eq. 6 weights into cdf [P] (int64, device); returns the
        subjects' totals as a list."""
        tot = (C.c_int64 * max(1, self.n_subjects))()
        self._check(load().svr_init_cdf(self.h, _ptr(image), _ptr(mask), float(lambda_init), _ptr(cdf), tot),
                    "svr_init_cdf")
        return [int(tot[k]) for k in range(self.n_subjects)]

    def svr_init_means(self, image, mask, pose, lambda_init, u, mean, pixel=None, value=None):
        self._check(load().svr_init_means(self.h, _ptr(image), _ptr(mask), _ptr(pose), float(lambda_init),
                                          _ptr(u), _ptr(mean), _ptr(pixel), _ptr(value)), "svr_init_means")

    def svr_slice_loss(self, pred, target, mask, sigma=None, log_omega=None, loss=None, grad_pred=None,
                       slice_sums=None, g_sigma=None, g_log_omega=None):
        self._check(load().svr_slice_loss(self.h, _ptr(pred), _ptr(target), _ptr(mask), _ptr(sigma), _ptr(log_omega),
                                          _ptr(loss), _ptr(grad_pred), _ptr(slice_sums), _ptr(g_sigma),
                                          _ptr(g_log_omega)), "svr_slice_loss")

    def svr_bias_apply(self, centres, width, beta, K, pred, bias=None):
        self._check(load().svr_bias_apply(self.h, _ptr(centres), float(width), _ptr(beta), int(K), _ptr(pred),
                                          _ptr(bias)), "svr_bias_apply")

    def svr_bias_backward(self, centres, width, beta, K, pred_biased, bias, grad_pred, g_beta, g_pose=None):
        self._check(load().svr_bias_backward(self.h, _ptr(centres), float(width), _ptr(beta), int(K),
                                             _ptr(pred_biased), _ptr(bias), _ptr(grad_pred), _ptr(g_beta),
                                             _ptr(g_pose)), "svr_bias_backward")

    def svr_densify_accumulate(self, g_mean, grad_acc, count):
        self._check(load().svr_densify_accumulate(self.h, _ptr(g_mean), _ptr(grad_acc), _ptr(count)),
                    "svr_densify_accumulate")

    def svr_densify(self, params, grad_acc, count, cfg, out, capacity, src=None, moments_in=None, moments_out=None):
        """params: (mean, log_scale, quat, amp) tensors; cfg: dict of svr_densify_cfg fields; out: four
        tensors with room for ``capacity`` Gaussians; moments_in / moments_out: (exp_avg, exp_avg_sq)
        pairs or None.  Returns the new per-subject offsets (int64 [S + 1]); raises SvrError with
        ``offsets`` set when they need more than ``capacity``."""
        P = svr_params(*[_ptr(t) for t in params[:4]], None)
        O = svr_grads(*[_ptr(t) for t in out[:4]], None)
        c = svr_densify_cfg(**{k: float(v) for k, v in cfg.items()})
        mi = moments_in or (None, None)
        mo = moments_out or (None, None)
        off = np.zeros(self.n_subjects + 1, np.int64)
        rc = load().svr_densify(self.h, C.byref(P), _ptr(grad_acc), _ptr(count), C.byref(c), C.byref(O),
                                int(capacity), _ptr(src), _ptr(mi[0]), _ptr(mi[1]), _ptr(mo[0]), _ptr(mo[1]),
                                off.ctypes.data)
        if rc != SVR_OK:
            err = SvrError(rc, f"svr_densify: {load().svr_last_error(self.h).decode()}")
            err.offsets = off
            raise err
        self.n_gauss = int(off[-1])
        return off

    def densify_params(self, params, grad_acc, count, cfg, exp_avg=None, exp_avg_sq=None):
        """svr_densify on an svr.Params (and its Adam moments, same layout):
        returns (new Params, new exp_avg, new exp_avg_sq, src); the output
        buffers are sized for the worst case 2N."""
        import torch
        N, M, dev = params.N, params.M, params.flat.device
        cap = 2 * N
        out = [torch.empty(max(cap * w, 1), dtype=torch.float32, device=dev) for w in (3, 3, 4, 1)]
        src = torch.empty(max(cap, 1), dtype=torch.int32, device=dev)
        mom = exp_avg is not None
        m_out = [torch.empty(11 * cap + 6 * M, dtype=torch.float32, device=dev) for _ in range(2)] if mom else None
        off = self.svr_densify(params.views()[:4], grad_acc, count, cfg, out, cap, src,
                               (exp_avg, exp_avg_sq) if mom else None, m_out)
        K = int(off[-1])
        new = Params(K, M, device=dev)
        v = new.views()
        for t, o, w in zip(v[:4], out, (3, 3, 4, 1)):
            t.copy_(o[:w * K].view(t.shape))
        v[4].copy_(params.views()[4])
        if mom:
            m_out = [t[:11 * K + 6 * M].clone() for t in m_out]
        return new, (m_out[0] if mom else None), (m_out[1] if mom else None), src[:K]

    def svr_adam_vector(self, p, g, m, v, lr, step, beta1=0.9, beta2=0.999, eps=1e-8, weight_decay=0.0):
        hp = svr_adam((C.c_float * 6)(*[lr] * 6), beta1, beta2, eps, weight_decay)
        self._check(load().svr_adam_vector(self.h, _ptr(p), _ptr(g), _ptr(m), _ptr(v), int(p.numel()), float(lr),
                                           C.byref(hp), int(step)), "svr_adam_vector")

    def svr_topk_build(self, mean, pose, K, nbr, mask=None):
        self._check(load().svr_topk_build(self.h, _ptr(mean), _ptr(pose), _ptr(mask), int(K), _ptr(nbr)),
                    "svr_topk_build")

    def svr_topk_forward(self, mean, log_scale, quat, amp, pose, nbr, K, delta, pred, target=None, mask=None,
                         sigma=None, loss=None, grad_pred=None):
        p = svr_params(*(_ptr(t) for t in (mean, log_scale, quat, amp, pose)))
        self._check(load().svr_topk_forward(self.h, C.byref(p), _ptr(sigma), _ptr(nbr), int(K), float(delta),
                                            _ptr(target), _ptr(mask), _ptr(pred), _ptr(loss), _ptr(grad_pred)),
                    "svr_topk_forward")

    def svr_topk_backward(self, mean, log_scale, quat, amp, pose, nbr, K, grad_pred, g_mean, g_log_scale, g_quat,
                          g_amp, g_pose, g_sigma=None):
        p = svr_params(*(_ptr(t) for t in (mean, log_scale, quat, amp, pose)))
        g = svr_grads(*(_ptr(t) for t in (g_mean, g_log_scale, g_quat, g_amp, g_pose)))
        self._check(load().svr_topk_backward(self.h, C.byref(p), _ptr(nbr), int(K), _ptr(grad_pred), C.byref(g),
                                             _ptr(g_sigma)), "svr_topk_backward")

    def svr_set_count_pairs(self, enable: bool):
        self._check(load().svr_set_count_pairs(self.h, int(bool(enable))), "svr_set_count_pairs")

    def svr_get_stats(self, sync: bool = False):
        s = svr_stats()
        self._check(load().svr_get_stats(self.h, SVR_STATS_SYNC if sync else 0, C.byref(s)),
                    "svr_get_stats")
        return s.as_dict()

    def svr_set_capacity(self, max_records: int, max_instances: int):
        """Fixed-capacity binning (0, 0: back to the default, synchronising mode)."""
        self._check(load().svr_set_capacity(self.h, int(max_records), int(max_instances)), "svr_set_capacity")

    def svr_set_checks(self, flags: int):
        self._check(load().svr_set_checks(self.h, int(flags)), "svr_set_checks")

    def svr_check_status(self):
        """(status, needed_records, needed_instances); the status is returned,
        not raised (SVR_OK, SVR_ERR_CAPACITY or SVR_ERR_NONFINITE)."""
        nr, ni = C.c_int64(0), C.c_int64(0)
        rc = load().svr_check_status(self.h, C.byref(nr), C.byref(ni))
        if rc not in (SVR_OK, SVR_ERR_CAPACITY, SVR_ERR_NONFINITE):
            self._check(rc, "svr_check_status")
        return rc, int(nr.value), int(ni.value)

    def svr_set_timing(self, enable: bool):
        self._check(load().svr_set_timing(self.h, int(bool(enable))), "svr_set_timing")

    def svr_set_timing_stages(self, stages=None):
        """Bracket only the named stages with events (None: all stages)."""
        if stages is None:
            mask = 0xFFFFFFFF
        else:
            order = list(self.svr_get_timing().keys())
            unknown = [s for s in stages if s not in order]
            if unknown:
                raise ValueError(f"unknown stages {unknown}")
            mask = 0
            for s in stages:
                mask |= 1 << order.index(s)
        self._check(load().svr_set_timing_stages(self.h, C.c_uint32(mask)), "svr_set_timing_stages")

    def svr_get_timing(self):
        """{stage: (calls, total_ms)}; synchronises the stream."""
        arr = (svr_timer * 32)()
        n = C.c_int(0)
        self._check(load().svr_get_timing(self.h, arr, 32, C.byref(n)), "svr_get_timing")
        return {arr[k].name.decode(): (int(arr[k].calls), float(arr[k].total_ms)) for k in range(n.value)}

    def svr_sort_pairs(self, keys, vals, key_bits):
        self._check(load().svr_sort_pairs(self.h, _ptr(keys), _ptr(vals), int(keys.numel()), int(key_bits)),
                    "svr_sort_pairs")

    def svr_sort_pairs_noalloc(self, keys, vals, key_bits):
        """Asynchronous on the context's stream; allocates nothing."""
        self._check(load().svr_sort_pairs_noalloc(self.h, _ptr(keys), _ptr(vals), int(keys.numel()),
                                                  int(key_bits)), "svr_sort_pairs_noalloc")

    def svr_autotune(self, mean, log_scale, quat, amp, pose, grad_pred, flags=SVR_TUNE_ALL,
                     cache_path=None, max_times=64):
        p = svr_params(_ptr(mean), _ptr(log_scale), _ptr(quat), _ptr(amp), _ptr(pose))
        out = svr_config()
        times = (C.c_float * max_times)()
        rc = load().svr_autotune(self.h, C.byref(p), _ptr(grad_pred), int(flags),
                                 cache_path.encode() if cache_path else None, C.byref(out), times,
                                 max_times)
        self._check(rc, "svr_autotune")
        return out.as_dict(), [t for t in times if t > 0]


class Params:
    """Device parameters in one flat float32 buffer, laid out like the Adam
    state of ``svr_step``: mean (3N), log_scale (3N), quat (4N), amp (N),
    pose (6M).  ``views()`` returns the five views."""

    def clone(self):
        p = Params(self.N, self.M, device=self.flat.device)
        p.flat.copy_(self.flat)
        return p

    def __init__(self, n_gauss, n_slices, device="cuda"):
        import torch
        self.N, self.M = int(n_gauss), int(n_slices)
        self.flat = torch.zeros(self.N * 11 + self.M * 6, dtype=torch.float32, device=device)

    def views(self):
        N, M, f = self.N, self.M, self.flat
        return (f[:3 * N].view(N, 3), f[3 * N:6 * N].view(N, 3), f[6 * N:10 * N].view(N, 4),
                f[10 * N:11 * N], f[11 * N:11 * N + 6 * M].view(M, 6))

    @classmethod
    def from_arrays(cls, mean, log_scale, quat, amp, pose, device="cuda"):
        import torch
        p = cls(len(amp), len(pose), device)
        for v, a in zip(p.views(), (mean, log_scale, quat, amp, pose)):
            v.copy_(torch.as_tensor(np.ascontiguousarray(a, np.float32)))
        return p


def _grad_fn():
    import torch

    class SvrRender(torch.autograd.Function):
        """loss, pred = SvrRender.apply(ctx, mean, log_scale, quat, amp, pose, target, mask).

        Forward: svr_project_bin + svr_forward (prediction, masked-MSE loss and
        dL/dpred).  Backward: svr_backward scaled by the upstream loss gradient.
        ``pred`` is not differentiable (gradients flow through the loss).

        svr_backward uses the context's last binning; when the context has
        binned other parameters since this forward (another render_loss on the
        same context), backward first bins the saved parameters again."""

        @staticmethod
        def forward(fctx, sctx, mean, log_scale, quat, amp, pose, target, mask):
            dev = mean.device
            sctx.svr_project_bin(mean, log_scale, quat, amp, pose)
            pred = torch.empty(sctx.n_pixels, dtype=torch.float32, device=dev)
            loss = torch.empty(1, dtype=torch.float32, device=dev)
            gpred = torch.empty_like(pred)
            sctx.svr_forward(pred, target, mask, loss=loss, grad_pred=gpred)
            fctx.sctx = sctx
            fctx.generation = sctx.bin_generation
            fctx.save_for_backward(gpred, mean, log_scale, quat, amp, pose)
            fctx.mark_non_differentiable(pred)
            return loss[0], pred

        @staticmethod
        def backward(fctx, g_loss, g_pred):
            gpred, mean, log_scale, quat, amp, pose = fctx.saved_tensors
            if fctx.sctx.bin_generation != fctx.generation:
                fctx.sctx.svr_project_bin(mean, log_scale, quat, amp, pose)
                fctx.generation = fctx.sctx.bin_generation
            grads = [torch.empty_like(t) for t in (mean, log_scale, quat, amp, pose)]
            scale = g_loss.reshape(1).to(torch.float32).contiguous()
            fctx.sctx.svr_backward(gpred, *grads, grad_scale=scale)
            return (None, *grads, None, None)

    return SvrRender


_svr_render = None


def SvrRender():
    global _svr_render
    if _svr_render is None:
        _svr_render = _grad_fn()
    return _svr_render


def render_loss(sctx, mean, log_scale, quat, amp, pose, target, mask):
    return SvrRender().apply(sctx, mean, log_scale, quat, amp, pose, target, mask)


class PoseNet:
    """The pose-proposal CNN (``svr_posenet_*``): argument marshalling only."""

    def __init__(self, device=0, seed=0, max_batch=256, stream=None):
        import torch
        lib = load()
        h = vp()
        if stream is None:
            stream = torch.cuda.current_stream(device).cuda_stream
        rc = lib.svr_posenet_create(C.byref(h), int(device), C.c_void_p(stream) if stream else None, int(seed),
                                    int(max_batch))
        if rc != SVR_OK:
            raise SvrError(rc, "svr_posenet_create")
        self.h = h
        self.device = device
        self.max_batch = max_batch
        self.n_params = int(lib.svr_posenet_num_params(h))

    def close(self):
        if getattr(self, "h", None) is not None and self.h.value:
            load().svr_posenet_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _chk(self, rc, what):
        if rc != SVR_OK:
            raise SvrError(rc, what)

    def get_params(self):
        out = np.zeros(self.n_params, np.float32)
        self._chk(load().svr_posenet_get_params(self.h, out.ctypes.data), "svr_posenet_get_params")
        return out

    def set_params(self, arr):
        a = np.ascontiguousarray(arr, np.float32)
        assert a.size == self.n_params
        self._chk(load().svr_posenet_set_params(self.h, a.ctypes.data), "svr_posenet_set_params")

    def prepare(self, slices, crops):
        B, H, W = slices.shape
        self._chk(load().svr_posenet_prepare(self.h, _ptr(slices), B, H, W, _ptr(crops)), "svr_posenet_prepare")

    def forward(self, crops, orient, out):
        self._chk(load().svr_posenet_forward(self.h, _ptr(crops), _ptr(orient), int(crops.shape[0]), _ptr(out)),
                  "svr_posenet_forward")

    def train_step(self, crops, orient, target, lr, loss=None):
        self._chk(load().svr_posenet_train_step(self.h, _ptr(crops), _ptr(orient), _ptr(target), int(crops.shape[0]),
                                                float(lr), _ptr(loss)), "svr_posenet_train_step")

    def grads(self, crops, orient, target, loss, grads_out):
        self._chk(load().svr_posenet_grads(self.h, _ptr(crops), _ptr(orient), _ptr(target), int(crops.shape[0]),
                                           _ptr(loss), _ptr(grads_out)), "svr_posenet_grads")


def _stream():
    import torch
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def conv3x3s2_forward(x, w, b, y, relu):
    B, Ci, H, W = x.shape
    rc = load().svr_conv3x3s2_forward(_stream(), _ptr(x), _ptr(w), _ptr(b), _ptr(y), B, Ci, H, W, w.shape[0], int(relu))
    if rc != SVR_OK:
        raise SvrError(rc, "svr_conv3x3s2_forward")


def conv3x3s2_dgrad(dy, y, w, dx):
    B, Ci, H, W = dx.shape
    rc = load().svr_conv3x3s2_dgrad(_stream(), _ptr(dy), _ptr(y), _ptr(w), _ptr(dx), B, Ci, H, W, w.shape[0])
    if rc != SVR_OK:
        raise SvrError(rc, "svr_conv3x3s2_dgrad")


def conv3x3s2_wgrad(dy, y, x, dw, db):
    B, Ci, H, W = x.shape
    rc = load().svr_conv3x3s2_wgrad(_stream(), _ptr(dy), _ptr(y), _ptr(x), _ptr(dw), _ptr(db), B, Ci, H, W,
                                    dw.shape[0])
    if rc != SVR_OK:
        raise SvrError(rc, "svr_conv3x3s2_wgrad")


def linear_forward(x, w, b, y, relu):
    rc = load().svr_linear_forward(_stream(), _ptr(x), _ptr(w), _ptr(b), _ptr(y), x.shape[0], x.shape[1], w.shape[0],
                                   int(relu))
    if rc != SVR_OK:
        raise SvrError(rc, "svr_linear_forward")


def linear_dgrad(dy, y, w, dx):
    rc = load().svr_linear_dgrad(_stream(), _ptr(dy), _ptr(y), _ptr(w), _ptr(dx), dy.shape[0], w.shape[1], w.shape[0])
    if rc != SVR_OK:
        raise SvrError(rc, "svr_linear_dgrad")


def linear_wgrad(dy, y, x, dw, db):
    rc = load().svr_linear_wgrad(_stream(), _ptr(dy), _ptr(y), _ptr(x), _ptr(dw), _ptr(db), dy.shape[0], x.shape[1],
                                 dw.shape[0])
    if rc != SVR_OK:
        raise SvrError(rc, "svr_linear_wgrad")
