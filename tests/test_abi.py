"""Host-side checks of the C ABI: the library loads, exports every symbol
include/svr.h declares, and validates arguments without a GPU."""
import ctypes as C
import os
import re

import numpy as np
import pytest

from paper_2512_11624_amd import svr, synth

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    names = set()
    for f in os.listdir(os.path.join(ROOT, "include")):
        if f.endswith(".h"):
            txt = open(os.path.join(ROOT, "include", f)).read()
            txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
            names |= set(re.findall(r"\b(svr_[a-z_0-9]+)\s*\(", txt))
    return names


def test_library_exports_every_declared_symbol():
    lib = svr.load()
    names = _declared()
    assert len(names) >= 15
    for n in sorted(names):
        assert hasattr(lib, n), n
    assert set(svr.declared_symbols()) == names


def test_abi_version_and_status_strings():
    lib = svr.load()
    assert lib.svr_abi_version() == 2
    for code, name in [(0, b"SVR_OK"), (-1, b"SVR_ERR_ARG"), (-2, b"SVR_ERR_HIP"), (-3, b"SVR_ERR_CAPACITY"),
                       (-4, b"SVR_ERR_STATE"), (-5, b"SVR_ERR_NODEVICE"), (-6, b"SVR_ERR_NONFINITE"),
                       (99, b"SVR_ERR_UNKNOWN")]:
        assert lib.svr_status_string(code) == name


def test_ctx_create_argument_errors():
    lib = svr.load()
    assert lib.svr_ctx_create(None, 0, None) == svr.SVR_ERR_ARG
    h = C.c_void_p()
    assert lib.svr_ctx_create(C.byref(h), -7, None) == svr.SVR_ERR_ARG
    assert lib.svr_ctx_destroy(None) == svr.SVR_OK


def test_host_only_context_validates_geometry():
    ctx = svr.Context(device=-1)
    p = synth.config1(0)
    ctx.svr_set_geometry(p)
    assert ctx.n_pixels == p.n_pixels
    st = ctx.svr_get_stats()
    assert st["n_tiles"] == 48 * 4 and st["key_bits"] == 8 + 6
    ctx.svr_set_config(tile=8)
    assert ctx.svr_get_stats()["n_tiles"] == 48 * 16
    ctx.svr_set_config(tile=32)
    assert ctx.svr_get_stats()["n_tiles"] == 48
    bad = synth.config1(0)
    bad.spacing[3, 1] = -1.0
    with pytest.raises(svr.SvrError) as e:
        ctx.svr_set_geometry(bad)
    assert e.value.status == svr.SVR_ERR_ARG and "spacing" in str(e.value)
    bad = synth.config1(0)
    bad.slice_subject[5] = 1
    with pytest.raises(svr.SvrError):
        ctx.svr_set_geometry(bad)          # subject out of range
    bad = synth.concat([synth.tiny(1), synth.tiny(2)])
    bad.slice_subject[:] = bad.slice_subject[::-1]
    with pytest.raises(svr.SvrError):
        ctx.svr_set_geometry(bad)          # subjects not grouped in order


def test_host_only_context_config_and_state_errors():
    ctx = svr.Context(device=-1)
    for cfg in (dict(tile=12), dict(batch=48), dict(batch=512), dict(persistent=2), dict(cutoff=0.0),
                dict(cutoff=9.0)):
        with pytest.raises(svr.SvrError) as e:
            ctx.svr_set_config(**cfg)
        assert e.value.status == svr.SVR_ERR_ARG
    lib = svr.load()
    assert lib.svr_project_bin(ctx.h, None) == svr.SVR_ERR_ARG
    dummy = C.c_void_p(16)
    p = svr.svr_params(dummy, dummy, dummy, dummy, dummy)
    assert lib.svr_project_bin(ctx.h, C.byref(p)) == svr.SVR_ERR_STATE      # no geometry yet
    ctx.svr_set_geometry(synth.config1(0))
    assert lib.svr_project_bin(ctx.h, C.byref(svr.svr_params())) == svr.SVR_ERR_ARG  # NULL pointers
    assert lib.svr_project_bin(ctx.h, C.byref(p)) == svr.SVR_ERR_NODEVICE
    assert lib.svr_forward(ctx.h, None, None, dummy, None, None, None) == svr.SVR_ERR_STATE
    assert lib.svr_forward(ctx.h, None, None, None, None, None, None) == svr.SVR_ERR_ARG
    assert lib.svr_forward(ctx.h, None, None, dummy, dummy, None, None) == svr.SVR_ERR_ARG
    g = svr.svr_grads(dummy, dummy, dummy, dummy, dummy)
    assert lib.svr_backward(ctx.h, dummy, None, C.byref(g)) == svr.SVR_ERR_STATE
    hp = svr.svr_adam((C.c_float * 6)(*[1e-2] * 6), 0.9, 0.999, 1e-8, 0.0)
    assert lib.svr_step(ctx.h, C.byref(g), C.byref(g), dummy, dummy, C.byref(hp), 0) == svr.SVR_ERR_ARG
    hp.beta1 = 1.5
    assert lib.svr_step(ctx.h, C.byref(g), C.byref(g), dummy, dummy, C.byref(hp), 1) == svr.SVR_ERR_ARG
    assert lib.svr_sort_pairs(ctx.h, None, None, 5, 8) == svr.SVR_ERR_ARG
    assert lib.svr_sort_pairs(ctx.h, dummy, dummy, 5, 33) == svr.SVR_ERR_ARG
    assert b"key_bits" in lib.svr_last_error(ctx.h)
    assert lib.svr_init_cdf(ctx.h, dummy, None, 0.5, dummy, None) == svr.SVR_ERR_NODEVICE
    assert lib.svr_init_means(ctx.h, dummy, None, dummy, 0.5, dummy, dummy, None, None) == svr.SVR_ERR_NODEVICE
    assert lib.svr_slice_loss(ctx.h, dummy, dummy, dummy, None, None, None, None, None, None, None) == \
        svr.SVR_ERR_NODEVICE
    assert lib.svr_topk_build(ctx.h, dummy, dummy, None, 8, dummy) == svr.SVR_ERR_NODEVICE


def test_capacity_error_on_too_many_subject_slices():
    ctx = svr.Context(device=-1)
    base = synth.tiny(0, n_slices=1)
    M = 4097
    rep = lambda a: np.repeat(a[:1], M, axis=0)
    p = synth.Problem(base.mean, base.log_scale, base.quat, base.amp, base.gauss_offsets,
                      np.zeros(M, np.int32), np.full(M, 2, np.int32), np.full(M, 2, np.int32),
                      rep(base.spacing), rep(base.psf_fwhm), rep(base.rot0), rep(base.trans0), rep(base.pose),
                      np.ones(4 * M, np.float32))
    with pytest.raises(svr.SvrError) as e:
        ctx.svr_set_geometry(p)
    assert e.value.status == svr.SVR_ERR_CAPACITY


def test_library_is_loaded_from_the_package_tree():
    lib = svr.load()
    assert os.path.dirname(svr.LIB_PATH) == os.path.join(ROOT, "paper_2512_11624_amd")


def test_capacity_and_check_argument_errors():
    """Fixed-capacity binning and finite checks: host-side argument checks."""
    ctx = svr.Context(device=-1)
    lib = svr.load()
    for rec, inst in ((-1, 10), (10, -1), (0, 10), (10, 0)):
        assert lib.svr_set_capacity(ctx.h, rec, inst) == svr.SVR_ERR_ARG
        assert b"capacities" in lib.svr_last_error(ctx.h)
    assert lib.svr_set_capacity(ctx.h, 2 ** 31, 10) == svr.SVR_ERR_CAPACITY
    assert lib.svr_set_capacity(ctx.h, 1000, 5000) == svr.SVR_OK   # host-only: nothing to allocate
    assert lib.svr_set_capacity(ctx.h, 0, 0) == svr.SVR_OK
    assert lib.svr_set_checks(ctx.h, 4) == svr.SVR_ERR_ARG
    assert lib.svr_set_checks(ctx.h, svr.SVR_CHECK_FINITE) == svr.SVR_OK
    assert lib.svr_set_checks(ctx.h, 0) == svr.SVR_OK
    nr, ni = C.c_int64(7), C.c_int64(7)
    assert lib.svr_check_status(ctx.h, C.byref(nr), C.byref(ni)) == svr.SVR_ERR_NODEVICE
    assert nr.value == 0 and ni.value == 0
    assert lib.svr_set_capacity(None, 1, 1) == svr.SVR_ERR_ARG
    assert lib.svr_check_status(None, None, None) == svr.SVR_ERR_ARG


def test_noalloc_sort_argument_errors():
    """svr_sort_pairs_noalloc: host-side checks before any device work."""
    ctx = svr.Context(device=-1)
    lib = svr.load()
    dummy = C.c_void_p(16)
    assert lib.svr_sort_pairs_noalloc(None, dummy, dummy, 10, 8) == svr.SVR_ERR_ARG
    assert lib.svr_sort_pairs_noalloc(ctx.h, dummy, dummy, -1, 8) == svr.SVR_ERR_ARG
    assert lib.svr_sort_pairs_noalloc(ctx.h, dummy, dummy, 10, 0) == svr.SVR_ERR_ARG
    assert lib.svr_sort_pairs_noalloc(ctx.h, dummy, dummy, 10, 33) == svr.SVR_ERR_ARG
    assert lib.svr_sort_pairs_noalloc(ctx.h, None, dummy, 10, 8) == svr.SVR_ERR_ARG
    assert lib.svr_sort_pairs_noalloc(ctx.h, dummy, dummy, svr.SVR_SORT_NOALLOC_MAX + 1, 8) == svr.SVR_ERR_CAPACITY
    assert b"allocation-free maximum" in lib.svr_last_error(ctx.h)
    assert lib.svr_sort_pairs_noalloc(ctx.h, dummy, dummy, svr.SVR_SORT_NOALLOC_MAX, 8) == svr.SVR_ERR_NODEVICE
