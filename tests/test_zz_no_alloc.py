"""The allocation-free sort entry point (svr_sort_pairs_noalloc) against the
allocating one (svr_sort_pairs), through the C ABI: bit-identical keys and
values on two calls in a row, the first at the maximum size and the second
smaller, both also checked against numpy's stable argsort."""
import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
if not torch.cuda.is_available():
    pytest.skip("needs a GPU", allow_module_level=True)

from paper_2512_11624_amd import svr  # noqa: E402


def _pairs(rng, n, bits):
    hi = 2 ** bits
    keys = rng.integers(0, hi, size=n, dtype=np.uint64).astype(np.uint32)
    keys[: n // 4] = keys[0]  # a long run of equal keys: the order of equals is checked
    # bits above key_bits travel with the keys and do not affect the order
    keys |= rng.integers(0, 2**32, size=n, dtype=np.uint64).astype(np.uint32) & ~np.uint32(hi - 1)
    vals = rng.integers(0, 2**32, size=n, dtype=np.uint64).astype(np.uint32)
    return keys, vals


def _dev(a):
    return torch.from_numpy(a.view(np.int32).copy()).cuda()


def test_noalloc_sort_matches_allocating_sort():
    ctx = svr.Context(0)
    rng = np.random.default_rng(42)
    try:
        for n, bits in ((svr.SVR_SORT_NOALLOC_MAX, 20), (300001, 13)):
            keys, vals = _pairs(rng, n, bits)
            ka, va = _dev(keys), _dev(vals)
            kb, vb = _dev(keys), _dev(vals)
            ctx.svr_sort_pairs(ka, va, bits)
            ctx.svr_sort_pairs_noalloc(kb, vb, bits)
            torch.cuda.synchronize()
            kb_h, vb_h = kb.cpu().numpy().view(np.uint32), vb.cpu().numpy().view(np.uint32)
            assert np.array_equal(kb_h, ka.cpu().numpy().view(np.uint32)), (n, bits)
            assert np.array_equal(vb_h, va.cpu().numpy().view(np.uint32)), (n, bits)
            order = np.argsort(keys & np.uint32(2 ** bits - 1), kind="stable")
            assert np.array_equal(kb_h, keys[order]), (n, bits)
            assert np.array_equal(vb_h, vals[order]), (n, bits)
        # above the maximum: refused on the host, the buffers untouched
        n = svr.SVR_SORT_NOALLOC_MAX + 1
        k = torch.zeros(n, dtype=torch.int32, device="cuda")
        v = torch.arange(n, dtype=torch.int32, device="cuda")
        with pytest.raises(svr.SvrError) as e:
            ctx.svr_sort_pairs_noalloc(k, v, 8)
        assert e.value.status == svr.SVR_ERR_CAPACITY
        torch.cuda.synchronize()
        assert torch.equal(v, torch.arange(n, dtype=torch.int32, device="cuda"))
    finally:
        ctx.close()
