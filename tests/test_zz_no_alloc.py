"""dgs_sort_pairs_noalloc (the sort whose scratch is a static device array)
against dgs_sort_pairs, through the C ABI, on consecutive calls of shrinking
size: the static array keeps each call's leftovers, which must not leak into
the next call's result."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

pytestmark = pytest.mark.gpu


def _keys(n, bits, seed):
    rng = np.random.default_rng(seed)
    # few distinct values so that ties (stability) matter
    k = rng.integers(0, max(4, n // 3), n, dtype=np.int64).astype(np.uint64) * np.uint64(0x9E3779B97F4A7C15)
    if bits < 64:
        k &= np.uint64((1 << bits) - 1)
    return k


def test_noalloc_sort_equals_allocating_sort():
    if not torch.cuda.is_available():
        pytest.skip("no HIP device")
    from paper_2508_03180_amd import _capi
    from paper_2508_03180_amd.renderer import Renderer
    r = Renderer(0)
    nmax = _capi.DGS_SORT_NOALLOC_MAX_KEYS
    # full size (6 passes, result in place), then smaller with an odd pass
    # count (result copied back from the scratch array), then small again
    for n, bits, seed in ((nmax, 47, 1), (300_001, 24, 2), (4_097, 64, 3)):
        print(f"noalloc sort n={n} bits={bits}", flush=True)
        k = _keys(n, bits, seed)
        v = np.arange(n, dtype=np.int32)
        ka = torch.from_numpy(k.view(np.int64)).cuda()
        va = torch.from_numpy(v).cuda()
        kb, vb = ka.clone(), va.clone()
        _capi.check(_capi.dgs_sort_pairs(r.ctx, ka.data_ptr(), va.data_ptr(), n, bits), r.ctx)
        _capi.check(_capi.dgs_sort_pairs_noalloc(r.ctx, kb.data_ptr(), vb.data_ptr(), n, bits), r.ctx)
        _capi.check(_capi.dgs_sync(r.ctx), r.ctx)
        assert torch.equal(ka, kb) and torch.equal(va, vb)
        order = np.argsort(k, kind="stable")
        np.testing.assert_array_equal(vb.cpu().numpy(), v[order])
    # sizes beyond the static array are refused before anything is enqueued
    big = torch.zeros(nmax + 1, dtype=torch.int64, device="cuda")
    bigv = torch.zeros(nmax + 1, dtype=torch.int32, device="cuda")
    assert _capi.dgs_sort_pairs_noalloc(r.ctx, big.data_ptr(), bigv.data_ptr(), nmax + 1, 40) == \
        _capi.DGS_ERR_INVALID_ARG
    assert "at most" in _capi.dgs_last_error(r.ctx)
    assert _capi.dgs_sort_pairs_noalloc(r.ctx, big.data_ptr(), bigv.data_ptr(), 0, 40) == _capi.DGS_OK
    assert _capi.dgs_sync(r.ctx) == _capi.DGS_OK
    r.close()
