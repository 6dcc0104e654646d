"""lc_search_noalloc (the walk with the library's fixed workspace array, for
callers that cannot allocate device memory) against lc_search with a caller
workspace, through the C-ABI: identical short-lists, distances, counts and
(E, D), on consecutive calls with a smaller second input, with the slot count
cut to what the array holds, and the rejection of an index too large for one
slot."""
import ctypes as C

import numpy as np
import pytest

import datagen
import oracle

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch():
    import torch as t
    assert t.cuda.is_available(), "GPU tests need a GPU"
    return t


def _same(a, b):
    for x, y in ((a.cand_ids, b.cand_ids), (a.cand_n, b.cand_n), (a.stats, b.stats),
                 (a.cand_adc.view(a.cand_ids.dtype), b.cand_adc.view(b.cand_ids.dtype))):
        assert x.shape == y.shape and bool((x == y).all())


def _calls(gix, q, torch, w):
    import paper_1804_09996_amd as lc
    qt = torch.from_numpy(q)
    first = None
    for lut_dt in (lc.LC_LUT_F32, lc.LC_LUT_F16):
        lut, sc = gix.build_lut(qt, lut_dt)
        # a full batch, then a smaller one with per-query ef, through the same array
        ref = gix.search(lut, sc, ef=None, ef_max=w.ef, S=w.shortlist)
        got = gix.search_noalloc(lut, sc, ef=None, ef_max=w.ef, S=w.shortlist)
        torch.cuda.synchronize()
        _same(got, ref)
        first = first or ref  # the float32 table's results
        lo, hi = 3, 3 + max(1, q.shape[0] // 5)
        ef = np.random.default_rng(3).integers(1, w.ef + 1, hi - lo).astype(np.int32)
        ref2 = gix.search(lut[lo:hi], None if sc is None else sc[lo:hi], ef=ef, ef_max=w.ef, S=w.shortlist // 2)
        got2 = gix.search_noalloc(lut[lo:hi], None if sc is None else sc[lo:hi], ef=ef, ef_max=w.ef,
                                  S=w.shortlist // 2)
        torch.cuda.synchronize()
        _same(got2, ref2)
    return first


def test_noalloc_equals_the_workspace_walk(c1_build, torch):
    import paper_1804_09996_amd as lc
    w, ix, db, q = c1_build
    gix = lc.Index.from_index(ix)
    ref = _calls(gix, q, torch, w)
    o = ix.search(q, w.ef, w.shortlist, w.topk)
    assert np.array_equal(ref.cand_ids.cpu().numpy(), o["cand_ids"])
    gix.close()


def test_noalloc_with_fewer_slots_than_the_full_grid(c1_build, torch):
    # the 10k-node graph inside an index of 6M nodes (the rest unlinked): each slot's visited bitset is then
    # 750 KB, so the 128 MiB array holds ~170 slots where lc_search launches thousands; same results
    import paper_1804_09996_amd as lc
    w, ix, db, q = c1_build
    big_n = 6_000_000
    rs = np.random.default_rng(9)
    codes = np.concatenate([ix.codes, rs.integers(0, 256, (big_n - ix.n, ix.codes.shape[1])).astype(np.uint8)])
    adj0 = np.full((big_n, ix.deg0), -1, np.int32)
    adj0[:ix.n] = ix.adj0
    up_base = np.full(big_n, -1, np.int32)
    up_base[:ix.n] = ix.up_base
    bidx = np.zeros(big_n, np.uint8)
    bidx[:ix.n] = ix.beta_idx
    arrays = {"proj": ix.proj, "centroids": ix.centroids, "codes": codes, "adj0": adj0, "up_base": up_base,
              "adj_up": ix.adj_up, "beta": ix.beta, "beta_idx": bidx}
    meta = {k: int(getattr(ix, k)) for k in ("d", "d_pad", "m", "deg0", "deg_up", "k_reg", "entry", "max_level")}
    gix = lc.Index(arrays, meta)
    qq = np.ascontiguousarray(np.tile(q, (5, 1)))  # 500 queries: lc_search launches 500 slots or more
    per_slot = 4 * ((big_n + 31) // 32) + 4 * 4096
    full = (lc.lib().lc_search_workspace_bytes(gix.handle, qq.shape[0], w.ef, w.shortlist) - 256) // per_slot
    fit = ((128 << 20) - 256) // per_slot
    assert 1 <= fit < full, (fit, full)
    ref = _calls(gix, qq, torch, w)
    small = lc.Index.from_index(ix)
    lut, _ = small.build_lut(torch.from_numpy(qq))
    r = small.search(lut, ef=None, ef_max=w.ef, S=w.shortlist)
    _same(ref, r)
    gix.close()
    small.close()


def test_noalloc_rejects_an_index_too_large_for_one_slot(c1_build, torch):
    # n = 2^31 - 1: one slot's visited bitset alone is 256 MiB, beyond the array; LC_ENOSPC before any walk
    import paper_1804_09996_amd as lc
    w, ix, db, q = c1_build
    gix = lc.Index.from_index(ix)
    v = lc.IndexView.from_buffer_copy(gix.view)
    v.n = 2 ** 31 - 1
    h = C.c_void_p()
    assert lc.lib().lc_index_bind(C.byref(v), C.byref(h)) == lc.LC_OK
    lut, _ = gix.build_lut(torch.from_numpy(q[:4]))
    out = [torch.empty((4, w.shortlist), dtype=torch.int32, device="cuda"),
           torch.empty((4, w.shortlist), dtype=torch.float32, device="cuda"),
           torch.empty(4, dtype=torch.int32, device="cuda")]
    rc = lc.lib().lc_search_noalloc(h, lut.data_ptr(), lc.LC_LUT_F32, None, 4, None, w.ef, w.shortlist,
                                    out[0].data_ptr(), out[1].data_ptr(), out[2].data_ptr(), None,
                                    C.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert rc == lc.LC_ENOSPC
    lc.lib().lc_index_release(h)
    torch.cuda.synchronize()
    # the array is still usable afterwards
    ref = gix.search(lut, ef=None, ef_max=w.ef, S=w.shortlist)
    got = gix.search_noalloc(lut, ef=None, ef_max=w.ef, S=w.shortlist)
    torch.cuda.synchronize()
    _same(got, ref)
    gix.close()
