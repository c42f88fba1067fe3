"""The allocation-free sort (htex_sort_batch_noalloc, for callers that
cannot allocate device memory): through the C ABI, the same permutation and
sorted batch as htex_sort_batch bit for bit, on calls in a row whose batches
shrink (the scratch array keeps the previous call's contents), with one,
two and three radix passes."""
import ctypes as C

import numpy as np
import pytest
import torch

import paper_2207_05618_amd as htex
from paper_2207_05618_amd import _lib

pytestmark = pytest.mark.gpu


def _batch(H, Q, seed, with_f):
    rng = np.random.default_rng(seed)
    h = rng.integers(-3, H + 3, Q).astype(np.int32)
    u = rng.standard_normal(Q).astype(np.float32)
    v = rng.standard_normal(Q).astype(np.float32)
    f = rng.standard_normal(Q).astype(np.float32) if with_f else None
    T = lambda a: None if a is None else torch.from_numpy(a).cuda()
    return T(h), T(u), T(v), T(f)


def _noalloc(H, h, u, v, f):
    q, Q = htex._queries(h, u, v, f)
    perm = torch.full((Q,), -7, dtype=torch.int32, device="cuda")
    ho = torch.full_like(h, -7)
    uo, vo = torch.full_like(u, -7.0), torch.full_like(v, -7.0)
    fo = torch.full_like(f, -7.0) if f is not None else None
    st = _lib.load().htex_sort_batch_noalloc(
        int(H), C.byref(q), perm.data_ptr(), ho.data_ptr(), uo.data_ptr(), vo.data_ptr(),
        fo.data_ptr() if fo is not None else None, torch.cuda.current_stream().cuda_stream)
    _lib.check(st)
    return perm, ho, uo, vo, fo


def _same(a, b):
    for x, y in zip(a, b):
        if x is None or y is None:
            assert x is None and y is None
            continue
        xa, ya = x.cpu().numpy(), y.cpu().numpy()
        np.testing.assert_array_equal(xa.view(np.uint32), ya.view(np.uint32))


# shrinking batches: the largest the scratch takes (two passes), then
# smaller ones with three passes and one pass
CALLS = [(785950, 1 << 20, True), (1 << 24, 300001, False), (392, 4097, True), (392, 1, False)]


def test_noalloc_sort_matches_workspace_sort():
    for i, (H, Q, with_f) in enumerate(CALLS):
        print(f"noalloc sort call {i}: H={H} Q={Q} f={with_f}", flush=True)
        h, u, v, f = _batch(H, Q, 100 + i, with_f)
        got = _noalloc(H, h, u, v, f)
        ref = htex.htex_sort_batch(H, h, u, v, f)
        torch.cuda.synchronize()
        _same(got, ref)


def test_noalloc_sort_refuses_batches_above_its_limit():
    h, u, v, f = _batch(392, 16, 1, False)
    q = _lib.htex_queries(_lib.HTEX_SORT_NOALLOC_MAX_Q + 1, h.data_ptr(), u.data_ptr(),
                          v.data_ptr(), None)
    st = _lib.load().htex_sort_batch_noalloc(392, C.byref(q), 16, 16, 16, 16, None, None)
    assert st == -3
