"""Ordering a batch by halfedge: perm equals the stable argsort of the keys
(h, invalid h last) bit for bit, the sorted batch equals the input gathered
through perm bit for bit, and every way back to input order (un-permute,
or sampling that writes through perm) gives the same bits as sampling the
batch as it came."""
import ctypes as C

import numpy as np
import pytest
import torch

import paper_2207_05618_amd as htex
from paper_2207_05618_amd import _lib
from htexgen.mesh import cube_mesh
from htexgen.queries import uniform_queries
from tests.gpu_helpers import Setup, t

pytestmark = pytest.mark.gpu


def _ref_perm(h, H):
    key = np.where((h >= 0) & (h < H), h, H).astype(np.int64)
    return np.argsort(key, kind="stable").astype(np.int32)


# H = 1 and 392 sort in one digit pass, 70000 and 785950 in two, 2^24 in three
CASES = [(392, 0), (392, 1), (392, 4095), (392, 4097), (1, 5000), (300, 123457),
         (785950, 1 << 20), (1 << 24, 300001), (70000, 8193), (2047, 20000), (2048, 20000)]


@pytest.mark.parametrize("H,Q", CASES)
def test_sort_matches_stable_argsort(H, Q):
    rng = np.random.default_rng(H + Q)
    h = rng.integers(-3, H + 3, Q).astype(np.int32) if Q else np.zeros(0, np.int32)
    print(f"sort_queries H={H} Q={Q}", flush=True)
    perm = htex.htex_sort_queries(H, t(h))
    torch.cuda.synchronize()
    np.testing.assert_array_equal(perm.cpu().numpy(), _ref_perm(h, H))


@pytest.mark.parametrize("H,Q", CASES)
@pytest.mark.parametrize("with_f", [True, False])
def test_sort_batch_carries_the_queries(H, Q, with_f):
    rng = np.random.default_rng(7 * H + Q)
    h = rng.integers(-3, H + 3, Q).astype(np.int32) if Q else np.zeros(0, np.int32)
    u = rng.standard_normal(Q).astype(np.float32)
    v = rng.standard_normal(Q).astype(np.float32)
    f = rng.standard_normal(Q).astype(np.float32) if with_f else None
    print(f"sort_batch H={H} Q={Q} f={with_f}", flush=True)
    perm, ho, uo, vo, fo = htex.htex_sort_batch(H, t(h), t(u), t(v), t(f) if with_f else None)
    torch.cuda.synchronize()
    ref = _ref_perm(h, H)
    np.testing.assert_array_equal(perm.cpu().numpy(), ref)
    np.testing.assert_array_equal(ho.cpu().numpy(), h[ref])
    # payloads are moved, never converted: compare the bits
    np.testing.assert_array_equal(uo.cpu().numpy().view(np.uint32), u[ref].view(np.uint32))
    np.testing.assert_array_equal(vo.cpu().numpy().view(np.uint32), v[ref].view(np.uint32))
    if with_f:
        np.testing.assert_array_equal(fo.cpu().numpy().view(np.uint32), f[ref].view(np.uint32))
    else:
        assert fo is None


def _ref_perm_by_key(h, H, key, K):
    hv = np.where((h >= 0) & (h < H), h, 0)
    k = np.where((h >= 0) & (h < H), key[hv].astype(np.int64), K)
    k = np.where((k >= 0) & (k < K), k, K)
    return np.argsort(k, kind="stable").astype(np.int32)


@pytest.mark.parametrize("H,K,Q", [(392, 196, 20000), (392, 1, 5000), (785950, 396966, 300001),
                                   (70000, 300, 8193), (2048, 5000, 4097)])
def test_sort_batch_by_key(H, K, Q):
    """Keyed order: perm equals the stable argsort of key[h] (invalid h and
    keys outside [0, K) last), and the sorted arrays are the input gathered
    through perm, bit for bit."""
    rng = np.random.default_rng(3 * H + K + Q)
    h = rng.integers(-3, H + 3, Q).astype(np.int32)
    key = rng.integers(0, K, H).astype(np.int32)
    key[::97] = K + 5          # out-of-range keys sort with the invalid queries
    key[1::101] = -2
    u = rng.standard_normal(Q).astype(np.float32)
    v = rng.standard_normal(Q).astype(np.float32)
    f = rng.standard_normal(Q).astype(np.float32)
    print(f"sort_batch_by_key H={H} K={K} Q={Q}", flush=True)
    perm, ho, uo, vo, fo = htex.htex_sort_batch(H, t(h), t(u), t(v), t(f), key=t(key), nkeys=K)
    torch.cuda.synchronize()
    ref = _ref_perm_by_key(h, H, key, K)
    np.testing.assert_array_equal(perm.cpu().numpy(), ref)
    np.testing.assert_array_equal(ho.cpu().numpy(), h[ref])
    for a, b in ((uo, u), (vo, v), (fo, f)):
        np.testing.assert_array_equal(a.cpu().numpy().view(np.uint32), b[ref].view(np.uint32))


def test_sample_in_edge_order_matches_direct():
    """A batch ordered by the edge of its halfedge, sampled with the sorted
    kernel and put back in input order, gives the direct path's bits."""
    m = cube_mesh()
    s = Setup(m, np.full(m.E, 5), has_mips=True, kind=1)
    q = uniform_queries(m.H, 100000, 19, log2f=(-7, 0), shuffle_seed=4)
    direct, _ = s.gpu(q, htex.HTEX_TRILINEAR)
    prep = htex.Prepared(s.dmesh, s.pool)
    perm, h2, u2, v2, f2 = htex.htex_sort_batch(m.H, t(q.h), t(q.u), t(q.v), t(q.f),
                                                key=s.dmesh.edge, nkeys=m.E)
    e = m.edge[h2.cpu().numpy()]
    assert (e[1:] >= e[:-1]).all()
    o = htex.htex_sample_prepared(prep, s.pool, h2, u2, v2, f2, filter=htex.HTEX_TRILINEAR,
                                  flags=htex.HTEX_QUERIES_SORTED)
    back = htex.htex_unpermute_results(perm, o)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(back.cpu().numpy(), direct)


@pytest.mark.parametrize("Q", [0, 1, 4097, 100003])
@pytest.mark.parametrize("dtype,channels,tri", [(htex.HTEX_F32, 4, True),
                                                (htex.HTEX_F32, 1, False),
                                                (htex.HTEX_BF16, 4, True),
                                                (htex.HTEX_FP8_E4M3, 1, True)])
def test_sample_reordered_matches_direct(Q, dtype, channels, tri):
    """One call that sorts a shuffled batch, samples it in halfedge order
    through the permutation and writes the rows in the batch's own order
    gives htex_sample_prepared's bits, invalid queries (NaN rows, counted)
    included, for the lane and the wavefront kernels."""
    m = cube_mesh()
    s = Setup(m, np.full(m.E, 4), has_mips=tri, kind=1, channels=channels)
    pool = s.pool if dtype == htex.HTEX_F32 else htex.htex_quantize(s.pool, dtype)
    q = uniform_queries(m.H, Q, 41 + Q, log2f=(-6, 0), shuffle_seed=6) if Q else None
    h = q.h.copy() if Q else np.zeros(0, np.int32)
    if Q > 10:
        h[::997] = -1
        h[5::1009] = m.H + 2
    u = q.u if Q else np.zeros(0, np.float32)
    v = q.v if Q else np.zeros(0, np.float32)
    f = q.f if Q else np.zeros(0, np.float32)
    filt = htex.HTEX_TRILINEAR if tri else htex.HTEX_BILINEAR
    prep = htex.Prepared(s.dmesh, pool)
    e0 = torch.zeros(1, dtype=torch.int32, device="cuda")
    e1 = torch.zeros(1, dtype=torch.int32, device="cuda")
    print(f"reordered Q={Q} dtype={dtype} C={channels} tri={tri}", flush=True)
    ft = t(f) if tri else None
    direct = htex.htex_sample_prepared(prep, pool, t(h), t(u), t(v), ft, filter=filt,
                                       err_count=e0)
    got = htex.htex_sample_prepared_reordered(prep, pool, t(h), t(u), t(v), ft, filter=filt,
                                              err_count=e1)
    torch.cuda.synchronize()
    d, g = direct.cpu().numpy(), got.cpu().numpy()
    assert g.shape == d.shape
    np.testing.assert_array_equal(g.view(np.uint32), d.view(np.uint32))
    assert int(e1.item()) == int(e0.item())
    if Q > 10:
        assert int(e0.item()) > 0


def test_sorted_input_is_identity_and_sampling_order_free():
    m = cube_mesh()
    s = Setup(m, np.full(m.E, 5), has_mips=True, kind=1)
    q = uniform_queries(m.H, 200000, 9, log2f=(-7, 0), shuffle_seed=3)
    direct, _ = s.gpu(q, htex.HTEX_TRILINEAR)
    perm = htex.htex_sort_queries(m.H, t(q.h))
    h2, u2, v2, f2 = htex.htex_permute_queries(perm, t(q.h), t(q.u), t(q.v), t(q.f))
    assert bool((h2[1:] >= h2[:-1]).all())
    prep = htex.Prepared(s.dmesh, s.pool)
    o_sorted = htex.htex_sample_prepared(prep, s.pool, h2, u2, v2, f2, filter=htex.HTEX_TRILINEAR,
                                         flags=htex.HTEX_QUERIES_SORTED)
    back = htex.htex_unpermute_results(perm, o_sorted)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(back.cpu().numpy(), direct)
    # the one-call sort gives the same sorted batch as sort + gather
    p3, h3, u3, v3, f3 = htex.htex_sort_batch(m.H, t(q.h), t(q.u), t(q.v), t(q.f))
    torch.cuda.synchronize()
    np.testing.assert_array_equal(p3.cpu().numpy(), perm.cpu().numpy())
    for a, b in ((h3, h2), (u3, u2), (v3, v2), (f3, f2)):
        np.testing.assert_array_equal(a.cpu().numpy(), b.cpu().numpy())
    # sampling the one-call sorted batch and un-permuting
    o3 = htex.htex_sample_prepared(prep, s.pool, h3, u3, v3, f3, filter=htex.HTEX_TRILINEAR,
                                   flags=htex.HTEX_QUERIES_SORTED)
    back2 = htex.htex_unpermute_results(p3, o3)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(back2.cpu().numpy(), direct)
    # an already sorted batch gets the identity
    p2 = htex.htex_sort_queries(m.H, h2)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(p2.cpu().numpy(), np.arange(q.Q, dtype=np.int32))


@pytest.mark.parametrize("dtype", [htex.HTEX_F32, htex.HTEX_BF16])
def test_sort_path_with_invalid_queries_and_one_channel(dtype):
    """Invalid queries sort last and come back to their own rows as NaN;
    one-channel results go back to input order."""
    m = cube_mesh()
    s = Setup(m, np.full(m.E, 4), has_mips=False, kind=0, channels=1)
    pool = s.pool if dtype == htex.HTEX_F32 else htex.htex_quantize(s.pool, dtype)
    q = uniform_queries(m.H, 50001, 31, shuffle_seed=5)
    h = q.h.copy()
    h[::997] = -1
    h[5::1009] = m.H + 2
    prep = htex.Prepared(s.dmesh, pool)
    err0 = torch.zeros(1, dtype=torch.int32, device="cuda")
    direct = htex.htex_sample_prepared(prep, pool, t(h), t(q.u), t(q.v), err_count=err0)
    perm, hs, us, vs, _ = htex.htex_sort_batch(m.H, t(h), t(q.u), t(q.v))
    err1 = torch.zeros(1, dtype=torch.int32, device="cuda")
    o_sorted = htex.htex_sample_prepared(prep, pool, hs, us, vs, err_count=err1)
    o2 = htex.htex_unpermute_results(perm, o_sorted)
    torch.cuda.synchronize()
    d = direct.cpu().numpy()
    assert d.shape == (q.Q, 1)
    assert np.isnan(d[::997]).all() and np.isnan(d[5::1009]).all()
    np.testing.assert_array_equal(o2.cpu().numpy(), d)
    assert int(err1.item()) == int(err0.item()) > 0
    # the invalid queries are the tail of the sorted batch
    nbad = int(((h < 0) | (h >= m.H)).sum())
    hs_ = hs.cpu().numpy()
    assert ((hs_[-nbad:] < 0) | (hs_[-nbad:] >= m.H)).all()
    assert ((hs_[:-nbad] >= 0) & (hs_[:-nbad] < m.H)).all()


def test_records_of_another_layout_cannot_read_outside_the_pool():
    """Records prepared for a larger pool, handed to the C ABI with a
    smaller one (the Python layer refuses this; the library must not read
    past the pool either): every query whose record does not fit is
    answered NaN and counted; records that fit sample normally."""
    m = cube_mesh()
    big = Setup(m, np.full(m.E, 5), has_mips=True, kind=0)
    small = Setup(m, np.full(m.E, 3), has_mips=True, kind=0)
    prep_big = htex.Prepared(big.dmesh, big.pool)
    q = uniform_queries(m.H, 20000, 3, log2f=(-6, 0))
    with pytest.raises(ValueError, match="another pool layout"):
        htex.htex_sample_prepared(prep_big, small.pool, t(q.h), t(q.u), t(q.v), t(q.f),
                                  filter=htex.HTEX_TRILINEAR)
    qt = (t(q.h), t(q.u), t(q.v), t(q.f))   # kept alive: qq holds their addresses
    qq, Q = htex._queries(*qt)
    out = torch.zeros((Q, 4), dtype=torch.float32, device="cuda")
    err = torch.zeros(1, dtype=torch.int32, device="cuda")
    L = _lib.load()
    st = L.htex_sample_prepared(m.H, prep_big.buf.data_ptr(), C.byref(small.pool.c), C.byref(qq),
                                htex.HTEX_TRILINEAR, 0, out.data_ptr(), err.data_ptr(),
                                torch.cuda.current_stream().cuda_stream)
    assert st == 0
    torch.cuda.synchronize()
    o = out.cpu().numpy()
    # a record fits when all three fetched edges end inside the small pool
    ext = ((4 << 10) - 1) // 3
    base = big.pool.base_host
    e = np.stack([m.edge[q.h], m.edge[m.next[q.h]], m.edge[m.prev[q.h]]], 1)
    fits = (base[e] + ext <= small.pool.total).all(1)
    assert fits.any() and (~fits).any()
    assert np.isnan(o[~fits]).all()
    assert np.isfinite(o[fits]).all()
    assert int(err.item()) == int((~fits).sum())


def test_wrappers_refuse_wrong_shapes():
    m = cube_mesh()
    s = Setup(m, np.full(m.E, 4), has_mips=False, kind=0)
    q = uniform_queries(m.H, 1000, 3)
    h, u, v = t(q.h), t(q.u), t(q.v)
    with pytest.raises(ValueError):
        htex.htex_sample(s.dmesh, s.pool, h, u, v, out=torch.empty((999, 4), device="cuda"))
    prep = htex.Prepared(s.dmesh, s.pool)
    with pytest.raises(ValueError):
        htex.htex_sample_prepared(prep, s.pool, h, u, v, out=torch.empty((1000, 1),
                                                                          device="cuda"))
    with pytest.raises(ValueError):
        htex.htex_sample_backward(s.dmesh, s.pool, h, u, v, torch.zeros((1000, 1), device="cuda"))
    with pytest.raises(ValueError):
        htex.htex_sample_backward(s.dmesh, s.pool, h, u, v, torch.zeros((1000, 4), device="cuda"),
                                  dtexels=torch.zeros((s.pool.total - 1, 4), device="cuda"))
    with pytest.raises(ValueError):
        htex.htex_unpermute_results(t(np.arange(1000, dtype=np.int32)),
                                    torch.zeros((1000, 2), device="cuda"))
