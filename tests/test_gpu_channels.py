"""One-channel pools (a scalar map per edge, e.g. displacement) on the GPU
against the FP64 oracle's one-channel pools: sampling (plain with its
integer trace, prepared), BF16 / FP8 storage, the gradient, mips, corner
pre-processing and the device fill.  Same bars as the RGBA tests."""
import numpy as np
import pytest
import torch

import oracle
import paper_2207_05618_amd as htex
from htexgen import device as gdev
from htexgen import pool as gpool
from htexgen.mesh import cube_mesh
from htexgen.queries import tessellated_queries, uniform_queries
from tests.fixtures import tiny_meshes
from tests.gpu_helpers import Setup, assert_debug_equal, assert_rel, t

pytestmark = pytest.mark.gpu

TOL = 1e-5


def _stored(s, qp, dtype):
    if dtype == htex.HTEX_BF16:
        vals = oracle.bf16_to_f64(qp.texels.cpu().numpy().view(np.uint16))
    else:
        vals = oracle.e4m3_pool_to_f64(s.log2res, s.pool.base_host, s.has_mips,
                                       qp.texels.cpu().numpy(), qp.scale.cpu().numpy())
    return oracle.Pool(s.log2res, s.pool.base_host, vals, s.has_mips)


@pytest.mark.parametrize("mesh_i", [0, 1, 3])
@pytest.mark.parametrize("filt", [htex.HTEX_BILINEAR, htex.HTEX_TRILINEAR])
def test_one_channel_sampling_parity(mesh_i, filt):
    m = tiny_meshes()[mesh_i]
    tri = filt == htex.HTEX_TRILINEAR
    s = Setup(m, np.random.default_rng(60 + mesh_i).integers(0, 7, m.E), has_mips=tri, kind=1,
              seed=61, channels=1)
    q = uniform_queries(m.H, 30001, 62 + mesh_i, log2f=(-9, 1.5) if tri else None)
    q.h[:2] = [-3, m.H]
    got, dg = s.gpu(q, filt, debug=True)
    ref, errs, do = s.ref(q, oracle.TRILINEAR if tri else oracle.BILINEAR, debug=True)
    assert got.shape == (q.Q, 1) and errs == 2
    assert_debug_equal(dg, do)
    assert_rel(got, ref, TOL)
    prep = htex.Prepared(s.dmesh, s.pool)
    f = t(q.f) if q.f is not None else None
    for flags in (0, htex.HTEX_QUERIES_SCATTERED):
        o2 = htex.htex_sample_prepared(prep, s.pool, t(q.h), t(q.u), t(q.v), f, filter=filt,
                                       flags=flags)
        torch.cuda.synchronize()
        np.testing.assert_array_equal(o2.cpu().numpy(), got)


@pytest.mark.parametrize("dtype", [htex.HTEX_BF16, htex.HTEX_FP8_E4M3])
def test_one_channel_quantized(dtype):
    m = tiny_meshes()[1]
    s = Setup(m, np.random.default_rng(7).integers(0, 6, m.E), has_mips=True, kind=1, seed=8,
              channels=1)
    qp = htex.htex_quantize(s.pool, dtype)
    torch.cuda.synchronize()
    src = s.pool.texels.cpu().numpy()
    if dtype == htex.HTEX_BF16:
        np.testing.assert_array_equal(qp.texels.cpu().numpy().view(np.uint16).reshape(-1),
                                      oracle.f32_to_bf16(src))
    else:
        codes, scale = oracle.quantize_e4m3(s.log2res, s.pool.base_host, True, src)
        np.testing.assert_array_equal(qp.scale.cpu().numpy(), scale)
        np.testing.assert_array_equal(qp.texels.cpu().numpy(), codes)
    q = uniform_queries(m.H, 20000, 9, log2f=(-8, 1))
    got, dg = s.gpu(q, htex.HTEX_TRILINEAR, debug=True, pool=qp)
    ref, _, do = s.ref(q, oracle.TRILINEAR, debug=True, opool=_stored(s, qp, dtype))
    assert_debug_equal(dg, do)
    assert_rel(got, ref, TOL)
    ref32, _, _ = s.ref(q, oracle.TRILINEAR)
    assert_rel(got, ref32, 4e-3 if dtype == htex.HTEX_BF16 else 6e-2)
    # the prepared kernels (all taps, in-bounds taps) give the same bits
    prep = htex.Prepared(s.dmesh, qp)
    for flags in (0, htex.HTEX_QUERIES_SCATTERED):
        o2 = htex.htex_sample_prepared(prep, qp, t(q.h), t(q.u), t(q.v), t(q.f),
                                       filter=htex.HTEX_TRILINEAR, flags=flags)
        torch.cuda.synchronize()
        np.testing.assert_array_equal(o2.cpu().numpy(), got)


@pytest.mark.parametrize("flags", [0, htex.HTEX_QUERIES_SORTED])
@pytest.mark.parametrize("filt", [htex.HTEX_BILINEAR, htex.HTEX_TRILINEAR])
def test_one_channel_backward(filt, flags):
    """Both scatter paths; levels of up to 64 x 64 one-channel texels fit the
    on-chip cache, larger ones go to global atomics."""
    m = cube_mesh()
    tri = filt == htex.HTEX_TRILINEAR
    s = Setup(m, np.random.default_rng(5).integers(3, 8, m.E), has_mips=tri, kind=1, channels=1)
    q = uniform_queries(m.H, 200000, 405, log2f=(-8, 0) if tri else None, sort=True)
    q.h[:2] = [-1, m.H]
    g = np.random.default_rng(406).standard_normal((q.Q, 1)).astype(np.float32)
    f = t(q.f) if q.f is not None else None
    d = htex.htex_sample_backward(s.dmesh, s.pool, t(q.h), t(q.u), t(q.v), t(g), f, filter=filt,
                                  flags=flags)
    torch.cuda.synchronize()
    ref, dabs = oracle.backward(s.omesh, s.opool, q.h, q.u, q.v, g.astype(np.float64), q.f,
                                filter=oracle.TRILINEAR if tri else oracle.BILINEAR,
                                with_abs=True)
    got = d.cpu().numpy()
    assert got.shape == ref.shape
    assert (np.abs(got - ref) <= 1e-4 * dabs + 1e-7).all()


def test_one_channel_mips_and_corners():
    m = tiny_meshes()[3]
    s = Setup(m, np.random.default_rng(2).integers(1, 7, m.E), has_mips=True, kind=0, seed=4,
              channels=1)
    got = s.pool.texels.cpu().numpy()
    assert_rel(got, s.opool.texels, 1e-6)   # box means of float32 values
    err = torch.zeros(1, dtype=torch.int32, device="cuda")
    htex.htex_corner_average(s.dmesh, s.pool, err_count=err)
    torch.cuda.synchronize()
    assert int(err.item()) == 0
    op = oracle.Pool(s.log2res, s.opool.base, got.astype(np.float64), True)
    ref = oracle.corner_average(s.omesh, op, m.vert, m.face, m.V, m.F)
    after = s.pool.texels.cpu().numpy()
    changed = ref != got
    np.testing.assert_array_equal(after[~changed], got[~changed])
    assert_rel(after, ref, 2.0 ** -24 * 1.01, floor=1e-30)


def test_one_channel_device_fill_matches_host_generator():
    m = cube_mesh()
    lr = np.random.default_rng(1).integers(0, 6, m.E).astype(np.uint8)
    base, total = gpool.layout(lr, True)
    host = gpool.fill_level0_host(1, 77, lr, base, total, m.boundary_edges(), True, channels=1)
    dev = torch.zeros((total, 1), dtype=torch.float32, device="cuda")
    gdev.fill_level0(dev, 1, 77, t(lr), t(base), m.boundary_edges())
    np.testing.assert_array_equal(dev.cpu().numpy(), host)


def test_displacement_on_tessellated_grid():
    """The vertex-stage workload: a one-channel displacement pool with
    processed corners, sampled on every patch of a tessellated grid,
    matches the oracle and has no cracks between patches."""
    from scipy.spatial import cKDTree
    m = cube_mesh()
    s = Setup(m, np.full(m.E, 4), has_mips=True, kind=1, seed=12, channels=1)
    htex.htex_corner_average(s.dmesh, s.pool)
    T = 4
    q = tessellated_queries(m.H, T, footprint=1.0 / T)
    got, _ = s.gpu(q, htex.HTEX_TRILINEAR)
    op = oracle.Pool(s.log2res, s.opool.base,
                     oracle.corner_average(s.omesh, s.opool, m.vert, m.face, m.V, m.F), True)
    ref, _, _ = s.ref(q, oracle.TRILINEAR, opool=op)
    assert_rel(got, ref, TOL)
    pos = np.asarray(m.positions)
    cen = np.zeros((m.F, 3))
    np.add.at(cen, m.face, pos[m.vert])
    cen /= np.bincount(m.face)[:, None]
    w = 1.0 - q.u.astype(np.float64) - q.v
    pts = (q.u[:, None] * pos[m.vert[q.h]] + q.v[:, None] * pos[m.vert[m.next[q.h]]]
           + w[:, None] * cen[m.face[q.h]])
    pairs = np.array(sorted(cKDTree(pts).query_pairs(1e-9)))
    assert np.abs(got[pairs[:, 0]] - got[pairs[:, 1]]).max() < 4e-7
