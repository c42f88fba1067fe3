"""Parity at the benchmark's full size, in the launch the benchmark times:
the ~194k-face sphere with 64x64 RGBA float32 textures and mips (34.8 GB),
8,294,400 sorted queries, trilinear.  The oracle cannot take the whole frame,
so it checks sampled outputs -- a contiguous slice of the sorted batch and
queries drawn across it -- with its texels from the host generator and its
own FP64 mips; properties that hold at any size (batch independence,
quantization error bounds) cover the rest.
"""
import numpy as np
import pytest
import torch

import oracle
import paper_2207_05618_amd as htex
from htexgen import device as gdev
from htexgen import pool as gpool
from htexgen.mesh import sphere_mesh
from htexgen.queries import uniform_queries
from htexgen.texels import PERLIN
from tests.gpu_helpers import assert_debug_equal, assert_rel, t

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def frame():
    mesh = sphere_mesh(n=183, seed=201)
    lr = np.full(mesh.E, 6, np.uint8)
    pool = htex.Pool(lr, True, htex.HTEX_F32)
    gdev.fill_level0(pool.texels, PERLIN, 202, pool.log2res, pool.base, mesh.boundary_edges())
    htex.htex_build_mips(pool)
    q = uniform_queries(mesh.H, 3840 * 2160, 203, log2f=(-3.2, -1.2), sort=True)
    dm = htex.Mesh.of(mesh)
    out, _ = htex.htex_sample(dm, pool, t(q.h), t(q.u), t(q.v), t(q.f),
                              filter=htex.HTEX_TRILINEAR, flags=htex.HTEX_QUERIES_SORTED)
    torch.cuda.synchronize()
    yield mesh, lr, pool, dm, q, out.cpu().numpy()
    del pool
    torch.cuda.empty_cache()


def _oracle_for(mesh, lr, qs):
    """Oracle mesh + pool restricted to the edges the queries touch (texels
    from the host generator, mips by the oracle)."""
    hs = np.unique(np.concatenate([qs.h, mesh.next[qs.h], mesh.prev[qs.h]]))
    edges = np.unique(mesh.edge[hs])
    remap = np.full(mesh.E, -1, np.int32)
    remap[edges] = np.arange(len(edges), dtype=np.int32)
    sub = lr[edges]
    base, total = gpool.layout(sub, True)
    lvl0 = np.zeros((total, 4), np.float32)
    bnd = mesh.boundary_edges()[edges]
    # fill edge by edge group (host generator keyed by the ORIGINAL edge id)
    from htexgen.texels import texel_values
    n = 1 << int(sub[0])
    jj, ii = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    for chunk in np.array_split(np.arange(len(edges)), max(1, len(edges) // 256)):
        vals = texel_values(PERLIN, 202, edges[chunk][:, None, None], n, bnd[chunk][:, None, None],
                            ii.reshape(-1)[None, :, None], jj.reshape(-1)[None, :, None],
                            np.arange(4)[None, None, :])
        rows = base[chunk][:, None] + np.arange(n * n)[None, :]
        lvl0[rows.reshape(-1)] = vals.reshape(-1, 4)
    op = oracle.Pool(sub, base, lvl0.astype(np.float64), True)
    op = oracle.Pool(sub, base, oracle.build_mips(op), True)
    om = oracle.Mesh(mesh.twin, mesh.next, mesh.prev, remap[mesh.edge], len(edges))
    return om, op, remap


def _samples(q):
    rng = np.random.default_rng(7)
    lo = q.Q // 3
    idx = np.concatenate([np.arange(lo, lo + 3000), rng.choice(q.Q, 400, replace=False)])
    return np.unique(idx)


def test_frame_sampled_parity(frame):
    mesh, lr, pool, dm, q, out = frame
    idx = _samples(q)
    qs = q.take(idx)
    om, op, remap = _oracle_for(mesh, lr, qs)
    ref, errs, do = oracle.sample(om, op, qs.h, qs.u, qs.v, qs.f, filter=oracle.TRILINEAR,
                                  debug=True)
    assert errs == 0
    assert_rel(out[idx], ref, 1e-5)
    # integer trace of the same queries (debug launch), edges mapped back
    _, dbg = htex.htex_sample(dm, pool, t(qs.h), t(qs.u), t(qs.v), t(qs.f),
                              filter=htex.HTEX_TRILINEAR, debug=True)
    dg = htex.debug_records(dbg).copy()
    dg["edge"] = remap[dg["edge"]]
    assert_debug_equal(dg, do)


def test_frame_unsorted_equals_sorted(frame):
    """Results do not depend on the batch or on the order: the shuffled frame
    gives the same bits per query."""
    mesh, lr, pool, dm, q, out = frame
    perm = np.random.default_rng(204).permutation(q.Q)
    qu = q.take(perm)
    o2, _ = htex.htex_sample(dm, pool, t(qu.h), t(qu.u), t(qu.v), t(qu.f),
                             filter=htex.HTEX_TRILINEAR)
    np.testing.assert_array_equal(o2.cpu().numpy(), out[perm])


def test_frame_prepared_equals_plain(frame):
    """The prepared fast path (what the benchmark times) gives the plain
    path's bits on the whole frame, with either kernel the hints select."""
    mesh, lr, pool, dm, q, out = frame
    prep = htex.Prepared(dm, pool)
    o2 = htex.htex_sample_prepared(prep, pool, t(q.h), t(q.u), t(q.v), t(q.f),
                                   filter=htex.HTEX_TRILINEAR, flags=htex.HTEX_QUERIES_SORTED)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(o2.cpu().numpy(), out)
    # the kernel for scattered batches (in-bounds taps only), on the
    # shuffled frame
    perm = np.random.default_rng(205).permutation(q.Q)
    qu = q.take(perm)
    o3 = htex.htex_sample_prepared(prep, pool, t(qu.h), t(qu.u), t(qu.v), t(qu.f),
                                   filter=htex.HTEX_TRILINEAR,
                                   flags=htex.HTEX_QUERIES_SCATTERED)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(o3.cpu().numpy(), out[perm])
    # the sort path the benchmark times on the shuffled frame: sort the batch
    # in one call, sample it sorted, results back to the shuffled order
    hu, uu, vu, fu = t(qu.h), t(qu.u), t(qu.v), t(qu.f)
    del o2, o3
    p4, h4, u4, v4, f4 = htex.htex_sort_batch(mesh.H, hu, uu, vu, fu)
    o4s = htex.htex_sample_prepared(prep, pool, h4, u4, v4, f4, filter=htex.HTEX_TRILINEAR,
                                    flags=htex.HTEX_QUERIES_SORTED)
    o4 = htex.htex_unpermute_results(p4, o4s)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(p4.cpu().numpy(), np.argsort(qu.h, kind="stable"))
    np.testing.assert_array_equal(o4.cpu().numpy(), out[perm])
    del p4, h4, u4, v4, f4, o4s, o4
    # the same in one call: sorted, sampled through the permutation, and
    # written back in the shuffled order
    o5 = htex.htex_sample_prepared_reordered(prep, pool, hu, uu, vu, fu,
                                             filter=htex.HTEX_TRILINEAR)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(o5.cpu().numpy(), out[perm])


def test_frame_quantized_error_bounds(frame):
    """BF16 and FP8 storage of the full pool: sampled error against the
    oracle on the float32 texels within 4e-3 and 6e-2 relative."""
    mesh, lr, pool, dm, q, out = frame
    idx = _samples(q)[:1500]
    qs = q.take(idx)
    om, op, _ = _oracle_for(mesh, lr, qs)
    ref, _, _ = oracle.sample(om, op, qs.h, qs.u, qs.v, qs.f, filter=oracle.TRILINEAR)
    for dtype, tol in ((htex.HTEX_BF16, 4e-3), (htex.HTEX_FP8_E4M3, 6e-2)):
        qp = htex.htex_quantize(pool, dtype)
        g, _ = htex.htex_sample(dm, qp, t(qs.h), t(qs.u), t(qs.v), t(qs.f),
                                filter=htex.HTEX_TRILINEAR)
        gn = g.cpu().numpy()
        worst = assert_rel(gn, ref, tol)
        rel = np.abs(gn.astype(np.float64) - ref) / np.maximum(np.abs(ref), 1e-6)
        print(f"frame {'bf16' if dtype == htex.HTEX_BF16 else 'fp8_e4m3'}: relative error "
              f"max {worst:.3e} mean {float(np.nanmean(rel)):.3e} over {qs.Q} queries x 4",
              flush=True)
        del qp
        torch.cuda.empty_cache()


# ------------------------------------------------ vertex-stage displacement --

@pytest.fixture(scope="module")
def disp_frame(frame):
    """The displacement map of the frame mesh as the benchmark builds it:
    one 64x64 float32 channel per edge, level 0 only, corners pre-processed,
    sampled at the vertices of every patch tessellated with T = 4."""
    mesh, lr, pool, dm, q, out = frame
    from htexgen.queries import tessellated_queries
    disp = htex.Pool(lr, False, htex.HTEX_F32, channels=1)
    gdev.fill_level0(disp.texels, 1, 501, disp.log2res, disp.base, mesh.boundary_edges())
    torch.cuda.synchronize()
    before = disp.texels.cpu().numpy()
    err = torch.zeros(1, dtype=torch.int32, device="cuda")
    htex.htex_corner_average(dm, disp, err_count=err)
    prep = htex.Prepared(dm, disp)
    tq = tessellated_queries(mesh.H, 4)
    o = htex.htex_sample_prepared(prep, disp, t(tq.h), t(tq.u), t(tq.v), None,
                                  filter=htex.HTEX_BILINEAR, flags=htex.HTEX_QUERIES_SORTED)
    torch.cuda.synchronize()
    yield mesh, disp, before, disp.texels.cpu().numpy(), int(err.item()), tq, o.cpu().numpy()
    del disp, prep
    torch.cuda.empty_cache()


def test_frame_corner_groups_hold_their_means(disp_frame):
    """Sampled vertices and faces of the full mesh: their corner texels all
    equal the float64 mean of the values before, rounded once."""
    mesh, disp, before, after, err, _, _ = disp_frame
    assert err == 0
    base = disp.base_host
    n = 64
    rng = np.random.default_rng(11)
    gi = np.nonzero(mesh.twin < np.arange(mesh.H))[0]          # larger halfedge of each edge
    gi = np.concatenate([gi, np.nonzero(mesh.twin < 0)[0]])
    gi = np.unique(gi)
    e = mesh.edge[gi]
    t = mesh.twin[gi]
    rows = np.concatenate([base[e] + n - 1, base[e] + (n - 1) * n, base[e],
                           np.where(t >= 0, base[e] + n * n - 1, -1)])
    keys = np.concatenate([mesh.vert[gi], mesh.vert[mesh.next[gi]], mesh.V + mesh.face[gi],
                           np.where(t >= 0, mesh.V + mesh.face[np.maximum(t, 0)], -1)])
    ok = rows >= 0
    rows, keys = rows[ok], keys[ok]
    pick = rng.choice(np.unique(keys), 3000, replace=False)
    sel = np.isin(keys, pick)
    rows, keys = rows[sel], keys[sel]
    order = np.argsort(keys, kind="stable")
    rows, keys = rows[order], keys[order]
    starts = np.r_[0, np.nonzero(np.diff(keys))[0] + 1, len(keys)]
    for a, b in zip(starts[:-1], starts[1:]):
        r = rows[a:b]
        want = np.float32(before[r, 0].astype(np.float64).mean())
        assert (after[r, 0] == want).all(), (keys[a], after[r, 0], want)


def test_frame_displacement_sampled_parity_and_crack_free(disp_frame):
    """Patches of a run of faces: GPU values against the oracle on the
    processed texels of the touched edges, and equal displacement wherever
    two of those patches share a surface point."""
    from scipy.spatial import cKDTree
    mesh, disp, _, after, _, tq, o = disp_frame
    f0 = mesh.F // 2
    hs = np.nonzero((mesh.face >= f0) & (mesh.face < f0 + 300))[0]
    hs = np.unique(np.concatenate([hs, mesh.twin[hs][mesh.twin[hs] >= 0]]))
    idx = np.nonzero(np.isin(tq.h, hs))[0]
    qs = tq.take(idx)
    touched = np.unique(np.concatenate([qs.h, mesh.next[qs.h], mesh.prev[qs.h]]))
    edges = np.unique(mesh.edge[touched])
    remap = np.full(mesh.E, -1, np.int32)
    remap[edges] = np.arange(len(edges), dtype=np.int32)
    sub = np.full(len(edges), 6, np.uint8)
    base, total = gpool.layout(sub, False)
    T = np.zeros((total, 1), np.float64)
    for i, e in enumerate(edges):
        T[base[i]:base[i] + 4096] = after[disp.base_host[e]:disp.base_host[e] + 4096]
    op = oracle.Pool(sub, base, T, False)
    om = oracle.Mesh(mesh.twin, mesh.next, mesh.prev, remap[mesh.edge], len(edges))
    ref, errs, _ = oracle.sample(om, op, qs.h, qs.u, qs.v)
    assert errs == 0
    assert_rel(o[idx], ref, 1e-5)
    pos = np.asarray(mesh.positions)
    cen = np.zeros((mesh.F, 3))
    np.add.at(cen, mesh.face, pos[mesh.vert])
    cen /= np.bincount(mesh.face, minlength=mesh.F)[:, None]
    w = 1.0 - qs.u.astype(np.float64) - qs.v
    pts = (qs.u[:, None] * pos[mesh.vert[qs.h]] + qs.v[:, None] * pos[mesh.vert[mesh.next[qs.h]]]
           + w[:, None] * cen[mesh.face[qs.h]])
    pairs = np.array(sorted(cKDTree(pts).query_pairs(1e-9)))
    assert len(pairs) > len(hs)
    got = o[idx]
    assert np.abs(got[pairs[:, 0]] - got[pairs[:, 1]]).max() < 4e-7


# ------------------------------------------------------ rasterized 4K frame --

def test_frame_rasterized_view_sampled_parity(frame):
    """The benchmark's rasterized view of the frame mesh (3840 x 2160, the
    oracle's intrinsic triangles): the whole frame sampled on the GPU in
    scanline order (trilinear at each pixel's footprint, and anisotropic
    with its derivatives); a contiguous run of pixels and scattered pixels
    checked against the oracle."""
    from htexgen.raster import rasterize, sphere_view
    mesh, lr, pool, dm, q, out = frame
    om = oracle.Mesh.of(mesh)
    T, bad = oracle.triangle_vertices(om, mesh.vert, mesh.positions)
    assert bad == 0
    fr = rasterize(T, sphere_view())
    f = fr.footprint()
    prep = htex.Prepared(dm, pool)
    o_tri = htex.htex_sample_prepared(prep, pool, t(fr.h), t(fr.u), t(fr.v), t(f),
                                      filter=htex.HTEX_TRILINEAR)
    o_an = htex.htex_sample_aniso_prepared(prep, pool, t(fr.h), t(fr.u), t(fr.v), t(fr.jac))
    torch.cuda.synchronize()
    rng = np.random.default_rng(12)
    lo = fr.Q // 2
    idx = np.unique(np.concatenate([np.arange(lo, lo + 2500), rng.choice(fr.Q, 500, replace=False)]))
    from htexgen.queries import Queries
    qs = Queries(fr.h[idx], fr.u[idx], fr.v[idx], f[idx])
    sub_m, sub_p, remap = _oracle_for(mesh, lr, qs)
    ref, errs, _ = oracle.sample(sub_m, sub_p, qs.h, qs.u, qs.v, qs.f, filter=oracle.TRILINEAR)
    assert errs == 0
    assert_rel(o_tri.cpu().numpy()[idx], ref, 1e-5)
    ref_a, errs, _ = oracle.sample_aniso(sub_m, sub_p, qs.h, qs.u, qs.v, fr.jac[idx])
    assert errs == 0
    assert_rel(o_an.cpu().numpy()[idx], ref_a, 1e-5)
