"""Corner pre-processing on the GPU (htex_corner_average) against the FP64
oracle, and the crack-free property it exists for, end to end through the
sampler.

Bar: each processed corner texel within one float32 rounding of the
oracle's FP64 mean (the kernel sums in float64 and rounds once), texels of
one group bit-identical to each other, every other texel bit-identical to
its input; tessellated patches agree at shared vertices within float32
rounding of the three-fetch blend.
"""
import numpy as np
import pytest
import torch

import oracle
import paper_2207_05618_amd as htex
from htexgen.mesh import cube_mesh, halfedges_from_faces, sphere_mesh
from htexgen.queries import tessellated_queries
from tests.fixtures import tiny_meshes
from tests.gpu_helpers import Setup, assert_rel, t

pytestmark = pytest.mark.gpu


def _meshes():
    return tiny_meshes() + [sphere_mesh(n=6, seed=5, frac_hole=0.05)]


def _run(s):
    before = s.pool.texels.cpu().numpy().copy()
    err = torch.zeros(1, dtype=torch.int32, device="cuda")
    htex.htex_corner_average(s.dmesh, s.pool, err_count=err)
    torch.cuda.synchronize()
    return before, s.pool.texels.cpu().numpy(), int(err.item())


@pytest.mark.parametrize("mesh_i", range(5))
@pytest.mark.parametrize("layout", ["uniform_mips", "mixed_mips", "mixed_level0"])
def test_corner_average_matches_oracle(mesh_i, layout):
    m = _meshes()[mesh_i]
    rng = np.random.default_rng(300 + mesh_i)
    if layout == "uniform_mips":
        lr, mips = np.full(m.E, 4), True
    else:
        lr, mips = rng.integers(0, 6, m.E), layout == "mixed_mips"
    s = Setup(m, lr, has_mips=mips, kind=1, seed=31 + mesh_i)
    before, after, err = _run(s)
    assert err == 0
    # the oracle starts from the very float32 values the device texel pool held
    op = oracle.Pool(s.log2res, s.opool.base, before.astype(np.float64), mips)
    ref = oracle.corner_average(s.omesh, op, m.vert, m.face, m.V, m.F)
    changed = ref != before
    np.testing.assert_array_equal(after[~changed], before[~changed])
    assert_rel(after, ref, 2.0 ** -24 * 1.01, floor=1e-30)
    # deterministic: a second pass over the same input gives the same bits
    s.pool.texels.copy_(t(before))
    _, again, _ = _run(s)
    np.testing.assert_array_equal(again, after)


def test_group_members_are_bit_identical():
    m = cube_mesh()
    s = Setup(m, np.full(m.E, 3), has_mips=True, kind=0, seed=5)
    _, after, _ = _run(s)
    base = s.opool.base
    for g in range(m.H):
        if not g > m.twin[g]:
            continue
        e = m.edge[g]
        n = 8
        # the (1, 0) corner of g's quad and the (0, 1) corner of Prev(g)'s quad
        # both lie on Vert(g) when Prev(g) is its edge's larger halfedge
        # (Vert(Next p) = Vert(g))
        p = m.prev[g]
        if not p > m.twin[p]:
            continue
        a = after[base[e] + n - 1]
        b = after[base[m.edge[p]] + (n - 1) * n]
        np.testing.assert_array_equal(a, b)


@pytest.mark.parametrize("filt", [htex.HTEX_BILINEAR, htex.HTEX_TRILINEAR])
def test_tessellated_patches_agree_after_preprocessing(filt):
    """Displacement sampled per tessellated patch: every pair of queries on
    one surface point (Alg. 1 triangle geometry) agrees once the corners are
    processed; before, the patches disagree at corners."""
    from scipy.spatial import cKDTree
    m = sphere_mesh(n=6, seed=5, frac_hole=0.05)
    s = Setup(m, np.full(m.E, 3), has_mips=True, kind=0, seed=11)
    T = 8
    q = tessellated_queries(m.H, T, footprint=1.0 / T if filt == htex.HTEX_TRILINEAR else None)
    pos = np.asarray(m.positions)
    cen = np.zeros((m.F, 3))
    np.add.at(cen, m.face, pos[m.vert])
    cen /= np.bincount(m.face)[:, None]
    w = 1.0 - q.u.astype(np.float64) - q.v
    pts = (q.u[:, None] * pos[m.vert[q.h]] + q.v[:, None] * pos[m.vert[m.next[q.h]]]
           + w[:, None] * cen[m.face[q.h]])
    pairs = np.array(sorted(cKDTree(pts).query_pairs(1e-9)))
    out0, _ = s.gpu(q, filt)
    _run(s)
    out1, _ = s.gpu(q, filt)
    gap0 = np.abs(out0[pairs[:, 0]] - out0[pairs[:, 1]]).max()
    gap1 = np.abs(out1[pairs[:, 0]] - out1[pairs[:, 1]]).max()
    assert gap0 > 1e-3
    assert gap1 < 4e-7, gap1
    # and the processed pool still samples like the oracle's processed pool
    op = oracle.Pool(s.log2res, s.opool.base,
                     oracle.corner_average(s.omesh, s.opool, m.vert, m.face, m.V, m.F), True)
    ref, _, _ = oracle.sample(s.omesh, op, q.h, q.u, q.v, q.f,
                              filter=oracle.TRILINEAR if filt else oracle.BILINEAR)
    assert_rel(out1, ref, 1e-5)


def test_overlong_face_ring_is_counted_and_left_alone():
    """A 70000-sided face (all boundary) has a Next cycle longer than the
    65536-halfedge walk limit: the lanes whose ownership walk would exceed
    it count an error (halfedges 0..4463) and the face's corners stay as
    they were; the vertex corners are still processed."""
    N = 70000
    m = halfedges_from_faces([list(range(N))])
    s = Setup(m, np.full(m.E, 1), has_mips=False, kind=0, seed=3)
    before, after, err = _run(s)
    assert err == N - 65536
    base = s.opool.base
    n = 2
    e0 = m.edge[0]
    np.testing.assert_array_equal(after[base[e0]], before[base[e0]])            # (0, 0)
    # each boundary vertex joins the (1, 0) corner of one quad and the
    # (0, 1) corner of the previous one
    g = 5
    a = after[base[m.edge[g]] + n - 1]
    b = after[base[m.edge[m.prev[g]]] + (n - 1) * n]
    np.testing.assert_array_equal(a, b)
    np.testing.assert_array_equal(
        a, ((before[base[m.edge[g]] + n - 1].astype(np.float64)
             + before[base[m.edge[m.prev[g]]] + (n - 1) * n]) / 2).astype(np.float32))


def test_corner_average_rejects_quantized_pools():
    m = cube_mesh()
    s = Setup(m, np.full(m.E, 2), has_mips=False)
    qp = htex.htex_quantize(s.pool, htex.HTEX_BF16)
    with pytest.raises(htex.HtexError):
        htex.htex_corner_average(s.dmesh, qp)
