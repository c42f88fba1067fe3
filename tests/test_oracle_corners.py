"""Pins for the oracle's corner pre-processing (Section 4.4, "Corner
Pre-processing") and for the crack-free displacement it exists for.

The oracle groups corner texels by vertex and face ids.  The tests here
group them another way -- by the 3D point each corner stands for, from the
intrinsic triangle vertices of Alg. 1 and the barycentric frame of Section
4.2 -- and check the paper's claim itself: after the pre-processing, every
intrinsic triangle that meets a mesh vertex (or a face centroid) returns
one value there, and a tessellated surface sampled per patch has no cracks
when its textures share one resolution.  Each claim is also shown to fail
without the pre-processing, so none of the checks is vacuous.
"""
import numpy as np
import pytest
from scipy.spatial import cKDTree

import oracle
from htexgen import pool as gpool
from htexgen.mesh import cube_mesh, sphere_mesh
from htexgen.queries import tessellated_queries
from tests.fixtures import load_fig2, tiny_meshes


def _meshes():
    # closed mixed-polygon cubes, the Fig. 2 mesh and an open strip (boundary
    # edges), plus a small sphere with holes
    return tiny_meshes() + [sphere_mesh(n=6, seed=5, frac_hole=0.05)]


def _setup(m, k=3, has_mips=True, mixed=False, seed=102):
    lr = np.full(m.E, k, np.uint8)
    if mixed:
        lr = np.random.default_rng(seed).integers(1, k + 1, size=m.E).astype(np.uint8)
    base, total = gpool.layout(lr, has_mips)
    T = gpool.fill_level0_host(0, seed, lr, base, total, m.boundary_edges(), has_mips)
    P = oracle.Pool(lr, base, T.astype(np.float64), has_mips)
    if has_mips:
        P = oracle.Pool(lr, base, oracle.build_mips(P), True)
    M = oracle.Mesh.of(m)
    C = oracle.Pool(lr, base, oracle.corner_average(M, P, m.vert, m.face, m.V, m.F), has_mips)
    return M, P, C


def _centroids(m, pos):
    c = np.zeros((m.F, 3))
    np.add.at(c, m.face, pos[m.vert])
    return c / np.bincount(m.face, minlength=m.F)[:, None]


def _positions(m):
    if m.positions is not None:
        return np.asarray(m.positions, np.float64)
    # meshes given without geometry: any injective placement will do
    return np.random.default_rng(9).normal(size=(m.V, 3))


def _corner_points(m, P):
    """Rows (texel index, resolution r, 3D point, is_boundary_mirror) for
    every corner texel of every level with n >= 2: Alg. 1 places Vert(h) at
    (u, v) = (1, 0), Vert(Next h) at (0, 1) and the face centroid at (0, 0)
    of h's triangle (Section 4.2); the larger halfedge of an edge keeps its
    (u, v) as quad coordinates (Alg. 2)."""
    pos = _positions(m)
    cen = _centroids(m, pos)
    rows = []
    for g in range(m.H):
        t = m.twin[g]
        if not g > t:
            continue
        e = m.edge[g]
        k = int(P.log2res[e])
        for l in range(0, k + 1 if P.has_mips else 1):
            n = 1 << (k - l)
            if n < 2:
                continue
            lv = int(P.base[e]) + sum(4 ** (k - mm) for mm in range(l))
            pts = [(lv + n - 1, pos[m.vert[g]], False),                 # (1, 0)
                   (lv + (n - 1) * n, pos[m.vert[m.next[g]]], False),   # (0, 1)
                   (lv, cen[m.face[g]], False)]                         # (0, 0)
            if t >= 0:
                pts.append((lv + (n - 1) * n + n - 1, cen[m.face[t]], False))
            else:
                pts.append((lv + (n - 1) * n + n - 1, None, True))     # mirror of (0, 0)
            for idx, p, mir in pts:
                rows.append((idx, n, p, mir, lv))
    return rows


@pytest.mark.parametrize("mesh_i", range(5))
@pytest.mark.parametrize("mixed", [False, True])
def test_corner_texels_on_one_point_share_their_mean(mesh_i, mixed):
    """Corner texels grouped by the 3D point they stand for (and by level
    resolution) all hold the mean of their original values; a boundary
    quad's far corner equals its (0, 0) corner; nothing else changes."""
    m = _meshes()[mesh_i]
    M, P, C = _setup(m, mixed=mixed)
    rows = _corner_points(m, P)
    real = [r for r in rows if not r[3]]
    pts = np.array([r[2] for r in real])
    tree = cKDTree(pts)
    groups = {}
    for a, b in tree.query_pairs(1e-9):
        groups.setdefault(a, {a}).add(b)
    # union-find over the close pairs, split by resolution
    parent = list(range(len(real)))

    def find(x):
        while parent[x] != x:
            parent[x] = parent[parent[x]]
            x = parent[x]
        return x

    for a, b in tree.query_pairs(1e-9):
        if real[a][1] == real[b][1]:
            parent[find(a)] = find(b)
    members = {}
    for i in range(len(real)):
        members.setdefault(find(i), []).append(real[i][0])
    for idx in members.values():
        mean = P.texels[idx].mean(axis=0)
        np.testing.assert_allclose(C.texels[idx], np.broadcast_to(mean, (len(idx), 4)),
                                   rtol=1e-13, atol=1e-15)
    # boundary far corners mirror the (0, 0) corner
    for idx, n, _, mir, lv in rows:
        if mir:
            np.testing.assert_array_equal(C.texels[idx], C.texels[lv])
    # everything else untouched
    touched = np.zeros(len(P.texels), bool)
    touched[[r[0] for r in rows]] = True
    np.testing.assert_array_equal(C.texels[~touched], P.texels[~touched])
    # idempotent
    again = oracle.corner_average(M, C, m.vert, m.face, m.V, m.F)
    np.testing.assert_allclose(again, C.texels, rtol=1e-14, atol=1e-16)


def _vertex_and_centroid_samples(m, M, pool, filt, f):
    """Sample every intrinsic triangle at its three corners: (1, 0) is
    Vert(h), (0, 1) is Vert(Next h), (0, 0) is the centroid of h's face."""
    H = m.H
    hh = np.repeat(np.arange(H, dtype=np.int32), 3)
    uu = np.tile(np.array([1, 0, 0], np.float32), H)
    vv = np.tile(np.array([0, 1, 0], np.float32), H)
    ff = None if f is None else np.full(3 * H, f, np.float32)
    out, errs, _ = oracle.sample(M, pool, hh, uu, vv, ff, filter=filt)
    assert errs == 0
    key = np.empty(3 * H, np.int64)
    key[0::3] = m.vert
    key[1::3] = m.vert[m.next]
    key[2::3] = m.V + m.face
    return key, out


def _spread(key, out):
    worst = 0.0
    for g in np.unique(key):
        s = out[key == g]
        worst = max(worst, float(np.abs(s - s[0]).max()))
    return worst


@pytest.mark.parametrize("mesh_i", range(5))
@pytest.mark.parametrize("filt,f", [(oracle.BILINEAR, None), (oracle.TRILINEAR, 0.2),
                                    (oracle.TRILINEAR, 0.3)])
def test_every_triangle_sees_one_value_at_vertices_and_centroids(mesh_i, filt, f):
    """The point of the pre-processing (Section 4.4): filtering is continuous
    at quad corners once their texels agree.  Every intrinsic triangle that
    meets a mesh vertex or a face centroid returns the same value there
    (footprints 0.2 and 0.3 blend levels of 8/4 and 4/2 texels); before the
    pre-processing the values differ."""
    m = _meshes()[mesh_i]
    M, P, C = _setup(m)
    key, before = _vertex_and_centroid_samples(m, M, P, filt, f)
    _, after = _vertex_and_centroid_samples(m, M, C, filt, f)
    assert _spread(key, before) > 1e-3
    assert _spread(key, after) < 1e-13


def test_coarsest_level_is_left_alone():
    """A 1x1 level is not pre-processed (its one texel is four corners at
    once), so a footprint that reaches it is not continuous at corners."""
    m = cube_mesh()
    M, P, C = _setup(m)
    k = 3
    for e in range(m.E):
        lv = int(P.base[e]) + sum(4 ** (k - mm) for mm in range(k))
        np.testing.assert_array_equal(C.texels[lv], P.texels[lv])
    key, after = _vertex_and_centroid_samples(m, M, C, oracle.TRILINEAR, 0.6)
    assert _spread(key, after) > 1e-4


def _surface_points(m, q):
    """3D point of each tessellated query: u Vert(h) + v Vert(Next h) +
    w centroid(Face h), Alg. 1's triangle with Section 4.2's frame."""
    pos = _positions(m)
    cen = _centroids(m, pos)
    w = 1.0 - q.u.astype(np.float64) - q.v
    return (q.u[:, None] * pos[m.vert[q.h]] + q.v[:, None] * pos[m.vert[m.next[q.h]]]
            + w[:, None] * cen[m.face[q.h]])


@pytest.mark.parametrize("mesh_i", range(5))
@pytest.mark.parametrize("filt", [oracle.BILINEAR, oracle.TRILINEAR])
def test_tessellated_displacement_is_crack_free(mesh_i, filt):
    """Crack-free displacement (Section 5.1, Fig. 8): a surface tessellated
    per intrinsic triangle evaluates shared vertices once per patch; with
    pre-processed corners and one texture resolution, every patch returns the
    same displacement at every shared vertex (on mesh edges, on the spokes
    to the face centroid, at vertices and centroids).  Without the
    pre-processing the patches disagree at corners."""
    m = _meshes()[mesh_i]
    M, P, C = _setup(m)
    T = 8
    q = tessellated_queries(m.H, T, footprint=1.0 / T if filt == oracle.TRILINEAR else None)
    pts = _surface_points(m, q)
    pairs = np.array(sorted(cKDTree(pts).query_pairs(1e-9)))
    assert len(pairs) > m.H * T   # every patch border is shared
    res = {}
    for name, pool in (("before", P), ("after", C)):
        out, errs, _ = oracle.sample(M, pool, q.h, q.u, q.v, q.f, filter=filt)
        assert errs == 0
        res[name] = np.abs(out[pairs[:, 0]] - out[pairs[:, 1]]).max()
    assert res["before"] > 1e-3
    assert res["after"] < 1e-13


def test_mixed_resolutions_may_crack():
    """With edges of different resolutions the pre-processing cannot make
    every corner region agree (the paper reports a few cracks in that case):
    the vertex values still differ somewhere."""
    m = cube_mesh()
    M, P, C = _setup(m, k=4, mixed=True)
    key, after = _vertex_and_centroid_samples(m, M, C, oracle.BILINEAR, None)
    assert _spread(key, after) > 1e-6


@pytest.mark.parametrize("mesh_i", [0, 3, 4])
def test_corner_averaging_is_an_orthogonal_projection(mesh_i):
    """Averaging over disjoint groups (plus copying the mirrored corner) is
    linear; on the texels it treats as free it is symmetric and idempotent,
    so its transpose is itself: a gradient passes through the
    pre-processing by applying the same averaging to it.  Checked with the
    adjoint identity on random pools (mirror copies excluded, as they are
    not free parameters)."""
    m = _meshes()[mesh_i]
    M, P, _ = _setup(m, k=3)
    rows = _corner_points(m, P)
    mirror = np.zeros(len(P.texels), bool)
    mirror[[r[0] for r in rows if r[3]]] = True
    rng = np.random.default_rng(5)
    x = rng.standard_normal(P.texels.shape)
    y = rng.standard_normal(P.texels.shape)
    x[mirror] = 0.0
    y[mirror] = 0.0
    Px = oracle.corner_average(M, oracle.Pool(P.log2res, P.base, x, True), m.vert, m.face, m.V, m.F)
    Py = oracle.corner_average(M, oracle.Pool(P.log2res, P.base, y, True), m.vert, m.face, m.V, m.F)
    Px[mirror] = 0.0
    Py[mirror] = 0.0
    lhs = float((Px * y).sum())
    rhs = float((x * Py).sum())
    assert abs(lhs - rhs) <= 1e-10 * max(1.0, abs(lhs))
