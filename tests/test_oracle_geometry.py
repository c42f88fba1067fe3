"""Pins for the oracle's intrinsic triangles (Alg. 1, Section 3.1) and their
barycentric frame (Section 4.2): the paper's worked example on the Fig. 2
mesh, tiling of planar faces (areas add up to the polygon's), the
adjacency the paper states (shared vertices with Next and Twin, a common
centroid per face), and agreement of the frame with Alg. 2's quad
parameterization and Alg. 3's neighbour maps on shared boundaries."""
import os

import numpy as np
import pytest

import oracle
from htexgen.mesh import cube_mesh, halfedges_from_faces, sphere_mesh
from tests.fixtures import GOLDEN, load_fig2


def _tri(m, pos=None):
    pos = m.positions if pos is None else pos
    return oracle.triangle_vertices(oracle.Mesh.of(m), m.vert, pos)


def test_fig2_worked_example():
    m = load_fig2()
    pos = np.random.default_rng(1).normal(size=(m.V, 3))
    T, bad = _tri(m, pos)
    assert bad == 0
    role = {"v0": 0, "v1": 1, "v2": 2}
    n = 0
    with open(os.path.join(GOLDEN, "fig2_triangle_t7.txt")) as fh:
        for line in fh:
            if not line.strip() or line.startswith("#"):
                continue
            f = line.split()
            h, r, hs = int(f[0]), f[1], [int(x) for x in f[2:]]
            want = pos[m.vert[hs]].mean(0)
            np.testing.assert_allclose(T[h, role[r]], want, rtol=1e-15, atol=1e-15)
            n += 1
    assert n == 3


def _area(a, b, c):
    return 0.5 * np.linalg.norm(np.cross(b - a, c - a), axis=-1)


def test_triangles_tile_planar_convex_faces():
    """The intrinsic triangulation does not change the surface: on a planar
    mesh of convex polygons (3 to 9 sides) the triangles of each face
    cover exactly its area (shoelace formula)."""
    rng = np.random.default_rng(2)
    faces, pts = [], []
    for f in range(40):
        k = int(rng.integers(3, 10))
        ang = np.sort(rng.uniform(0, 2 * np.pi, k))
        c = rng.uniform(-10, 10, 2)
        r = rng.uniform(0.5, 2.0)
        p = np.stack([c[0] + r * np.cos(ang), c[1] + r * np.sin(ang), np.zeros(k)], 1)
        faces.append(list(range(len(pts), len(pts) + k)))
        pts.extend(p)
    pts = np.array(pts)
    m = halfedges_from_faces(faces, positions=pts)
    T, _ = _tri(m)
    A = _area(T[:, 0], T[:, 1], T[:, 2])
    for f, fv in enumerate(faces):
        p = pts[fv]
        shoe = 0.5 * abs(np.dot(p[:, 0], np.roll(p[:, 1], -1)) - np.dot(p[:, 1], np.roll(p[:, 0], -1)))
        np.testing.assert_allclose(A[m.face == f].sum(), shoe, rtol=1e-12)


@pytest.mark.parametrize("make", [cube_mesh, lambda: sphere_mesh(n=8, seed=3, frac_hole=0.05)])
def test_adjacency_of_intrinsic_triangles(make):
    """Section 3.1: t_h and t_Next(h) share the vertex Vert(Next h); t_h and
    t_Twin(h) share the mesh edge (reversed); all triangles of a face share
    the face centroid."""
    m = make()
    T, bad = _tri(m)
    assert bad == 0
    np.testing.assert_array_equal(T[:, 0], T[m.next, 2])
    i = np.nonzero(m.twin >= 0)[0]
    np.testing.assert_array_equal(T[i, 0], T[m.twin[i], 2])
    np.testing.assert_array_equal(T[i, 2], T[m.twin[i], 0])
    cen = np.zeros((m.F, 3))
    np.add.at(cen, m.face, m.positions[m.vert])
    cen /= np.bincount(m.face)[:, None]
    np.testing.assert_allclose(T[:, 1], cen[m.face], rtol=1e-13, atol=1e-15)


def _point(T, h, u, v):
    u = np.asarray(u, np.float64)[:, None]
    v = np.asarray(v, np.float64)[:, None]
    w = 1.0 - u - v
    return u * T[h, 2] + v * T[h, 0] + w * T[h, 1]


def test_frame_agrees_with_the_quad_and_neighbour_maps():
    """(u, v) on t_h and on a neighbour name one surface point exactly when
    Alg. 2 / Alg. 3 say so: the twin's (1-u, 1-v) on the shared edge
    (x + y = 1 in the quad), and Next's (v, -u) / Prev's (-v, u) on the
    spokes to the centroid (u = 0 and v = 0)."""
    m = sphere_mesh(n=6, seed=4, frac_hole=0.05)
    T, _ = _tri(m)
    t = np.linspace(0, 1, 11)
    i = np.nonzero(m.twin >= 0)[0]
    for h in i:
        a = _point(T, h, t, 1 - t)
        b = _point(T, m.twin[h], 1 - t, t)
        np.testing.assert_allclose(a, b, atol=1e-13)
    for h in range(m.H):
        np.testing.assert_allclose(_point(T, h, 0 * t, t), _point(T, m.next[h], t, 0 * t),
                                   atol=1e-13)
        np.testing.assert_allclose(_point(T, h, t, 0 * t), _point(T, m.prev[h], 0 * t, t),
                                   atol=1e-13)


def test_unresolvable_halfedges_are_reported():
    m = cube_mesh()
    vert = m.vert.copy()
    vert[5] = m.V + 3
    T, bad = oracle.triangle_vertices(oracle.Mesh.of(m), vert, m.positions)
    assert bad > 0 and np.isnan(T[5]).all()
