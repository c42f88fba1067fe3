"""CPU checks of the raster-order query generator (htexgen/raster.py), on
intrinsic triangles from the oracle (Alg. 1): every query's surface point
(Section 4.2's frame) lies on its pixel's centre ray, the visible triangle
is the nearest front face hit by that ray (brute force), and the
derivatives are the differences of (u, v) between neighbouring pixels of
one triangle."""
import numpy as np
import pytest

import oracle
from htexgen.mesh import sphere_mesh
from htexgen.raster import rasterize, sphere_view


@pytest.fixture(scope="module")
def small():
    m = sphere_mesh(n=6, seed=3, frac_hole=0.05)
    T, bad = oracle.triangle_vertices(oracle.Mesh.of(m), m.vert, m.positions)
    assert bad == 0
    cam = sphere_view(96, 54)
    return m, T, cam, rasterize(T, cam)


def _points(T, fr):
    u = fr.u.astype(np.float64)[:, None]
    v = fr.v.astype(np.float64)[:, None]
    P = T[fr.h]
    return u * P[:, 2] + v * P[:, 0] + (1 - u - v) * P[:, 1]


def test_surface_points_lie_on_pixel_rays(small):
    m, T, cam, fr = small
    assert fr.Q > 0.5 * cam.width * cam.height
    x, y, _ = cam.project(_points(T, fr))
    np.testing.assert_allclose(x, fr.pixel % cam.width + 0.5, atol=2e-4)
    np.testing.assert_allclose(y, fr.pixel // cam.width + 0.5, atol=2e-4)
    assert (fr.u >= -1e-6).all() and (fr.v >= -1e-6).all() and (fr.u + fr.v <= 1 + 1e-6).all()
    assert (np.diff(fr.pixel) > 0).all()          # scanline order


def test_visible_triangle_is_the_nearest_front_face(small):
    """Brute force: intersect every pixel-centre ray with every intrinsic
    triangle facing the camera; the nearest hit's depth equals the
    generator's (ties on shared edges may pick either triangle)."""
    m, T, cam, fr = small
    r, up, f = cam.basis()
    t = np.tan(0.5 * cam.fov_y)
    aspect = cam.width / cam.height
    nrm = np.cross(T[:, 0] - T[:, 2], T[:, 1] - T[:, 2])
    front = ((cam.eye - T[:, 2]) * nrm).sum(1) > 0
    Tf = T[front]
    depth = np.full(cam.width * cam.height, np.inf)
    for pix in range(cam.width * cam.height):
        px, py = pix % cam.width + 0.5, pix // cam.width + 0.5
        d = f + (2 * px / cam.width - 1) * t * aspect * r + (1 - 2 * py / cam.height) * t * up
        e1 = Tf[:, 0] - Tf[:, 2]
        e2 = Tf[:, 1] - Tf[:, 2]
        s = cam.eye - Tf[:, 2]
        pv = np.cross(d, e2)
        det = (e1 * pv).sum(1)
        inv = 1.0 / det
        a = (s * pv).sum(1) * inv
        qv = np.cross(s, e1)
        b = (d * qv).sum(1) * inv
        tau = (e2 * qv).sum(1) * inv
        hit = (a >= -1e-12) & (b >= -1e-12) & (a + b <= 1 + 1e-12) & (tau > 0)
        if hit.any():
            depth[pix] = (tau[hit] * (d @ f)).min()
    covered = np.isfinite(depth)
    assert set(np.nonzero(covered)[0]) == set(fr.pixel.tolist())
    np.testing.assert_allclose(fr.depth, depth[fr.pixel], rtol=1e-9)


def test_derivatives_are_neighbour_differences(small):
    m, T, cam, fr = small
    where = -np.ones(cam.width * cam.height, np.int64)
    where[fr.pixel] = np.arange(fr.Q)
    right = fr.pixel + 1
    ok = (fr.pixel % cam.width < cam.width - 1) & (where[np.minimum(right, len(where) - 1)] >= 0)
    j = where[right[ok]]
    same = fr.h[ok] == fr.h[j]
    i = np.nonzero(ok)[0][same]
    j = j[same]
    assert len(i) > 100
    np.testing.assert_allclose(fr.jac[i, 0], fr.u[j] - fr.u[i], atol=2e-6)
    np.testing.assert_allclose(fr.jac[i, 1], fr.v[j] - fr.v[i], atol=2e-6)
    down = fr.pixel + cam.width
    ok = (down < len(where)) & (where[np.minimum(down, len(where) - 1)] >= 0)
    j = where[down[ok]]
    same = fr.h[ok] == fr.h[j]
    i = np.nonzero(ok)[0][same]
    j = j[same]
    np.testing.assert_allclose(fr.jac[i, 2], fr.u[j] - fr.u[i], atol=2e-6)
    np.testing.assert_allclose(fr.jac[i, 3], fr.v[j] - fr.v[i], atol=2e-6)
