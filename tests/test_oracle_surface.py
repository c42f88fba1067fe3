"""End-to-end pin of the parameterization: a function defined on the
surface in 3D, baked into the textures at each texel centre's surface point
(Section 4.2 read backwards on Alg. 1's triangles), is reproduced by Alg. 3
at every query's surface point, with an error that shrinks as the texture
resolution doubles.  A mistake in the reflection of Alg. 2, the neighbour
maps of Alg. 3, the triangle vertices of Alg. 1 or the texel addressing
makes the error of order one instead."""
import numpy as np
import pytest

import oracle
from htexgen import pool as gpool
from htexgen.mesh import cube_mesh, sphere_mesh
from htexgen.queries import uniform_queries

A = np.array([[0.3, -0.2, 0.5], [1.0, 0.0, 0.0], [0.0, 0.7, -0.1], [0.2, 0.2, 0.2]])


def _f(p):
    return p @ A.T + 0.5


def _bake(m, M, T, k, has_mips):
    lr = np.full(m.E, k, np.uint8)
    base, total = gpool.layout(lr, has_mips)
    X = oracle.texel_positions(M, T, oracle.Pool(lr, base, np.zeros((total, 4)), has_mips))
    tex = np.where(np.isnan(X[:, :1]), 0.0, _f(np.nan_to_num(X)))
    if has_mips:
        # level 0 baked, coarser levels box-filtered from it as in use
        l0 = np.zeros(total, bool)
        for e in range(m.E):
            l0[base[e]:base[e] + 4 ** k] = True
        tex[~l0] = 0.0
        P = oracle.Pool(lr, base, tex, True)
        return oracle.Pool(lr, base, oracle.build_mips(P), True)
    return oracle.Pool(lr, base, tex, False)


@pytest.mark.parametrize("which", ["cube", "sphere"])
def test_surface_function_is_reproduced_and_converges(which):
    m = cube_mesh() if which == "cube" else sphere_mesh(n=8, seed=3, frac_hole=0.05)
    M = oracle.Mesh.of(m)
    T, bad = oracle.triangle_vertices(M, m.vert, m.positions)
    assert bad == 0
    q = uniform_queries(m.H, 20000, 5)
    u = q.u.astype(np.float64)[:, None]
    v = q.v.astype(np.float64)[:, None]
    want = _f(u * T[q.h, 2] + v * T[q.h, 0] + (1 - u - v) * T[q.h, 1])
    elen = np.median(np.linalg.norm(m.positions[m.vert] - m.positions[m.vert[m.next]], axis=1))
    errs = []
    for k in (3, 4, 5, 6):
        out, e, _ = oracle.sample(M, _bake(m, M, T, k, False), q.h, q.u, q.v)
        assert e == 0
        err = np.abs(out - want).max()
        assert err <= 1.5 * elen / 2 ** k, (k, err)
        errs.append(err)
    assert all(a / b > 2.0 for a, b in zip(errs[:-1], errs[1:])), errs
    # trilinear with footprints below a texel of 64 x 64 reads levels 0-1
    # of the same baked chain and stays within a texel of level 1
    f = np.exp2(np.random.default_rng(6).uniform(-9, -6, q.Q)).astype(np.float32)
    out, _, _ = oracle.sample(M, _bake(m, M, T, 6, True), q.h, q.u, q.v, f,
                              filter=oracle.TRILINEAR)
    assert np.abs(out - want).max() <= 1.5 * elen / 2 ** 5


def test_wrong_reflection_is_caught():
    """Baking the upper-right half of each quad from the larger halfedge's
    triangle (i.e. ignoring Alg. 2's reflection) breaks reproduction."""
    m = cube_mesh()
    M = oracle.Mesh.of(m)
    T, _ = oracle.triangle_vertices(M, m.vert, m.positions)
    T_wrong = T.copy()
    i = np.nonzero(m.twin >= 0)[0]
    T_wrong[i] = T[np.maximum(i, m.twin[i])]      # both halves from one triangle
    q = uniform_queries(m.H, 5000, 7)
    u = q.u.astype(np.float64)[:, None]
    v = q.v.astype(np.float64)[:, None]
    want = _f(u * T[q.h, 2] + v * T[q.h, 0] + (1 - u - v) * T[q.h, 1])
    out, _, _ = oracle.sample(M, _bake(m, M, T_wrong, 5, False), q.h, q.u, q.v)
    assert np.abs(out - want).max() > 0.1
