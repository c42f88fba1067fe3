"""Property-based pins of the oracle on generated meshes (hypothesis): mixed
polygons from split and merged cube grids, and small spheres with holes
(boundary edges).  On each: Alg. 3 against the independent tent-kernel
formulation, constant textures reproduced under trilinear filtering with
the normalization channel in its bounds, and the twin-diagonal seam bit
for bit."""
import numpy as np
import pytest
from hypothesis import HealthCheck, given, settings
from hypothesis import strategies as st

import oracle
from htexgen import pool as gpool
from htexgen.mesh import cube_mesh, sphere_mesh
from htexgen.queries import uniform_queries
from tests.test_oracle_pins import _brute

SETTINGS = settings(max_examples=20, deadline=None, derandomize=True,
                    suppress_health_check=[HealthCheck.too_slow])


@st.composite
def meshes(draw):
    if draw(st.booleans()):
        n = draw(st.integers(1, 3))
        return cube_mesh(n=n, seed=draw(st.integers(0, 10 ** 6)),
                         n_split=draw(st.integers(0, 2 * n * n)),
                         n_merge=draw(st.integers(0, n * n // 2)))
    return sphere_mesh(n=draw(st.integers(3, 5)), seed=draw(st.integers(0, 10 ** 6)),
                       frac_hole=draw(st.sampled_from([0.0, 0.05, 0.1])))


@SETTINGS
@given(m=meshes(), seed=st.integers(0, 10 ** 6))
def test_alg3_matches_tent_kernel_on_generated_meshes(m, seed):
    M = oracle.Mesh.of(m)
    assert oracle.validate(M) == (0, -1)
    rng = np.random.default_rng(seed)
    lr = rng.integers(0, 4, m.E).astype(np.uint8)
    base, total = gpool.layout(lr, False)
    T = gpool.fill_level0_host(0, seed % 1000, lr, base, total, m.boundary_edges(), False)
    P = oracle.Pool(lr, base, T.astype(np.float64), False)
    q = uniform_queries(m.H, 60, seed)
    out, errs, _ = oracle.sample(M, P, q.h, q.u, q.v)
    assert errs == 0
    ref = _brute(m, lr, base, P.texels, q.h, q.u, q.v)
    np.testing.assert_allclose(out, ref, rtol=1e-12, atol=1e-14)


@SETTINGS
@given(m=meshes(), seed=st.integers(0, 10 ** 6))
def test_constants_and_normalization_on_generated_meshes(m, seed):
    rng = np.random.default_rng(seed)
    lr = rng.integers(0, 5, m.E).astype(np.uint8)
    base, total = gpool.layout(lr, True)
    c = rng.uniform(0.1, 2.0, 4)
    P = oracle.Pool(lr, base, np.tile(c, (total, 1)), True)
    M = oracle.Mesh.of(m)
    q = uniform_queries(m.H, 200, seed, log2f=(-8, 1))
    out, errs, d = oracle.sample(M, P, q.h, q.u, q.v, q.f, filter=oracle.TRILINEAR, debug=True)
    np.testing.assert_allclose(out, np.tile(c, (q.Q, 1)), rtol=1e-12)
    assert (d["W"] >= 0.25 - 1e-12).all()


@SETTINGS
@given(m=meshes(), seed=st.integers(0, 10 ** 6))
def test_twin_seam_on_generated_meshes(m, seed):
    lr = np.full(m.E, 3, np.uint8)
    base, total = gpool.layout(lr, False)
    T = gpool.fill_level0_host(1, seed % 1000, lr, base, total, m.boundary_edges(), False)
    P = oracle.Pool(lr, base, T.astype(np.float64), False)
    M = oracle.Mesh.of(m)
    hs = np.nonzero(m.twin >= 0)[0]
    uu = (np.arange(4, 29) / 32.0).astype(np.float32)     # >= 1/2 texel from the ends
    h = np.repeat(hs, len(uu)).astype(np.int32)
    u = np.tile(uu, len(hs))
    a, _, _ = oracle.sample(M, P, h, u, (1 - u).astype(np.float32))
    b, _, _ = oracle.sample(M, P, m.twin[h].astype(np.int32), (1 - u).astype(np.float32), u)
    np.testing.assert_array_equal(a, b)
