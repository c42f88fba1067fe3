"""Pins for the oracle's one-channel pools (a displacement map is one value
per texel).  Alg. 3 filters every channel with the same weights and
normalizes each by the same border-normalization channel, so a
one-channel pool must give exactly channel c of a four-channel pool whose
channel c holds the same values -- for sampling, the gradient, the mips and
the corner pre-processing.  The four-channel oracle is pinned elsewhere.
"""
import numpy as np
import pytest

import oracle
from htexgen import pool as gpool
from htexgen.queries import tessellated_queries, uniform_queries
from tests.fixtures import tiny_meshes


def _pools(m, lr, has_mips, seed=5):
    base, total = gpool.layout(lr, has_mips)
    T = gpool.fill_level0_host(1, seed, lr, base, total, m.boundary_edges(), has_mips)
    P4 = oracle.Pool(lr, base, T.astype(np.float64), has_mips)
    if has_mips:
        P4 = oracle.Pool(lr, base, oracle.build_mips(P4), True)
    return base, P4


@pytest.mark.parametrize("mesh_i", range(4))
@pytest.mark.parametrize("c", [0, 3])
def test_one_channel_pool_is_a_channel_of_four(mesh_i, c):
    m = tiny_meshes()[mesh_i]
    lr = np.random.default_rng(mesh_i).integers(0, 5, m.E).astype(np.uint8)
    base, P4 = _pools(m, lr, True)
    # level 0 only copied: the one-channel mips are built by the oracle itself
    lvl0 = P4.texels[:, c:c + 1].copy()
    P1 = oracle.Pool(lr, base, lvl0, True)
    P1 = oracle.Pool(lr, base, oracle.build_mips(P1), True)
    np.testing.assert_array_equal(P1.texels[:, 0], P4.texels[:, c])
    M = oracle.Mesh.of(m)
    q = uniform_queries(m.H, 3000, 17 + mesh_i, log2f=(-7, 1))
    for filt in (oracle.BILINEAR, oracle.TRILINEAR):
        o4, e4, d4 = oracle.sample(M, P4, q.h, q.u, q.v, q.f, filter=filt, debug=True)
        o1, e1, d1 = oracle.sample(M, P1, q.h, q.u, q.v, q.f, filter=filt, debug=True)
        assert o1.shape == (q.Q, 1) and e1 == e4
        np.testing.assert_array_equal(o1[:, 0], o4[:, c])
        np.testing.assert_array_equal(d1, d4)
        dout = np.random.default_rng(3).normal(size=(q.Q, 4))
        g4 = oracle.backward(M, P4, q.h, q.u, q.v, dout, q.f, filter=filt)
        g1 = oracle.backward(M, P1, q.h, q.u, q.v, dout[:, c:c + 1].copy(), q.f, filter=filt)
        np.testing.assert_array_equal(g1[:, 0], g4[:, c])
    C4 = oracle.corner_average(M, P4, m.vert, m.face, m.V, m.F)
    C1 = oracle.corner_average(M, P1, m.vert, m.face, m.V, m.F)
    np.testing.assert_array_equal(C1[:, 0], C4[:, c])
    e, x, y = 1, 0.3, 0.7
    w4 = oracle.texture_fetch(P4, e, x, y)
    w1 = oracle.texture_fetch(P1, e, x, y)
    assert w1[1] == w4[1] and w1[0][0] == w4[0][c] and len(w1[0]) == 1


def test_one_channel_fp8_scale_is_the_channel_maximum():
    m = tiny_meshes()[0]
    lr = np.full(m.E, 3, np.uint8)
    base, P4 = _pools(m, lr, True)
    t1 = P4.texels[:, 1:2].astype(np.float32)
    codes, scale = oracle.quantize_e4m3(lr, base, True, t1)
    assert codes.shape == t1.shape
    per_edge = int((4 ** np.arange(4)).sum())      # texels of an 8x8 mip chain
    for e in range(m.E):
        seg = t1[base[e]:base[e] + per_edge, 0]
        assert scale[e] == np.float32(np.abs(seg).max()) / np.float32(448.0)
        want = oracle.f64_to_e4m3((seg / scale[e]).astype(np.float32))
        np.testing.assert_array_equal(codes[base[e]:base[e] + per_edge, 0], want)
    deq = oracle.e4m3_pool_to_f64(lr, base, True, codes, scale)
    tab = oracle.e4m3_table()
    np.testing.assert_array_equal(deq[base[2]:base[2] + per_edge, 0],
                                  tab[codes[base[2]:base[2] + per_edge, 0]] * np.float64(scale[2]))


def test_tessellated_queries_cover_each_patch_once():
    q = tessellated_queries(5, 4, footprint=0.25)
    assert q.Q == 5 * 15
    pts = set(zip(q.h.tolist(), (q.u * 4).astype(int).tolist(), (q.v * 4).astype(int).tolist()))
    assert len(pts) == q.Q
    assert ((q.u + q.v) <= 1).all() and (q.f == np.float32(0.25)).all()
