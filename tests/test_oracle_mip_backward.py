"""Pins for the oracle's mip-chain transpose (gradients of every level folded
into level 0, for training a pool whose mips are box means of level 0):
the adjoint identity against the pinned box-filter mips, conservation of
the gradient's sum, a closed form, and finite differences through mips and
trilinear sampling (Alg. 3 with LINEAR_MIPMAP_LINEAR fetches)."""
import numpy as np
import pytest

import oracle
from htexgen import pool as gpool
from htexgen.queries import uniform_queries
from tests.fixtures import tiny_meshes


def _level0_rows(lr, base):
    rows = []
    for e in range(len(lr)):
        rows.append(base[e] + np.arange(1 << (2 * int(lr[e]))))
    return np.concatenate(rows)


@pytest.mark.parametrize("channels", [4, 1])
def test_adjoint_of_the_box_mip_chain(channels):
    rng = np.random.default_rng(1)
    lr = rng.integers(0, 7, 40).astype(np.uint8)
    base, total = gpool.layout(lr, True)
    l0 = _level0_rows(lr, base)
    x = np.zeros((total, channels))
    x[l0] = rng.standard_normal((len(l0), channels))
    P = oracle.Pool(lr, base, x, True)
    y = oracle.build_mips(P)                 # every level from level 0
    r = rng.standard_normal((total, channels))
    g = oracle.mip_backward(P, r)
    lhs = float((y * r).sum())
    rhs = float((x[l0] * g[l0]).sum())
    assert abs(lhs - rhs) <= 1e-12 * max(1.0, abs(lhs))


def test_gradient_sum_is_conserved_and_closed_form():
    lr = np.array([1, 3, 0], np.uint8)
    base, total = gpool.layout(lr, True)
    P = oracle.Pool(lr, base, np.zeros((total, 4)), True)
    r = np.random.default_rng(2).standard_normal((total, 4))
    g = oracle.mip_backward(P, r)
    for e in range(3):
        k = int(lr[e])
        cnt = ((4 << (2 * k)) - 1) // 3
        n0 = 1 << (2 * k)
        np.testing.assert_allclose(g[base[e]:base[e] + n0].sum(0),
                                   r[base[e]:base[e] + cnt].sum(0), rtol=1e-12)
    # 2x2 + 1x1: the 1x1 gradient is shared out in quarters
    d = np.zeros((total, 4))
    d[base[0] + 4] = [4.0, -8.0, 1.0, 0.0]
    g = oracle.mip_backward(P, d)
    np.testing.assert_array_equal(g[base[0]:base[0] + 4], np.tile([1.0, -2.0, 0.25, 0.0], (4, 1)))
    # a 1x1 texture has no coarser level: its gradient is unchanged
    d[base[2]] = [3.0, 0, 0, 0]
    np.testing.assert_array_equal(oracle.mip_backward(P, d)[base[2]], [3.0, 0, 0, 0])


@pytest.mark.parametrize("mesh_i", [0, 3])
def test_finite_differences_through_mips_and_trilinear_sampling(mesh_i):
    """L(x) = sum(sample(mips(x)) * dout) is linear in level 0 x; its
    gradient is mip_backward(backward(dout)) on level 0.  Central
    differences of L at random level-0 texels agree to rounding."""
    m = tiny_meshes()[mesh_i]
    rng = np.random.default_rng(3 + mesh_i)
    lr = rng.integers(1, 5, m.E).astype(np.uint8)
    base, total = gpool.layout(lr, True)
    l0 = _level0_rows(lr, base)
    x = np.zeros((total, 4))
    x[l0] = rng.uniform(0, 1, (len(l0), 4))
    M = oracle.Mesh.of(m)
    q = uniform_queries(m.H, 3000, 5 + mesh_i, log2f=(-6, 1))
    dout = rng.standard_normal((q.Q, 4))

    def loss(xx):
        P = oracle.Pool(lr, base, xx, True)
        P = oracle.Pool(lr, base, oracle.build_mips(P), True)
        out, _, _ = oracle.sample(M, P, q.h, q.u, q.v, q.f, filter=oracle.TRILINEAR)
        return float((out * dout).sum())

    P = oracle.Pool(lr, base, oracle.build_mips(oracle.Pool(lr, base, x, True)), True)
    dt = oracle.backward(M, P, q.h, q.u, q.v, dout, q.f, filter=oracle.TRILINEAR)
    g = oracle.mip_backward(P, dt)
    # the texels every query touches through some level carry a gradient
    picks = rng.choice(l0, 40, replace=False)
    eps = 1e-3
    for t in picks:
        for c in (0, 2):
            xp = x.copy()
            xm = x.copy()
            xp[t, c] += eps
            xm[t, c] -= eps
            fd = (loss(xp) - loss(xm)) / (2 * eps)
            assert abs(fd - g[t, c]) <= 1e-7 * max(1.0, abs(fd)), (t, c, fd, g[t, c])
    # the gradient without the mip transpose misses the coarse levels' share
    assert np.abs(g[l0] - dt[l0]).max() > 1e-3
