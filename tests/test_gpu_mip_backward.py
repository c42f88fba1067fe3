"""The mip-chain transpose on the GPU (htex_mip_backward) against the FP64
oracle, the full trilinear gradient with respect to level 0 (sample
backward, then the transpose) on mixed resolutions, and trilinear training
of level 0 with the mips rebuilt after every step.

Bar: the transpose within 2^-21 of the oracle scaled by the transpose of
|gradient| (float32 sums of a few terms per level); the full gradient
within 1e-4 of the sum of absolute contributions, as for the plain
backward."""
import numpy as np
import pytest
import torch

import oracle
import paper_2207_05618_amd as htex
from htexgen import pool as gpool
from htexgen.mesh import cube_mesh
from htexgen.queries import uniform_queries
from tests.fixtures import tiny_meshes
from tests.gpu_helpers import Setup, t

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("channels", [4, 1])
@pytest.mark.parametrize("clear", [False, True])
def test_mip_backward_matches_oracle(channels, clear):
    rng = np.random.default_rng(20)
    lr = rng.integers(0, 9, 300).astype(np.uint8)
    pool = htex.Pool(lr, True, channels=channels)
    d = rng.standard_normal((pool.total, channels)).astype(np.float32)
    g = htex.htex_mip_backward(pool, t(d), clear_coarse=clear)
    torch.cuda.synchronize()
    got = g.cpu().numpy()
    op = oracle.Pool(lr, pool.base_host, np.zeros((1, channels)), True)
    ref = oracle.mip_backward(op, d.astype(np.float64))
    scale = oracle.mip_backward(op, np.abs(d).astype(np.float64))
    level0 = np.zeros(pool.total, bool)
    for e in range(len(lr)):
        level0[pool.base_host[e]:pool.base_host[e] + (1 << (2 * int(lr[e])))] = True
    assert (np.abs(got[level0] - ref[level0]) <= 2.0 ** -21 * scale[level0] + 1e-30).all()
    if clear:
        coarse = ~level0
        # padding texels between edges stay as they were
        pad = np.ones(pool.total, bool)
        for e in range(len(lr)):
            k = int(lr[e])
            pad[pool.base_host[e]:pool.base_host[e] + ((4 << (2 * k)) - 1) // 3] = False
        np.testing.assert_array_equal(got[coarse & ~pad], 0)
        np.testing.assert_array_equal(got[pad], d[pad])
    else:
        assert (np.abs(got - ref) <= 2.0 ** -21 * scale + 1e-30).all()


@pytest.mark.parametrize("flags", [0, htex.HTEX_QUERIES_SORTED])
def test_trilinear_gradient_with_respect_to_level0(flags):
    m = cube_mesh()
    s = Setup(m, np.random.default_rng(21).integers(1, 7, m.E), has_mips=True, kind=1, seed=22)
    q = uniform_queries(m.H, 200000, 23, log2f=(-8, 1), sort=True)
    g = np.random.default_rng(24).standard_normal((q.Q, 4)).astype(np.float32)
    d = htex.htex_sample_backward(s.dmesh, s.pool, t(q.h), t(q.u), t(q.v), t(g), t(q.f),
                                  filter=htex.HTEX_TRILINEAR, flags=flags)
    htex.htex_mip_backward(s.pool, d, clear_coarse=True)
    torch.cuda.synchronize()
    got = d.cpu().numpy()
    dt, dabs = oracle.backward(s.omesh, s.opool, q.h, q.u, q.v, g.astype(np.float64), q.f,
                               filter=oracle.TRILINEAR, with_abs=True)
    ref = oracle.mip_backward(s.opool, dt)
    scale = oracle.mip_backward(s.opool, dabs)
    lvl0 = np.zeros(len(got), bool)
    for e in range(m.E):
        b = s.pool.base_host[e]
        lvl0[b:b + (1 << (2 * int(s.log2res[e])))] = True
    assert (np.abs(got[lvl0] - ref[lvl0]) <= 1e-4 * scale[lvl0] + 1e-7).all()
    assert (got[~lvl0] == 0).all()


def test_trilinear_training_of_level0():
    """Adam on level 0 only (mips rebuilt from it after every step, gradient
    folded through the mip chain) fits a trilinearly sampled target."""
    m = tiny_meshes()[0]
    lr = np.random.default_rng(25).integers(2, 6, m.E).astype(np.uint8)
    base, total = gpool.layout(lr, True)
    dm = htex.Mesh.of(m)
    tgt = htex.Pool(lr, True, texels=t(gpool.fill_level0_host(1, 26, lr, base, total,
                                                               m.boundary_edges(), True)))
    htex.htex_build_mips(tgt)
    q = uniform_queries(m.H, 400000, 27, log2f=(-7, 0), sort=True)
    h, u, v, f = t(q.h), t(q.u), t(q.v), t(q.f)
    y, _ = htex.htex_sample(dm, tgt, h, u, v, f, filter=htex.HTEX_TRILINEAR)
    tex = torch.full((total, 4), 0.5, dtype=torch.float32, device="cuda")
    pool = htex.Pool(lr, True, texels=tex)
    tex.requires_grad_(True)
    opt = torch.optim.Adam([tex], lr=0.02)
    losses = []
    for it in range(200):
        with torch.no_grad():
            htex.htex_build_mips(pool)
        opt.zero_grad(set_to_none=False)
        o = htex.HtexSample.apply(tex, dm, pool, h, u, v, f, htex.HTEX_TRILINEAR,
                                  htex.HTEX_QUERIES_SORTED, True)
        loss = ((o - y) ** 2).mean()
        loss.backward()
        opt.step()
        losses.append(float(loss.item()))
    assert losses[-1] < 1e-3 * losses[0], (losses[0], losses[-1])
