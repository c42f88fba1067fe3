"""Pins for the oracle's anisotropic filtering (Section 5.1, Fig. 7; the
reading is the OpenGL anisotropic-filtering extension's filter applied to
each of Alg. 3's fetches).

The probe count and the probe points are integer-deciding float32 steps;
the rest composes the already pinned trilinear fetch.  Pins: the isotropic
case is plain trilinear sampling; probe counts against exact rational
ratios; linear textures return their value at the footprint centre (the
probes are symmetric and summed before the division); an independent
composition of single fetches in Python; axis symmetries; constants.
"""
from fractions import Fraction

import numpy as np
import pytest

import oracle
from htexgen import pool as gpool
from tests.fixtures import tiny_meshes
from htexgen.queries import uniform_queries


def _setup(m, k=5, kind=1, seed=3, texels=None):
    lr = np.full(m.E, k, np.uint8) if np.isscalar(k) else np.asarray(k, np.uint8)
    base, total = gpool.layout(lr, True)
    if texels is None:
        T = gpool.fill_level0_host(kind, seed, lr, base, total, m.boundary_edges(), True)
    else:
        T = texels(lr, base, total)
    P = oracle.Pool(lr, base, T.astype(np.float64), True)
    P = oracle.Pool(lr, base, oracle.build_mips(P), True)
    return oracle.Mesh.of(m), P, lr, base


def _jac(Q, seed, ratio_hi=40.0):
    """Random derivative pairs: a major axis of random direction and length
    2^U[-9, -2], a minor axis of random direction shorter by a log-uniform
    ratio in [1, ratio_hi]."""
    rng = np.random.default_rng(seed)
    L = np.exp2(rng.uniform(-9, -2, Q))
    r = np.exp(rng.uniform(0, np.log(ratio_hi), Q))
    a, b = rng.uniform(0, 2 * np.pi, (2, Q))
    J = np.stack([L * np.cos(a), L * np.sin(a), L / r * np.cos(b), L / r * np.sin(b)], 1)
    swap = rng.random(Q) < 0.5
    J[swap] = J[swap][:, [2, 3, 0, 1]]
    return J.astype(np.float32)


def test_isotropic_footprint_is_trilinear():
    """Equal axis lengths: one probe at (u, v) with footprint |d/dx|, i.e.
    Alg. 3 with trilinear fetches, bit for bit."""
    m = tiny_meshes()[0]
    M, P, _, _ = _setup(m)
    q = uniform_queries(m.H, 4000, 5)
    rng = np.random.default_rng(6)
    a = (np.exp2(rng.uniform(-9, 0, q.Q)) * rng.choice([-1, 1], q.Q)).astype(np.float32)
    b = (np.exp2(rng.uniform(-9, 0, q.Q)) * rng.choice([-1, 1], q.Q)).astype(np.float32)
    J = np.stack([a, b, -b, a], 1)
    f = np.sqrt(a * a + b * b)            # float32, one rounding per operation
    out, errs, n = oracle.sample_aniso(M, P, q.h, q.u, q.v, J)
    ref, _, _ = oracle.sample(M, P, q.h, q.u, q.v, f, filter=oracle.TRILINEAR)
    assert errs == 0 and (n == 1).all()
    np.testing.assert_array_equal(out, ref)


def test_probe_count_against_exact_ratios():
    m = tiny_meshes()[0]
    M, P, _, _ = _setup(m, k=3)
    Q = 20000
    J = _jac(Q, 7)
    h = np.zeros(Q, np.int32)
    u = np.full(Q, 0.25, np.float32)
    _, _, n = oracle.sample_aniso(M, P, h, u, u, J, max_aniso=16)
    checked = 0
    for i in range(0, Q, 7):
        px2 = Fraction(float(J[i, 0])) ** 2 + Fraction(float(J[i, 1])) ** 2
        py2 = Fraction(float(J[i, 2])) ** 2 + Fraction(float(J[i, 3])) ** 2
        r2 = max(px2, py2) / min(px2, py2)      # exact squared ratio
        c = 1
        while Fraction(c * c) < r2:
            c += 1                              # c = ceil(exact ratio)
        # skip ratios within 1e-5 of an integer: float32 decides those
        near = any(abs(float(r2) ** 0.5 - j) < 1e-5 * j for j in (c - 1, c))
        if near:
            continue
        assert n[i] == min(c, 16), (i, float(r2) ** 0.5, n[i])
        checked += 1
    assert checked > 2500
    # degenerate footprints
    Jd = np.array([[1e-3, 0, 0, 0], [0, 0, 0, 0], [0, 1e-3, 1e-3, 0], [3e-3, 0, 0, 1e-3]],
                  np.float32)
    _, _, nd = oracle.sample_aniso(M, P, h[:4], u[:4], u[:4], Jd, max_aniso=16)
    np.testing.assert_array_equal(nd, [16, 1, 1, 3])
    _, _, nd = oracle.sample_aniso(M, P, h[:4], u[:4], u[:4], Jd, max_aniso=2)
    np.testing.assert_array_equal(nd, [2, 1, 1, 2])


def _ramp(lr, base, total):
    """Level 0 of every edge holds (x, y, 1, x y) at its texel centres; box
    mips of a function linear in x and y stay exact at coarser centres for
    the first three channels."""
    T = np.zeros((total, 4), np.float64)
    for e in range(len(lr)):
        n = 1 << int(lr[e])
        jj, ii = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
        x = (ii + 0.5) / n
        y = (jj + 0.5) / n
        T[base[e]:base[e] + n * n] = np.stack([x, y, np.ones_like(x), x * y], -1).reshape(-1, 4)
    return T


def test_linear_texture_returns_the_footprint_centre():
    """Probes sit symmetrically about (u, v) and every probe that stays
    inside its quad has normalization 1, so a texture linear in the quad
    coordinates returns its value at (u, v) for any probe count."""
    m = tiny_meshes()[0]
    M, P, lr, _ = _setup(m, k=6, texels=_ramp)
    rng = np.random.default_rng(8)
    Q = 3000
    h = rng.integers(0, m.H, Q).astype(np.int32)
    # points of the own triangle whose footprint stays inside the quad
    u = rng.uniform(0.25, 0.45, Q).astype(np.float32)
    v = rng.uniform(0.25, 0.45, Q).astype(np.float32)
    J = _jac(Q, 9)
    J *= np.float32(0.5) / np.maximum(np.abs(J).max(1, keepdims=True), 1e-30) * \
        np.exp2(rng.uniform(-6, -2, (Q, 1))).astype(np.float32)   # axes shorter than 0.125
    out, errs, n = oracle.sample_aniso(M, P, h, u, v, J)
    assert errs == 0 and n.max() > 8
    flip = ~(h > m.twin[h])
    x = np.where(flip, 1 - u.astype(np.float64), u)
    y = np.where(flip, 1 - v.astype(np.float64), v)
    np.testing.assert_allclose(out[:, 0], x, atol=2e-6)
    np.testing.assert_allclose(out[:, 1], y, atol=2e-6)
    np.testing.assert_allclose(out[:, 2], 1.0, atol=1e-12)


def _probe_points(J, u, v, max_aniso):
    """Probe count, footprint and points, in float32 with numpy (one
    rounding per operation)."""
    f32 = np.float32
    px = np.sqrt(J[0] * J[0] + J[1] * J[1])
    py = np.sqrt(J[2] * J[2] + J[3] * J[3])
    xm = px >= py
    pmax, pmin = (px, py) if xm else (py, px)
    au, av = (J[0], J[1]) if xm else (J[2], J[3])
    if pmax == 0:
        return 1, f32(0), [(u, v)]
    with np.errstate(divide="ignore"):
        ratio = f32(pmax / pmin)
    n = max_aniso if ratio > max_aniso else int(np.ceil(ratio))
    f = f32(pmax / f32(n))
    pts = []
    for i in range(1, n + 1):
        t = f32(f32(i) / f32(n + 1)) - f32(0.5)
        pts.append((f32(u + f32(t * au)), f32(v + f32(t * av))))
    return n, f, pts


def test_composition_of_single_fetches():
    """The probes composed in Python from the pinned single-fetch oracle:
    Alg. 3's three fetches (with Alg. 2's reflection) at every probe, colour
    and normalization summed over all of them, then divided."""
    m = tiny_meshes()[1]
    lr = np.random.default_rng(10).integers(2, 7, m.E)
    M, P, _, _ = _setup(m, k=lr)
    q = uniform_queries(m.H, 300, 11)
    J = _jac(q.Q, 12)
    out, _, n = oracle.sample_aniso(M, P, q.h, q.u, q.v, J, max_aniso=8)
    for i in range(q.Q):
        N, f, pts = _probe_points(J[i], q.u[i], q.v[i], 8)
        assert n[i] == N
        Cs, Ws = np.zeros(4), 0.0
        h = int(q.h[i])
        for (pu, pv) in pts:
            pu, pv = float(pu), float(pv)
            for g, a, b in ((h, pu, pv), (m.next[h], pv, -pu), (m.prev[h], -pv, pu)):
                x, y = (a, b) if g > m.twin[g] else (1 - a, 1 - b)
                c, w = oracle.texture_fetch(P, int(m.edge[g]), x, y, float(f),
                                            filter=oracle.TRILINEAR)
                Cs += c
                Ws += w
        np.testing.assert_allclose(out[i], Cs / Ws, rtol=1e-12, atol=1e-15)


def test_axis_symmetries_and_constants():
    m = tiny_meshes()[3]
    M, P, _, _ = _setup(m, k=4)
    q = uniform_queries(m.H, 5000, 13)
    J = _jac(q.Q, 14)
    a, _, na = oracle.sample_aniso(M, P, q.h, q.u, q.v, J)
    # the screen axes swapped: same footprint
    b, _, nb = oracle.sample_aniso(M, P, q.h, q.u, q.v, J[:, [2, 3, 0, 1]].copy())
    np.testing.assert_array_equal(na, nb)
    np.testing.assert_allclose(a, b, rtol=0, atol=1e-15)
    # the major axis reversed: the probe set mirrors about (u, v)
    c, _, _ = oracle.sample_aniso(M, P, q.h, q.u, q.v, -J)
    np.testing.assert_allclose(a, c, rtol=1e-6, atol=1e-6)
    # a constant texture is returned for any footprint
    MC, PC, _, _ = _setup(m, k=4, texels=lambda lr, base, total: np.full((total, 4), 0.375))
    o, _, _ = oracle.sample_aniso(MC, PC, q.h, q.u, q.v, J)
    np.testing.assert_allclose(o, 0.375, rtol=1e-13)


def test_invalid_queries():
    m = tiny_meshes()[0]
    M, P, _, _ = _setup(m, k=2)
    h = np.array([0, -1, 1, 2, 3], np.int32)
    u = np.array([0.2, 0.2, np.nan, 0.2, 0.2], np.float32)
    J = np.full((5, 4), 1e-3, np.float32)
    J[3, 1] = np.inf
    J[4, 2] = np.nan
    out, errs, n = oracle.sample_aniso(M, P, h, u, u, J)
    assert errs == 4
    assert np.isfinite(out[0]).all() and np.isnan(out[1:]).all()
    np.testing.assert_array_equal(n[1:], 0)
