"""Pins for the FP64 oracle: each test checks it against something other than
itself -- the paper's Fig. 2 table and prose, closed forms, invariants the
method guarantees, library routines (scipy, torch conversions) and brute
force with an independent formulation of the filter.
"""
from fractions import Fraction

import numpy as np
import pytest
import scipy.ndimage as ndi

import oracle
from htexgen import pool as gpool
from htexgen.mesh import cube_mesh, halfedges_from_faces
from tests.fixtures import GOLDEN, load_fig2, tiny_meshes
from htexgen.queries import uniform_queries

RNG = np.random.default_rng(12345)


def _pool(mesh, log2res, has_mips=False, kind=0, seed=102, texels=None):
    base, total = gpool.layout(log2res, has_mips)
    if texels is None:
        T = gpool.fill_level0_host(kind, seed, log2res, base, total,
                                   mesh.boundary_edges(), has_mips).astype(np.float64)
    else:
        T = texels
    P = oracle.Pool(log2res, base, T, has_mips)
    if has_mips:
        P = oracle.Pool(log2res, base, oracle.build_mips(P), True)
    return P, base


def _level_view(P, e, l):
    k = int(P.log2res[e])
    off = sum(4 ** (k - m) for m in range(l))
    n = 1 << (k - l)
    s = int(P.base[e]) + off
    return P.texels[s:s + n * n].reshape(n, n, 4)


# ------------------------------------------------------------ Fig. 2 ------

def test_fig2_table_is_a_valid_halfedge_mesh():
    m = load_fig2()
    M = oracle.Mesh(m.twin, m.next, m.prev, m.edge, m.E, vert=m.vert)
    assert oracle.validate(M) == (0, -1)
    assert (m.H, m.E, m.F, m.V) == (12, 9, 3, 7)


def test_fig2_prose_navigation():
    m = load_fig2()
    ops = {"prev": m.prev, "next": m.next, "twin": m.twin, "edge": m.edge}
    n = 0
    with open(f"{GOLDEN}/fig2_navigation.txt") as fh:
        for line in fh:
            if not line.strip() or line.startswith("#"):
                continue
            op, h, val = line.split()
            h, val = int(h), int(val)
            if op == "facesize":
                assert np.count_nonzero(m.face == m.face[h]) == val
            else:
                assert ops[op][h] == val, line
            n += 1
    assert n == 10


def test_generator_reproduces_fig2_table():
    m = load_fig2()
    faces = [list(m.vert[m.face == f]) for f in range(m.F)]
    g = halfedges_from_faces(faces)
    for name in ("twin", "next", "prev", "vert", "face"):
        np.testing.assert_array_equal(getattr(g, name), getattr(m, name), err_msg=name)
    # same partition of halfedges into edges, up to relabelling
    pairs = {(a, b) for a, b in zip(g.edge, m.edge)}
    assert len(pairs) == m.E == g.E


def test_fig2_upper_right_halfedges():
    """Alg. 2: the larger halfedge of a pair (and every boundary halfedge)
    keeps (u, v); the smaller is reflected.  On Fig. 2 that reflects exactly
    h0, h1 and h5."""
    m = load_fig2()
    M = oracle.Mesh(m.twin, m.next, m.prev, m.edge, m.E)
    P, _ = _pool(m, np.full(m.E, 2, np.uint8))
    h = np.arange(12, dtype=np.int32)
    _, _, d = oracle.sample(M, P, h, np.full(12, 0.3, np.float32),
                            np.full(12, 0.3, np.float32), debug=True)
    assert set(np.nonzero(d["flip"][:, 0])[0]) == {0, 1, 5}
    np.testing.assert_array_equal(d["next"], m.next)
    np.testing.assert_array_equal(d["prev"], m.prev)
    np.testing.assert_array_equal(d["edge"][:, 0], m.edge)
    np.testing.assert_array_equal(d["edge"][:, 1], m.edge[m.next])
    np.testing.assert_array_equal(d["edge"][:, 2], m.edge[m.prev])


# ----------------------------------------------- the fetch vs a library ---

@pytest.mark.parametrize("k", [0, 1, 2, 3, 4])
def test_texture_fetch_matches_scipy_grid_constant(k):
    """One fetch = bilinear interpolation with texel centres at (i+1/2)/n and a
    zero border (CLAMP_TO_BORDER); its normalization channel = the same
    interpolation of an all-ones texture.  scipy's map_coordinates with
    order=1, mode='grid-constant' is that filter."""
    m = cube_mesh()
    log2res = np.full(m.E, k, np.uint8)
    P, base = _pool(m, log2res, kind=0)
    n = 1 << k
    for e in (0, 17, 101):
        T = _level_view(P, e, 0)
        xs = RNG.uniform(-0.7, 1.7, 40)
        ys = RNG.uniform(-0.7, 1.7, 40)
        # exact texel centres and borders too
        xs = np.concatenate([xs, (np.arange(n) + 0.5) / n, [0.0, 1.0, 0.5 / n]])
        ys = np.concatenate([ys, (np.arange(n)[::-1] + 0.5) / n, [1.0, 0.0, 1.0]])
        for x, y in zip(xs, ys):
            C, W = oracle.texture_fetch(P, e, x, y)
            coords = np.array([[y * n - 0.5], [x * n - 0.5]])
            for c in range(4):
                ref = ndi.map_coordinates(T[:, :, c], coords, order=1, mode="grid-constant",
                                          cval=0.0)[0]
                assert abs(C[c] - ref) <= 1e-12, (x, y, c)
            refW = ndi.map_coordinates(np.ones((n, n)), coords, order=1,
                                       mode="grid-constant", cval=0.0)[0]
            assert abs(W - refW) <= 1e-12


def test_trilinear_fetch_blends_scipy_levels():
    """LINEAR_MIPMAP_LINEAR: levels floor(lambda) and floor(lambda)+1 blended by
    the fraction of lambda = log2(f n0), lambda computed here with numpy's log2
    of the product (the oracle splits the exponent of f instead)."""
    m = cube_mesh()
    k = 4
    P, base = _pool(m, np.full(m.E, k, np.uint8), has_mips=True, kind=1)
    for _ in range(60):
        e = int(RNG.integers(0, m.E))
        lam = RNG.uniform(-1.5, k + 1.5)
        f = float(np.float32(2.0 ** lam / (1 << k)))
        lam = np.log2(np.float64(f) * (1 << k))
        x, y = RNG.uniform(-0.3, 1.3, 2)

        def interp(l):
            T = _level_view(P, e, l)
            n = T.shape[0]
            co = np.array([[y * n - 0.5], [x * n - 0.5]])
            col = [ndi.map_coordinates(T[:, :, c], co, order=1, mode="grid-constant")[0]
                   for c in range(4)]
            w = ndi.map_coordinates(np.ones((n, n)), co, order=1, mode="grid-constant")[0]
            return np.array(col), w

        if lam <= 0:
            refC, refW = interp(0)
        elif lam >= k:
            refC, refW = interp(k)
        else:
            l0 = int(np.floor(lam))
            fr = lam - l0
            c0, w0 = interp(l0)
            c1, w1 = interp(l0 + 1)
            refC, refW = (1 - fr) * c0 + fr * c1, (1 - fr) * w0 + fr * w1
        C, W = oracle.texture_fetch(P, e, x, y, f=f, filter=oracle.TRILINEAR)
        np.testing.assert_allclose(C, refC, rtol=0, atol=1e-12)
        assert abs(W - refW) < 1e-12


# --------------------------------------------------- closed forms -------

def _interior_queries(m, n_min, count, rng):
    """Queries whose every filter tap of the own fetch is inside the quad and
    whose neighbour fetches read only the zero border (u, v > 1/(2 n_min))."""
    lo = 0.5 / n_min + 1e-3
    h = rng.integers(0, m.H, count).astype(np.int32)
    u = rng.uniform(lo, 1 - 2 * lo, count)
    v = rng.uniform(lo, 1 - lo - u)
    return h, u.astype(np.float32), v.astype(np.float32)


@pytest.mark.parametrize("mesh_i", [0, 1, 2, 3])
def test_linear_ramp_reproduces_quad_coordinates(mesh_i):
    """Bilinear filtering reproduces bilinear functions exactly.  With texel
    (i, j) holding (x_i, y_j, 1, x_i y_j) at its centre x_i = (i+1/2)/n, an
    interior query returns (x, y, 1, x y) for the quad point of Alg. 2:
    (u, v) for the larger halfedge of a pair or a boundary halfedge, else
    (1-u, 1-v) (the larger halfedge takes the lower-left half, Section 4.2).
    This pins the reflection rule, its direction, the texel centre convention
    and the axis order (x indexes columns)."""
    m = tiny_meshes()[mesh_i]
    k = 4
    n = 1 << k
    log2res = np.full(m.E, k, np.uint8)
    base, total = gpool.layout(log2res, False)
    T = np.zeros((total, 4))
    xc = (np.arange(n) + 0.5) / n
    ramp = np.stack(np.broadcast_arrays(xc[None, :], xc[:, None], 1.0,
                                        xc[None, :] * xc[:, None]), -1).reshape(-1, 4)
    for e in range(m.E):
        T[base[e]:base[e] + n * n] = ramp
    P = oracle.Pool(log2res, base, T, False)
    M = oracle.Mesh.of(m)
    h, u, v = _interior_queries(m, n, 300, np.random.default_rng(mesh_i))
    out, errs, _ = oracle.sample(M, P, h, u, v)
    assert errs == 0
    keep = h > m.twin[h]
    x = np.where(keep, u.astype(np.float64), 1 - u.astype(np.float64))
    y = np.where(keep, v.astype(np.float64), 1 - v.astype(np.float64))
    ref = np.stack([x, y, np.ones_like(x), x * y], -1)
    np.testing.assert_allclose(out, ref, rtol=0, atol=1e-14)


def test_texel_centre_returns_texel():
    """A query whose quad point is an interior texel centre returns that texel
    (all bilinear weight on one tap, W = 1)."""
    m = cube_mesh()
    k = 3
    n = 1 << k
    P, base = _pool(m, np.full(m.E, k, np.uint8))
    M = oracle.Mesh.of(m)
    for h in range(0, m.H, 7):
        keep = h > m.twin[h]
        for i, j in ((1, 1), (2, 4), (5, 1), (3, 3), (1, 5)):
            x, y = (i + 0.5) / n, (j + 0.5) / n      # quad point, lower-left half
            if not keep:
                x, y = 1 - x, 1 - y                  # upper-right half for the twin
                i, j = n - 1 - i, n - 1 - j
            u, v = (x, y) if keep else (1 - x, 1 - y)
            out, _, _ = oracle.sample(M, P, [h], [u], [v])
            np.testing.assert_array_equal(out[0], _level_view(P, m.edge[h], 0)[j, i])


@pytest.mark.parametrize("mixed", [False, True])
def test_constant_texture_reproduces_constant_and_weight_bounds(mixed):
    """Normalization (c_i / c_n of Alg. 3): any constant pool returns the
    constant; the normalization weight W is in [1/2, 1] when every texture has
    the same resolution and at least 1/4 otherwise."""
    for m in tiny_meshes():
        rng = np.random.default_rng(m.H)
        log2res = (rng.integers(0, 6, m.E) if mixed else np.full(m.E, 4)).astype(np.uint8)
        base, total = gpool.layout(log2res, True)
        T = np.full((total, 4), 0.0)
        T[:] = [0.25, 0.5, 0.75, 1.0]
        P = oracle.Pool(log2res, base, T, True)
        M = oracle.Mesh.of(m)
        q = uniform_queries(m.H, 4000, 7, log2f=(-8, 1))
        for filt in (oracle.BILINEAR, oracle.TRILINEAR):
            out, errs, d = oracle.sample(M, P, q.h, q.u, q.v, q.f, filter=filt, debug=True)
            assert errs == 0
            np.testing.assert_allclose(out, np.broadcast_to([0.25, 0.5, 0.75, 1.0], out.shape),
                                       rtol=1e-14)
            np.testing.assert_allclose(d["W"], d["wf"].sum(1), rtol=1e-15)
            assert d["W"].min() >= (0.25 if mixed else 0.5) - 1e-12
            if not mixed:
                assert d["W"].max() <= 1 + 1e-12


def test_lod_closed_form():
    """Texels of level l all equal to l: an interior query with footprint f
    returns clamp(lambda, 0, k) with lambda = log2(f 2^k) (trilinear blending of
    the two levels around lambda), and the debug levels equal
    clamp(floor(lambda), 0, k)."""
    m = cube_mesh()
    k = 4
    log2res = np.full(m.E, k, np.uint8)
    base, total = gpool.layout(log2res, True)
    T = np.zeros((total, 4))
    for e in range(m.E):
        off = base[e]
        for l in range(k + 1):
            nn = 1 << (k - l)
            T[off:off + nn * nn] = l
            off += nn * nn
    P = oracle.Pool(log2res, base, T, True)
    M = oracle.Mesh.of(m)
    rng = np.random.default_rng(5)
    h, u, v = _interior_queries(m, 2, 2000, rng)
    lam_t = rng.uniform(-1.5, k - 1 - 1e-3, len(h))
    f = (2.0 ** lam_t / (1 << k)).astype(np.float32)
    lam = np.log2(f.astype(np.float64) * (1 << k))
    out, _, d = oracle.sample(M, P, h, u, v, f, filter=oracle.TRILINEAR, debug=True)
    np.testing.assert_allclose(out[:, 0], np.clip(lam, 0, k), rtol=0, atol=1e-12)
    np.testing.assert_array_equal(d["level"][:, 0, 0], np.clip(np.floor(lam), 0, k))
    # bilinear ignores the footprint
    outb, _, _ = oracle.sample(M, P, h, u, v, f, filter=oracle.BILINEAR)
    np.testing.assert_array_equal(outb[:, 0], 0.0)


def test_special_footprints():
    m = cube_mesh()
    k = 3
    log2res = np.full(m.E, k, np.uint8)
    P, base = _pool(m, log2res, has_mips=True, kind=1)
    M = oracle.Mesh.of(m)
    h = np.array([5, 5, 5, 5, 5], np.int32)
    u = np.full(5, 0.3, np.float32)
    v = np.full(5, 0.3, np.float32)
    f = np.array([0.0, -1.0, np.nan, np.inf, 1e-42], np.float32)
    _, _, d = oracle.sample(M, P, h, u, v, f, filter=oracle.TRILINEAR, debug=True)
    np.testing.assert_array_equal(d["level"][:, 0, 0], [0, 0, 0, k, 0])
    np.testing.assert_array_equal(d["level"][:, 0, 1], [-1] * 5)


# --------------------------------------------------- brute force --------

def _brute(m, log2res, base, T, h, u, v):
    """Independent formulation: the bilinear filter as a tent kernel
    max(0, 1-|s-i|) max(0, 1-|t-j|) summed over every texel of the texture
    (zero outside), for the three fetches of Alg. 3."""
    out = np.zeros((len(h), 4))
    for q in range(len(h)):
        hq, uq, vq = int(h[q]), float(u[q]), float(v[q])
        num = np.zeros(4)
        den = 0.0
        for g, a, b in ((hq, uq, vq), (int(m.next[hq]), vq, -uq), (int(m.prev[hq]), -vq, uq)):
            x, y = (a, b) if g > m.twin[g] else (1 - a, 1 - b)
            e = int(m.edge[g])
            n = 1 << int(log2res[e])
            idx = np.arange(n)
            wx = np.maximum(0.0, 1 - np.abs(x * n - 0.5 - idx))
            wy = np.maximum(0.0, 1 - np.abs(y * n - 0.5 - idx))
            w = wy[:, None] * wx[None, :]
            tex = T[base[e]:base[e] + n * n].reshape(n, n, 4)
            num += (w[:, :, None] * tex).sum((0, 1))
            den += w.sum()
        with np.errstate(invalid="ignore"):   # 0 / 0 off every texture: NaN, as the oracle
            out[q] = num / den
    return out


@pytest.mark.parametrize("mesh_i", [0, 1, 2, 3])
def test_brute_force_tent_filter(mesh_i):
    m = tiny_meshes()[mesh_i]
    rng = np.random.default_rng(100 + mesh_i)
    log2res = rng.integers(0, 4, m.E).astype(np.uint8)
    P, base = _pool(m, log2res, kind=0, seed=9)
    M = oracle.Mesh.of(m)
    q = uniform_queries(m.H, 400, 11 + mesh_i)
    # plus points slightly outside the triangle and exactly on its legs
    h = np.concatenate([q.h, rng.integers(0, m.H, 40)]).astype(np.int32)
    u = np.concatenate([q.u, rng.uniform(-0.2, 1.1, 30), np.zeros(10)]).astype(np.float32)
    v = np.concatenate([q.v, rng.uniform(-0.2, 1.1, 30), rng.uniform(0, 1, 10)]).astype(np.float32)
    out, errs, _ = oracle.sample(M, P, h, u, v)
    ref = _brute(m, log2res, base, P.texels, h, u, v)
    fin = np.isfinite(ref[:, 0])
    np.testing.assert_allclose(out[fin], ref[fin], rtol=1e-12, atol=1e-14)
    assert np.isnan(out[~fin]).all()


# --------------------------------------------------- seams --------------

def _uniform_res_setup(m, k=4, mips=False, kind=0):
    log2res = np.full(m.E, k, np.uint8)
    P, base = _pool(m, log2res, has_mips=mips, kind=kind)
    return oracle.Mesh.of(m), P


@pytest.mark.parametrize("mesh_i", [0, 1, 3])
def test_twin_diagonal_seam_bit_identical(mesh_i):
    """A point on the mesh edge, sampled from either triangle of its quad,
    gives the same value (Section 3.2: the halfedge/twin pair forms one quad),
    bit for bit, at least half a texel from the quad corners."""
    m = tiny_meshes()[mesh_i]
    M, P = _uniform_res_setup(m)
    n = 16
    hs = np.nonzero(m.twin >= 0)[0]
    for h in hs:
        mm = np.arange(2, 63)
        uu = (mm / 64.0).astype(np.float32)
        a, _, _ = oracle.sample(M, P, np.full(len(uu), h, np.int32), uu, 1 - uu)
        b, _, _ = oracle.sample(M, P, np.full(len(uu), m.twin[h], np.int32), 1 - uu, uu)
        np.testing.assert_array_equal(a, b)
    assert n == 16


@pytest.mark.parametrize("mesh_i", [0, 1, 2, 3])
@pytest.mark.parametrize("eps", [0.0, 1.0 / 128, 1.0 / 37])
def test_next_prev_seams_bit_identical(mesh_i, eps):
    """Alg. 3 unfolds the Next triangle with (v, -u) and the Prev triangle with
    (-v, u).  So (h, -eps, v) and (Next h, v, eps) name the same surface point
    and read the same two non-empty fetches; likewise (h, u, -eps) and
    (Prev h, eps, u).  At least half a texel from the shared corner the third
    fetch is empty on both sides and the results agree bit for bit."""
    m = tiny_meshes()[mesh_i]
    M, P = _uniform_res_setup(m, k=4)
    t = (np.arange(9, 60) / 64.0).astype(np.float32)   # t * 16 >= 1/2 + margin
    e = np.float32(eps)
    for h in range(m.H):
        hh = np.full(len(t), h, np.int32)
        a, _, _ = oracle.sample(M, P, hh, np.full(len(t), -e, np.float32), t)
        b, _, _ = oracle.sample(M, P, np.full(len(t), m.next[h], np.int32), t,
                                np.full(len(t), e, np.float32))
        np.testing.assert_array_equal(a, b)
        c, _, _ = oracle.sample(M, P, hh, t, np.full(len(t), -e, np.float32))
        d, _, _ = oracle.sample(M, P, np.full(len(t), m.prev[h], np.int32),
                                np.full(len(t), e, np.float32), t)
        np.testing.assert_array_equal(c, d)


def test_seam_test_catches_wrong_neighbour_map():
    """The seam test above fails for a plausible mistake: fetching the Next
    quad at (-u, v) instead of (v, -u) (simulated by sampling the point the
    wrong map would read)."""
    m = cube_mesh()
    M, P = _uniform_res_setup(m, k=4)
    t = (np.arange(9, 60) / 64.0).astype(np.float32)
    h = 10
    a, _, _ = oracle.sample(M, P, np.full(len(t), m.next[h], np.int32), t,
                            np.zeros(len(t), np.float32))
    wrong, _, _ = oracle.sample(M, P, np.full(len(t), m.next[h], np.int32),
                                np.zeros(len(t), np.float32), t)
    assert not np.array_equal(a, wrong)


def test_renumbering_invariance():
    """The orientation rule is consistent: relabelling the halfedges with a
    random permutation, and point-reflecting (x, y) -> (1-x, 1-y) the texture of
    every edge whose larger halfedge changed, leaves every result unchanged."""
    m = cube_mesh()
    k = 3
    M, P = _uniform_res_setup(m, k=k, mips=True, kind=1)
    rng = np.random.default_rng(3)
    pi = rng.permutation(m.H).astype(np.int32)
    inv = np.argsort(pi)
    tw = np.where(m.twin[inv] >= 0, pi[np.maximum(m.twin[inv], 0)], -1).astype(np.int32)
    nx = pi[m.next[inv]]
    pv = pi[m.prev[inv]]
    ed = m.edge[inv]
    M2 = oracle.Mesh(tw, nx, pv, ed, m.E)
    T2 = P.texels.copy()
    for e in range(m.E):
        hs = np.nonzero(m.edge == e)[0]
        if len(hs) < 2:
            continue
        old_large = hs.max()
        new_large = inv[pi[hs].max()]
        if old_large != new_large:
            for l in range(k + 1):
                V = _level_view(P, e, l)
                nn = V.shape[0]
                off = int(P.base[e]) + sum(4 ** (k - mm) for mm in range(l))
                T2[off:off + nn * nn] = V[::-1, ::-1].reshape(-1, 4)
    P2 = oracle.Pool(P.log2res, P.base, T2, True)
    q = uniform_queries(m.H, 3000, 21, log2f=(-6, 0))
    a, _, _ = oracle.sample(M, P, q.h, q.u, q.v, q.f, filter=oracle.TRILINEAR)
    b, _, _ = oracle.sample(M2, P2, pi[q.h], q.u, q.v, q.f, filter=oracle.TRILINEAR)
    np.testing.assert_allclose(a, b, rtol=1e-13, atol=1e-15)


# ------------------------------------------- exact integer tap bases ----

def _adversarial_coords(n):
    vals = []
    for m_ in range(0, n + 1):
        for off in (Fraction(1, 2), Fraction(0), Fraction(1)):
            c = (m_ + off) / n
            f = np.float32(float(c))
            for d in range(-3, 4):
                vals.append(np.nextafter(f, np.float32(2), dtype=np.float32) if d > 0 else f)
                f2 = f
                for _ in range(abs(d)):
                    f2 = np.nextafter(f2, np.float32(2 if d > 0 else -2), dtype=np.float32)
                vals.append(f2)
    vals += [np.float32(0.0), np.float32(-0.0), np.float32(1e-40), np.float32(2 ** -30),
             np.nextafter(np.float32(1), np.float32(0))]
    return np.array([v for v in vals if 0 <= v <= 1], dtype=np.float32)


@pytest.mark.parametrize("k", [0, 2, 4, 6])
def test_tap_bases_exact_against_rationals(k):
    """The debug tap bases i0 = floor(x n - 1/2), j0 = floor(y n - 1/2) are
    exact (checked with rational arithmetic) on coordinates a few ulps around
    every texel centre and texel edge, for all three fetches (their
    coordinates are u, v, -u, -v, 1-u, 1-v, 1+u, 1+v)."""
    m = cube_mesh()
    M, P = _uniform_res_setup(m, k=k)
    n = 1 << k
    cs = _adversarial_coords(n)
    rng = np.random.default_rng(k)
    u = rng.permutation(cs)
    v = rng.permutation(cs)
    h = rng.integers(0, m.H, len(u)).astype(np.int32)
    _, _, d = oracle.sample(M, P, h, u, v, debug=True)
    for q in range(len(h)):
        hq = int(h[q])
        U, V = Fraction(float(u[q])), Fraction(float(v[q]))
        for s, (g, a, b) in enumerate(((hq, U, V), (int(m.next[hq]), V, -U),
                                       (int(m.prev[hq]), -V, U))):
            x, y = (a, b) if g > m.twin[g] else (1 - a, 1 - b)
            i0 = (x * n - Fraction(1, 2)).__floor__()
            j0 = (y * n - Fraction(1, 2)).__floor__()
            assert d["i0"][q, s, 0] == i0 and d["j0"][q, s, 0] == j0, (q, s)


# --------------------------------------------------- backward -----------

@pytest.mark.parametrize("filt", [oracle.BILINEAR, oracle.TRILINEAR])
def test_backward_finite_differences_and_adjoint(filt):
    """The output is linear in the texels, so central differences in FP64 are
    exact up to rounding, and <g, J dT> = <J^T g, dT> for any dT."""
    m = cube_mesh(n=2, seed=7, n_split=3, n_merge=1)
    rng = np.random.default_rng(8)
    log2res = rng.integers(1, 4, m.E).astype(np.uint8)
    mips = filt == oracle.TRILINEAR
    P, base = _pool(m, log2res, has_mips=mips, kind=0)
    M = oracle.Mesh.of(m)
    q = uniform_queries(m.H, 600, 4, log2f=(-5, 0))
    g = rng.standard_normal((q.Q, 4))
    grad = oracle.backward(M, P, q.h, q.u, q.v, g, q.f, filter=filt)
    total = P.texels.shape[0]
    for _ in range(40):
        t = int(rng.integers(0, total))
        c = int(rng.integers(0, 4))
        eps = 1e-3
        Tp = P.texels.copy()
        Tm = P.texels.copy()
        Tp[t, c] += eps
        Tm[t, c] -= eps
        op, _, _ = oracle.sample(M, oracle.Pool(log2res, base, Tp, mips), q.h, q.u, q.v, q.f,
                                 filter=filt)
        om, _, _ = oracle.sample(M, oracle.Pool(log2res, base, Tm, mips), q.h, q.u, q.v, q.f,
                                 filter=filt)
        fd = ((op - om) * g).sum() / (2 * eps)
        assert abs(fd - grad[t, c]) <= 1e-9 * max(1.0, abs(fd)), (t, c)
    dT = rng.standard_normal(P.texels.shape)
    Jd, _, _ = oracle.sample(M, oracle.Pool(log2res, base, dT, mips), q.h, q.u, q.v, q.f,
                             filter=filt)
    # J dT is the forward map applied to dT (the output is linear in T)
    lhs = (g * Jd).sum()
    rhs = (grad * dT).sum()
    assert abs(lhs - rhs) <= 1e-10 * abs(lhs)


# --------------------------------------------------- mips ---------------

def test_mips_box_filter_matches_numpy_block_mean():
    m = cube_mesh()
    rng = np.random.default_rng(2)
    log2res = rng.integers(0, 6, m.E).astype(np.uint8)
    P, base = _pool(m, log2res, has_mips=True, kind=0)
    for e in range(0, m.E, 13):
        k = int(log2res[e])
        for l in range(1, k + 1):
            fine = _level_view(P, e, l - 1)
            nn = fine.shape[0] // 2
            ref = fine.reshape(nn, 2, nn, 2, 4).mean(axis=(1, 3))
            np.testing.assert_allclose(_level_view(P, e, l), ref, rtol=1e-15)
        # total mass is preserved level to level (x 1/4 per level)
        s0 = _level_view(P, e, 0).sum((0, 1))
        np.testing.assert_allclose(_level_view(P, e, k)[0, 0] * 4 ** k, s0, rtol=1e-13)


def test_boundary_mirror_is_preserved_by_mips():
    """Boundary edges carry mirrored content (Section 4.3): the upper-right
    half reflects the lower-left across x + y = 1; the box filter keeps that
    symmetry at every level."""
    m = tiny_meshes()[3]
    k = 4
    P, base = _pool(m, np.full(m.E, k, np.uint8), has_mips=True, kind=1)
    bnd = np.nonzero(m.boundary_edges())[0]
    assert len(bnd) > 0
    for e in bnd:
        for l in range(k + 1):
            V = _level_view(P, e, l)
            np.testing.assert_allclose(V, V.transpose(1, 0, 2)[::-1, ::-1], rtol=1e-15)


# --------------------------------------------------- quantization -------

def test_bf16_rounding_matches_torch():
    torch = pytest.importorskip("torch")
    x = np.concatenate([
        RNG.standard_normal(20000).astype(np.float32) * 10,
        RNG.random(5000).astype(np.float32),
        np.array([0.0, -0.0, np.inf, -np.inf, 3.3895314e38, 1e-40, 1.00390625, 1.01171875,
                  1.0078125, -1.00390625], np.float32),
    ])
    # exact ties: low 16 bits = 0x8000
    ties = (RNG.integers(0, 2 ** 15, 2000).astype(np.uint32) << 16 | 0x8000).view(np.float32)
    x = np.concatenate([x, ties[np.isfinite(ties)]])
    ours = oracle.f32_to_bf16(x)
    ref = torch.from_numpy(x).to(torch.bfloat16).view(torch.int16).numpy().view(np.uint16)
    np.testing.assert_array_equal(ours, ref)
    back = oracle.bf16_to_f64(ours)
    np.testing.assert_array_equal(back.astype(np.float32),
                                  torch.from_numpy(ref.view(np.int16)).view(torch.bfloat16)
                                  .float().numpy())


def test_e4m3_table_and_rounding_match_torch():
    torch = pytest.importorskip("torch")
    tab = oracle.e4m3_table()
    ref = torch.arange(256, dtype=torch.uint8).view(torch.float8_e4m3fn).float().numpy()
    np.testing.assert_array_equal(np.isnan(tab), np.isnan(ref))
    ok = ~np.isnan(ref)
    np.testing.assert_array_equal(tab[ok], ref[ok])
    assert np.nanmax(tab) == 448.0
    # rounding of in-range values, including every midpoint between codes
    fin = np.unique(np.abs(tab[ok]))
    mids = (fin[1:] + fin[:-1]) / 2
    x = np.concatenate([RNG.uniform(-448, 448, 20000), mids, -mids, fin, -fin,
                        RNG.uniform(-2 ** -6, 2 ** -6, 2000)]).astype(np.float32)
    ours = oracle.f64_to_e4m3(x.astype(np.float64))
    theirs = torch.from_numpy(x).to(torch.float8_e4m3fn).view(torch.uint8).numpy()
    np.testing.assert_array_equal(ours, theirs)
    # saturation beyond the largest finite value
    big = np.array([449.0, 464.0, 500.0, 1e30, -1e9])
    np.testing.assert_array_equal(oracle.f64_to_e4m3(big), [0x7e, 0x7e, 0x7e, 0x7e, 0xfe])


def test_quantized_relative_error_bounds():
    """Round-to-nearest relative error of a normal value is at most
    2^-p / (1 + 2^-p) with p = 8 for bfloat16 and 4 for E4M3."""
    x = RNG.uniform(0.01, 1.0, 50000).astype(np.float32)
    b = oracle.bf16_to_f64(oracle.f32_to_bf16(x))
    assert (np.abs(b - x) / x).max() <= 2 ** -8 / (1 + 2 ** -8)
    m = cube_mesh()
    log2res = np.full(m.E, 3, np.uint8)
    base, total = gpool.layout(log2res, False)
    T = gpool.fill_level0_host(1, 5, log2res, base, total, m.boundary_edges(), False)
    codes, scale = oracle.quantize_e4m3(log2res, base, False, T)
    D = oracle.e4m3_pool_to_f64(log2res, base, False, codes, scale)
    used = np.zeros(total, bool)
    for e in range(m.E):
        used[base[e]:base[e] + 64] = True
        mx = np.abs(T[base[e]:base[e] + 64]).max()
        assert scale[e] == np.float32(mx) / np.float32(448.0)
    t = T[used].astype(np.float64)
    d = D[used]
    normal = t / np.repeat(scale, 64)[:, None] >= 2 ** -6
    assert (np.abs(d - t) / t)[normal].max() <= 2 ** -4 / (1 + 2 ** -4) + 1e-7


# --------------------------------------------------- mesh validation ----

def test_generated_meshes_validate():
    for m in tiny_meshes():
        M = oracle.Mesh(m.twin, m.next, m.prev, m.edge, m.E, vert=m.vert)
        assert oracle.validate(M)[0] == 0


@pytest.mark.parametrize("plant", ["twin", "next", "edge", "vert", "range", "dup_edge"])
def test_validation_catches_planted_mistakes(plant):
    m = cube_mesh()
    tw, nx, pv, ed, vt = (m.twin.copy(), m.next.copy(), m.prev.copy(), m.edge.copy(),
                          m.vert.copy())
    if plant == "twin":
        tw[5] = tw[6]
    elif plant == "next":
        nx[3], nx[4] = nx[4], nx[3]
    elif plant == "edge":
        ed[7] = (ed[7] + 1) % m.E
    elif plant == "vert":
        vt[m.twin[9]] = (vt[m.twin[9]] + 1) % m.V
    elif plant == "range":
        pv[0] = m.H
    elif plant == "dup_edge":
        ed[ed == 3] = 4
    rc, bad = oracle.validate(oracle.Mesh(tw, nx, pv, ed, m.E, vert=vt))
    assert rc != 0


def test_invalid_queries_give_nan_and_count():
    m = cube_mesh()
    M, P = _uniform_res_setup(m, k=2)
    h = np.array([0, -1, m.H, 3, 4], np.int32)
    u = np.array([0.2, 0.2, 0.2, np.nan, 0.1], np.float32)
    v = np.array([0.2, 0.2, 0.2, 0.1, np.inf], np.float32)
    out, errs, _ = oracle.sample(M, P, h, u, v)
    assert errs == 4
    assert np.isfinite(out[0]).all() and np.isnan(out[1:]).all()


def test_backward_fd_config4_shape():
    """Config 4's shape: the tiny cube, 32x32 RGBA float32 textures, N(0,1)
    upstream gradients; FP64 central differences on 512 sampled texel
    channels (restricted to the queries that can touch each texel, which is
    exact for a linear map) agree with the oracle gradient."""
    m = cube_mesh()
    lr = np.full(m.E, 5, np.uint8)
    P, base = _pool(m, lr, kind=1, seed=401)
    M = oracle.Mesh.of(m)
    q = uniform_queries(m.H, 40000, 405, sort=True)
    g = np.random.default_rng(403).standard_normal((q.Q, 4))
    grad = oracle.backward(M, P, q.h, q.u, q.v, g)
    rng = np.random.default_rng(404)
    n = 32 * 32
    for _ in range(512):
        e = int(rng.integers(0, m.E))
        t = int(base[e] + rng.integers(0, n))
        c = int(rng.integers(0, 4))
        near = np.isin(m.edge[q.h], [e]) | np.isin(m.edge[m.next[q.h]], [e]) | \
            np.isin(m.edge[m.prev[q.h]], [e])
        sel = np.nonzero(near)[0]
        eps = 1e-3
        Tp, Tm = P.texels.copy(), P.texels.copy()
        Tp[t, c] += eps
        Tm[t, c] -= eps
        op, _, _ = oracle.sample(M, oracle.Pool(lr, base, Tp, False), q.h[sel], q.u[sel], q.v[sel])
        om, _, _ = oracle.sample(M, oracle.Pool(lr, base, Tm, False), q.h[sel], q.u[sel], q.v[sel])
        fd = ((op - om) * g[sel]).sum() / (2 * eps)
        assert abs(fd - grad[t, c]) <= 1e-9 * max(1.0, abs(fd))
