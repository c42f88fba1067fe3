"""Seeded texel values for per-edge square textures (level 0 only).

Input generator only: every value is a pure function of
(seed, edge, row j, column i, channel c) built from the splitmix64 mixing
function (Steele, Lea and Flood, "Fast splittable pseudorandom number
generators", OOPSLA 2014), so a device fill kernel can produce the same bits
independently.  Mip levels are not generated here.

Three fills:

* ``uniform``: each texel channel is an independent 24-bit uniform value in
  [0, 1): ``(hash >> 40) * 2^-24`` (exact in float32).
* ``smooth``: value noise on a lattice of 8-texel cells.  Each lattice point
  carries an integer value in [1, 63]; a texel blends its cell's four corner
  values with the integer smooth ramp R[f] (R[f] + R[7-f] = 64), giving an
  integer numerator below 2^18 that is scaled by 2^-18 (exact in float32).
  Values lie in [1/64, 63/64].
* ``perlin``: Perlin gradient noise (K. Perlin, "Improving Noise",
  SIGGRAPH 2002) in the plane of each edge's texture, per channel, on a
  lattice of 8-texel cells: every lattice point carries a gradient picked by
  hash from the eight directions (+-1, 0), (0, +-1), (+-1, +-1); a texel
  centre at offset (x, y) in its cell (x, y in sixteenths of a cell, odd)
  takes the dot products of the four corner gradients with its offsets from
  the corners, blended with Perlin's quintic fade 6t^5 - 15t^4 + 10t^3.  At
  t = m/16 the fade is F(m) / 2^20 with the integer F(m) = 6m^5 - 240m^4 +
  2560m^3, so the noise is an exact integer N / 2^44 (|noise| < 1).  It is
  rounded down to 2^-18 steps, M = floor(N / 2^26) + 2^18 in [0, 2^19], and
  the texel is (2^18 + 31 M) 2^-24 = 1/64 + (62/64)(1/2 + noise/2): values
  in [1/64, 63/64], exact in float32.

Boundary edges carry mirrored content (paper Section 4.3, "Texture Data"):
the upper-right half of the quad (texel centres with i + j > n - 1) belongs
to the virtual twin and repeats the lower-left half reflected across the
diagonal x + y = 1, i.e. T[j][i] = T[n-1-i][n-1-j].
"""
from __future__ import annotations

import numpy as np

M64 = np.uint64(0xFFFFFFFFFFFFFFFF)
GOLDEN = np.uint64(0x9E3779B97F4A7C15)
MIX1 = np.uint64(0xBF58476D1CE4E5B9)
MIX2 = np.uint64(0x94D049BB133111EB)

UNIFORM = 0
SMOOTH = 1
PERLIN = 2

# integer smooth ramp over the 8 texel centres of a lattice cell
RAMP = np.array([1, 6, 14, 25, 39, 50, 58, 63], dtype=np.int64)

# Perlin's quintic fade at the 8 texel centres of a cell, t = (2f + 1) / 16:
# 2^20 fade(t) = 6m^5 - 240m^4 + 2560m^3 with m = 2f + 1
FADE_M = np.arange(1, 16, 2, dtype=np.int64)
FADE = 6 * FADE_M ** 5 - 240 * FADE_M ** 4 + 2560 * FADE_M ** 3
# the eight lattice gradients
GRAD = np.array([[1, 0], [-1, 0], [0, 1], [0, -1], [1, 1], [-1, 1], [1, -1], [-1, -1]],
                dtype=np.int64)


def splitmix64(z):
    z = np.asarray(z, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = z + GOLDEN
        z = (z ^ (z >> np.uint64(30))) * MIX1
        z = (z ^ (z >> np.uint64(27))) * MIX2
    return z ^ (z >> np.uint64(31))


def hash5(seed, a, b, c, d):
    """64-bit hash of five non-negative integers (broadcasting)."""
    x = splitmix64(np.uint64(seed))
    for k in (a, b, c, d):
        x = splitmix64(x ^ np.asarray(k, dtype=np.int64).astype(np.uint64))
    return x


def _mirror_src(i, j, n, boundary):
    """Source texel for mirrored boundary content."""
    m = boundary & ((i + j) > (n - 1))
    si = np.where(m, n - 1 - j, i)
    sj = np.where(m, n - 1 - i, j)
    return si, sj


def texel_values(kind: int, seed: int, e, n, boundary, i, j, c) -> np.ndarray:
    """float32 texel values for broadcast arrays of (edge, res, boundary, i, j, c).

    `n` is the level-0 resolution of edge `e` (a power of two), `boundary`
    whether the edge is a lone boundary halfedge.
    """
    e = np.asarray(e, dtype=np.int64)
    n = np.asarray(n, dtype=np.int64)
    i = np.asarray(i, dtype=np.int64)
    j = np.asarray(j, dtype=np.int64)
    c = np.asarray(c, dtype=np.int64)
    boundary = np.asarray(boundary, dtype=bool)
    si, sj = _mirror_src(i, j, n, boundary)
    if kind == UNIFORM:
        hv = hash5(seed, e, sj * n + si, c, 0)
        return ((hv >> np.uint64(40)).astype(np.int64).astype(np.float32)
                * np.float32(2.0 ** -24))
    if kind == PERLIN:
        return _perlin(seed, e, c, si, sj)
    if kind != SMOOTH:
        raise ValueError("unknown texel fill")
    a, fa = si >> 3, si & 7
    b, fb = sj >> 3, sj & 7
    rx1 = RAMP[fa]
    rx0 = 64 - rx1
    ry1 = RAMP[fb]
    ry0 = 64 - ry1
    # hash each lattice point once per (edge, channel), then gather
    shape = np.broadcast(e, c, a, b).shape
    eb, cb, ab, bb = (np.broadcast_to(x, shape) for x in (e, c, a, b))
    ue, einv = np.unique(eb.reshape(-1), return_inverse=True)
    nl = int(ab.max()) + 2 if ab.size else 2
    ci = np.arange(4)[None, :, None, None]
    la = np.arange(nl)[None, None, :, None]
    lb = np.arange(nl)[None, None, None, :]
    table = (hash5(seed, ue[:, None, None, None], ci, la, lb) % np.uint64(63)).astype(np.int64) + 1
    ei = einv.reshape(shape)

    def lat(aa, bb_):
        return table[ei, cb, aa, bb_]

    num = (rx0 * ry0 * lat(ab, bb) + rx1 * ry0 * lat(ab + 1, bb)
           + rx0 * ry1 * lat(ab, bb + 1) + rx1 * ry1 * lat(ab + 1, bb + 1))
    return num.astype(np.float32) * np.float32(2.0 ** -18)


def _perlin(seed, e, c, si, sj):
    """Perlin gradient noise texels (integer arithmetic, see the module
    docstring)."""
    a, fa = si >> 3, si & 7
    b, fb = sj >> 3, sj & 7
    x = 2 * fa + 1             # offsets from the cell's lower corner, in 1/16
    y = 2 * fb + 1
    wx1, wy1 = FADE[fa], FADE[fb]
    wx0, wy0 = (1 << 20) - wx1, (1 << 20) - wy1

    def corner(da, db):
        g = GRAD[(hash5(seed, e, c, a + da, b + db) & np.uint64(7)).astype(np.int64)]
        return g[..., 0] * (x - 16 * da) + g[..., 1] * (y - 16 * db)

    N = (wx0 * wy0 * corner(0, 0) + wx1 * wy0 * corner(1, 0)
         + wx0 * wy1 * corner(0, 1) + wx1 * wy1 * corner(1, 1))
    M = (N >> 26) + (1 << 18)                 # floor(N / 2^26) + 2^18
    M = np.clip(M, 0, 1 << 19)
    return (((1 << 18) + 31 * M).astype(np.float32) * np.float32(2.0 ** -24))


def perlin_reference(seed, e, c, si, sj):
    """The same noise in float64 from Perlin's formula (fade and dot
    products in floating point), before the 2^-18 rounding: for checking
    the integer form."""
    si = np.asarray(si, np.int64)
    sj = np.asarray(sj, np.int64)
    a, b = si >> 3, sj >> 3
    px = ((si & 7) + 0.5) / 8.0
    py = ((sj & 7) + 0.5) / 8.0
    fade = lambda t: t * t * t * (t * (t * 6.0 - 15.0) + 10.0)
    tot = 0.0
    for da in (0, 1):
        for db in (0, 1):
            g = GRAD[(hash5(seed, e, c, a + da, b + db) & np.uint64(7)).astype(np.int64)]
            dot = g[..., 0] * (px - da) + g[..., 1] * (py - db)
            wx = fade(px) if da else 1.0 - fade(px)
            wy = fade(py) if db else 1.0 - fade(py)
            tot = tot + wx * wy * dot
    return tot


def edge_level0(kind: int, seed: int, e: int, k: int, boundary: bool) -> np.ndarray:
    """[n, n, 4] float32 level-0 texels of one edge (row j, column i, channel)."""
    n = 1 << k
    j, i, c = np.meshgrid(np.arange(n), np.arange(n), np.arange(4), indexing="ij")
    return texel_values(kind, seed, e, n, boundary, i, j, c)
