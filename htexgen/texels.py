"""Seeded texel values for per-edge square textures (level 0 only).

Input generator only: every value is a pure function of
(seed, edge, row j, column i, channel c) built from the splitmix64 mixing
function (Steele, Lea and Flood, "Fast splittable pseudorandom number
generators", OOPSLA 2014), so a device fill kernel can produce the same bits
independently.  Mip levels are not generated here.

Two fills:

* ``uniform``: each texel channel is an independent 24-bit uniform value in
  [0, 1): ``(hash >> 40) * 2^-24`` (exact in float32).
* ``smooth``: value noise on a lattice of 8-texel cells.  Each lattice point
  carries an integer value in [1, 63]; a texel blends its cell's four corner
  values with the integer smooth ramp R[f] (R[f] + R[7-f] = 64), giving an
  integer numerator below 2^18 that is scaled by 2^-18 (exact in float32).
  Values lie in [1/64, 63/64].

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

# integer smooth ramp over the 8 texel centres of a lattice cell
RAMP = np.array([1, 6, 14, 25, 39, 50, 58, 63], dtype=np.int64)


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


def edge_level0(kind: int, seed: int, e: int, k: int, boundary: bool) -> np.ndarray:
    """[n, n, 4] float32 level-0 texels of one edge (row j, column i, channel)."""
    n = 1 << k
    j, i, c = np.meshgrid(np.arange(n), np.arange(n), np.arange(4), indexing="ij")
    return texel_values(kind, seed, e, n, boundary, i, j, c)
