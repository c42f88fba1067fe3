"""Query batches: (halfedge h, barycentric (u, v), footprint f).

h is uniform over [0, H); (u, v) is uniform over the triangle u, v >= 0,
u + v <= 1 (two uniforms, folded when their sum exceeds 1), rounded to
float32.  The footprint f is the isotropic screen-space filter width in quad
parameter units, log-uniform: log2 f ~ U[lo, hi].  `sort=True` orders the batch
by h (stable), as a rasteriser walking triangles would deliver it.
"""
from __future__ import annotations

import dataclasses

import numpy as np


@dataclasses.dataclass
class Queries:
    h: np.ndarray   # int32 [Q]
    u: np.ndarray   # float32 [Q]
    v: np.ndarray   # float32 [Q]
    f: np.ndarray | None  # float32 [Q] or None

    @property
    def Q(self):
        return len(self.h)

    def take(self, idx):
        return Queries(self.h[idx], self.u[idx], self.v[idx],
                       None if self.f is None else self.f[idx])


def uniform_queries(H: int, Q: int, seed: int, log2f=None, sort: bool = False,
                    shuffle_seed: int | None = None) -> Queries:
    rng = np.random.default_rng(seed)
    h = rng.integers(0, H, size=Q, dtype=np.int64)
    r = rng.random((2, Q))
    fold = r[0] + r[1] > 1.0
    u = np.where(fold, 1.0 - r[0], r[0])
    v = np.where(fold, 1.0 - r[1], r[1])
    f = None
    if log2f is not None:
        lo, hi = log2f
        f = np.exp2(rng.uniform(lo, hi, size=Q)).astype(np.float32)
    q = Queries(h.astype(np.int32), u.astype(np.float32), v.astype(np.float32), f)
    if sort:
        q = q.take(np.argsort(q.h, kind="stable"))
    elif shuffle_seed is not None:
        q = q.take(np.random.default_rng(shuffle_seed).permutation(Q))
    return q


def tessellated_queries(H: int, T: int, footprint: float | None = None,
                        halfedges=None) -> Queries:
    """Vertex-stage queries of a uniformly tessellated intrinsic triangulation:
    every halfedge's triangle (or those in `halfedges`) is cut into T^2
    sub-triangles and each patch evaluates its (T+1)(T+2)/2 grid vertices
    (u, v) = (i/T, j/T), i + j <= T, row by row (j outer), as a tessellator
    emits them.  Vertices on patch borders are evaluated by every patch that
    owns them.  `footprint` (quad units, e.g. 1/T for a filter as wide as a
    sub-triangle) is stored for every query, or None for bilinear use.
    For T a power of two every coordinate is exact in float32.
    """
    hs = np.arange(H, dtype=np.int32) if halfedges is None else np.asarray(halfedges, np.int32)
    jj, ii = np.meshgrid(np.arange(T + 1), np.arange(T + 1), indexing="ij")
    keep = (ii + jj) <= T
    gi, gj = ii[keep], jj[keep]           # row-major over j, then i
    P = len(gi)
    h = np.repeat(hs, P)
    u = np.tile((gi / T).astype(np.float32), len(hs))
    v = np.tile((gj / T).astype(np.float32), len(hs))
    f = None if footprint is None else np.full(len(h), footprint, np.float32)
    return Queries(h, u, v, f)


def aniso_jacobians(Q: int, seed: int, minor, ratio=(1.0, 16.0)) -> np.ndarray:
    """Screen-space derivatives (du/dx, dv/dx, du/dy, dv/dy) of an elliptic
    pixel footprint per query: the minor axis has length `minor` (array or
    scalar, quad units), the major axis is longer by a log-uniform factor in
    `ratio`; the major axis points in a uniform random direction and the
    minor axis at a uniform random angle to it (screen axes need not be
    orthogonal in texture space); which screen axis is the major one is a
    coin flip.  float32 [Q, 4]."""
    rng = np.random.default_rng(seed)
    lo, hi = ratio
    r = np.exp(rng.uniform(np.log(lo), np.log(hi), Q))
    mn = np.broadcast_to(np.asarray(minor, np.float64), (Q,))
    a = rng.uniform(0.0, 2.0 * np.pi, Q)
    b = a + rng.uniform(0.25 * np.pi, 0.75 * np.pi, Q) * rng.choice([-1.0, 1.0], Q)
    major = np.stack([r * mn * np.cos(a), r * mn * np.sin(a)], 1)
    minor_v = np.stack([mn * np.cos(b), mn * np.sin(b)], 1)
    swap = rng.random(Q) < 0.5
    J = np.where(swap[:, None], np.concatenate([minor_v, major], 1),
                 np.concatenate([major, minor_v], 1))
    return np.ascontiguousarray(J, dtype=np.float32)
