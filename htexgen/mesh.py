"""Seeded polygon-mesh generators and halfedge construction.

This module is an input generator only: it builds halfedge arrays from
polygon face lists.  It holds none of the sampling arithmetic.

Halfedge convention (paper Section 2, "Halfedge Mesh Representation", Fig. 2):
every halfedge h carries Twin, Next, Prev, Vert, Edge and Face; Vert(h) is the
tail of h, so h runs from Vert(h) to Vert(Next(h)); Twin(h) = -1 marks a
boundary halfedge.  Halfedges are numbered face-major (all halfedges of face 0,
then face 1, ...), as in Fig. 2, so Next/Prev neighbours have adjacent ids.
Edge ids are assigned in the order of each edge's smallest halfedge id.
"""
from __future__ import annotations

import dataclasses

import numpy as np


@dataclasses.dataclass
class Mesh:
    twin: np.ndarray
    next: np.ndarray
    prev: np.ndarray
    vert: np.ndarray
    edge: np.ndarray
    face: np.ndarray
    H: int
    E: int
    F: int
    V: int
    positions: np.ndarray | None = None  # [V,3] float64, optional

    def face_sizes(self) -> np.ndarray:
        return np.bincount(self.face, minlength=self.F)

    def boundary_edges(self) -> np.ndarray:
        """bool[E]: True where the edge is a lone boundary halfedge."""
        b = np.zeros(self.E, dtype=bool)
        b[self.edge[self.twin < 0]] = True
        return b

    def arrays(self):
        return dict(twin=self.twin, next=self.next, prev=self.prev,
                    vert=self.vert, edge=self.edge, face=self.face)


def halfedges_from_faces(faces, V: int | None = None, positions=None) -> Mesh:
    """Build face-major halfedge arrays from oriented polygon face lists.

    Raises ValueError for faces with fewer than 3 vertices, repeated vertices
    inside a face, or two halfedges with the same direction (non-manifold or
    inconsistently oriented input).
    """
    sizes = np.fromiter((len(f) for f in faces), dtype=np.int64, count=len(faces))
    if np.any(sizes < 3):
        raise ValueError("face with fewer than 3 vertices")
    F = len(faces)
    H = int(sizes.sum())
    vert = np.fromiter((v for f in faces for v in f), dtype=np.int64, count=H)
    if V is None:
        V = int(vert.max()) + 1 if H else 0
    start = np.zeros(F + 1, dtype=np.int64)
    np.cumsum(sizes, out=start[1:])
    face = np.repeat(np.arange(F, dtype=np.int64), sizes)
    local = np.arange(H, dtype=np.int64) - start[face]
    sz = sizes[face]
    nxt = start[face] + (local + 1) % sz
    prv = start[face] + (local - 1 + sz) % sz
    for f in faces:
        if len(set(f)) != len(f):
            raise ValueError("face with a repeated vertex")
    tail = vert
    head = vert[nxt]
    kdir = tail * V + head
    krev = head * V + tail
    order = np.argsort(kdir, kind="stable")
    sk = kdir[order]
    if H > 1 and np.any(sk[1:] == sk[:-1]):
        raise ValueError("two halfedges share a direction (non-manifold or misoriented)")
    pos = np.searchsorted(sk, krev)
    pos_c = np.minimum(pos, H - 1)
    found = sk[pos_c] == krev
    twin = np.where(found, order[pos_c], -1)
    key = np.where(twin >= 0, np.minimum(np.arange(H), twin), np.arange(H))
    uniq, edge = np.unique(key, return_inverse=True)
    E = len(uniq)
    i32 = lambda a: np.ascontiguousarray(a, dtype=np.int32)
    return Mesh(twin=i32(twin), next=i32(nxt), prev=i32(prv), vert=i32(vert),
                edge=i32(edge), face=i32(face), H=H, E=E, F=F, V=V,
                positions=positions)


# ---------------------------------------------------------------- cube grids

def _cube_grid(n: int):
    """Quads of a cube whose 6 sides are n x n grids, oriented outwards.

    Returns (faces, positions) with positions on the cube [-1,1]^3.
    """
    ids = {}
    pos = []

    def vid(p):
        k = tuple(p)
        if k not in ids:
            ids[k] = len(pos)
            pos.append(k)
        return ids[k]

    faces = []
    # each side: fixed axis a at value s in {0, n}; (b, c) span the side with
    # b x c pointing outwards.
    for a in range(3):
        for s in (0, n):
            b, c = (a + 1) % 3, (a + 2) % 3
            if s == 0:
                b, c = c, b
            for x in range(n):
                for y in range(n):
                    quad = []
                    for dx, dy in ((0, 0), (1, 0), (1, 1), (0, 1)):
                        p = [0, 0, 0]
                        p[a] = s
                        p[b] = x + dx
                        p[c] = y + dy
                        quad.append(vid(p))
                    faces.append(quad)
    P = np.asarray(pos, dtype=np.float64) * (2.0 / n) - 1.0
    return faces, P


def _merge(f1, f2, a, b):
    """Merge two faces that share the edge {a,b}; f1 holds a->b, f2 holds b->a."""
    i = f1.index(a)
    r1 = f1[i + 1:] + f1[:i + 1]          # starts after a ... ends at a; begins with b
    j = f2.index(b)
    r2 = f2[j + 1:] + f2[:j + 1]          # begins with a, ends at b
    # r1 = [b, ..., a], r2 = [a, ..., b]
    out = r1 + r2[1:-1]
    return out


def _edges_of(f):
    k = len(f)
    return [(f[i], f[(i + 1) % k]) for i in range(k)]


class _FaceSet:
    """Mutable face list with a directed-edge -> face map."""

    def __init__(self, faces):
        self.faces = {i: list(f) for i, f in enumerate(faces)}
        self.dmap = {}
        for i, f in self.faces.items():
            for e in _edges_of(f):
                self.dmap[e] = i
        self.next_id = len(faces)

    def remove(self, i):
        f = self.faces.pop(i)
        for e in _edges_of(f):
            del self.dmap[e]
        return f

    def add(self, f):
        i = self.next_id
        self.next_id += 1
        self.faces[i] = f
        for e in _edges_of(f):
            self.dmap[e] = i
        return i

    def neighbour(self, i, k):
        """Face across the k-th edge of face i, and that edge (a, b)."""
        f = self.faces[i]
        a, b = f[k], f[(k + 1) % len(f)]
        return self.dmap.get((b, a)), (a, b)

    def merge(self, i, j, a, b):
        f1 = self.remove(i)
        f2 = self.remove(j)
        m = _merge(f1, f2, a, b)
        if len(set(m)) != len(m):
            raise RuntimeError("merge produced a non-simple polygon")
        return self.add(m)

    def split(self, i, diag):
        f = self.remove(i)
        a, b, c, d = f
        if diag == 0:
            return self.add([a, b, c]), self.add([a, c, d])
        return self.add([b, c, d]), self.add([b, d, a])


def cube_mesh(n: int = 4, seed: int = 101, n_split: int = 8, n_merge: int = 4) -> Mesh:
    """Closed cube of 6 n x n quad grids; seeded so that `n_split` quads are cut
    into two triangles along a random diagonal and `n_merge` disjoint pairs of
    edge-adjacent unsplit quads are merged into hexagons.

    n=4 gives the 96-quad tiny mesh: F=100 (80 quads, 16 triangles, 4 hexagons),
    V=98, E=196, H=392.
    """
    rng = np.random.default_rng(seed)
    faces, P = _cube_grid(n)
    nq = len(faces)
    order = rng.permutation(nq)
    fs = _FaceSet(faces)
    used = set()
    merged = 0
    for i in order:
        if merged == n_merge:
            break
        i = int(i)
        if i in used:
            continue
        ks = rng.permutation(4)
        for k in ks:
            j, (a, b) = fs.neighbour(i, int(k))
            if j is None or j in used or j >= nq:
                continue
            used.add(i)
            used.add(j)
            fs.merge(i, j, a, b)
            merged += 1
            break
    rest = [int(i) for i in rng.permutation(nq) if int(i) not in used]
    for i in rest[:n_split]:
        fs.split(i, int(rng.integers(0, 2)))
    out = [fs.faces[k] for k in sorted(fs.faces)]
    return halfedges_from_faces(out, V=len(P), positions=P)


def sphere_mesh(n: int = 183, seed: int = 201, frac_tri: float = 0.20,
                frac_poly: float = 0.10, frac_hole: float = 0.01) -> Mesh:
    """Seeded mixed-polygon sphere: a cube-sphere with n x n quads per side,
    edited so that about `frac_tri` of the faces are triangles, `frac_poly`
    are 5- to 8-gons (equal shares of 5, 6, 7, 8) and the rest quads, then
    `frac_hole` of the faces are removed as vertex-disjoint single-face holes
    (about 2% of the edges become boundary edges).

    Polygons are made by merging edge-adjacent faces: 4+3 -> 5, 4+4 -> 6,
    4+4+3 -> 7, 4+4+4 -> 8 (the triangle being half of a split quad).
    n=183 gives about 196k faces before holes.
    """
    rng = np.random.default_rng(seed)
    faces, P = _cube_grid(n)
    P = P / np.linalg.norm(P, axis=1, keepdims=True)
    nq = len(faces)
    # counts relative to the final face count F = nq / (1 + 0.25*frac_poly*10 ...)
    # per-polygon quad consumption: 5:2 (one of them split), 6:2, 7:3, 8:3
    k_each = frac_poly / 4.0
    # tris: 2*s + k5 + k7 = frac_tri * F ; quads consumed = F*k_each*(2+2+3+3) + s
    s_frac = (frac_tri - 2 * k_each) / 2.0
    F_est = nq / (1.0 - frac_tri - frac_poly + k_each * 10 + s_frac)
    k = int(round(k_each * F_est))
    n_split = int(round(s_frac * F_est))
    fs = _FaceSet(faces)
    used = set()

    def free(j):
        return j is not None and j < nq and j not in used

    counts = {5: 0, 6: 0, 7: 0, 8: 0}
    order = [int(i) for i in rng.permutation(nq)]
    ptr = 0
    targets = [5, 6, 7, 8]
    want = {t: k for t in targets}
    while any(counts[t] < want[t] for t in targets) and ptr < len(order):
        i = order[ptr]
        ptr += 1
        if not free(i):
            continue
        pending = [t for t in targets if counts[t] < want[t]]
        t = pending[int(rng.integers(0, len(pending)))]
        kk = int(rng.integers(0, 4))
        j, (a, b) = fs.neighbour(i, kk)
        if not free(j):
            continue
        if t in (7, 8):
            # third face across the far side of j, in a row
            fj = fs.faces[j]
            kb = fj.index(b)          # j holds edge b->a at position kb
            kc = (kb + 2) % 4
            c, (c0, c1) = fs.neighbour(j, kc)
            if not free(c) or c == i:
                continue
            if set(fs.faces[c]) & set(fs.faces[i]):
                continue
        if t == 5:
            # split j so that the triangle holding (b,a) merges with i
            used.update((i, j))
            t1, t2 = fs.split(j, int(rng.integers(0, 2)))
            tri = t1 if (b, a) in _edges_of(fs.faces[t1]) else t2
            fs.merge(i, tri, a, b)
        elif t == 6:
            used.update((i, j))
            fs.merge(i, j, a, b)
        elif t == 8:
            used.update((i, j, c))
            m = fs.merge(i, j, a, b)
            fs.merge(m, c, c0, c1)
        else:  # 7
            used.update((i, j, c))
            m = fs.merge(i, j, a, b)
            t1, t2 = fs.split(c, int(rng.integers(0, 2)))
            tri = t1 if (c1, c0) in _edges_of(fs.faces[t1]) else t2
            fs.merge(m, tri, c0, c1)
        counts[t] += 1
    rest = [i for i in order if free(i)]
    for i in rest[:n_split]:
        fs.split(i, int(rng.integers(0, 2)))
    # holes: vertex-disjoint faces removed
    keys = sorted(fs.faces)
    n_hole = int(round(frac_hole * len(keys)))
    touched = set()
    removed = 0
    for idx in rng.permutation(len(keys)):
        if removed == n_hole:
            break
        fi = keys[int(idx)]
        f = fs.faces[fi]
        # keep hole rims disjoint: no vertex of f or of its neighbours touched
        ring = set(f)
        if ring & touched:
            continue
        nbr_ok = True
        for kk in range(len(f)):
            j, _ = fs.neighbour(fi, kk)
            if j is None:
                nbr_ok = False
                break
        if not nbr_ok:
            continue
        touched |= ring
        fs.remove(fi)
        removed += 1
    out = [fs.faces[kk] for kk in sorted(fs.faces)]
    return halfedges_from_faces(out, V=len(P), positions=P)
