"""Shared fixtures for tests: meshes, pools and query batches."""
import os

import numpy as np

from htexgen import pool as gpool
from htexgen.mesh import Mesh, cube_mesh, halfedges_from_faces
from htexgen.queries import uniform_queries

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def load_fig2():
    """The Fig. 2 halfedge table as a dict of int32 arrays."""
    rows = []
    with open(os.path.join(GOLDEN, "fig2_halfedges.txt")) as fh:
        for line in fh:
            line = line.strip()
            if line and not line.startswith("#"):
                rows.append([int(t) for t in line.split()])
    a = np.array(rows, dtype=np.int32)
    assert (a[:, 0] == np.arange(12)).all()
    names = ["twin", "next", "prev", "vert", "edge", "face"]
    d = {n: np.ascontiguousarray(a[:, i + 1]) for i, n in enumerate(names)}
    return Mesh(H=12, E=int(d["edge"].max()) + 1, F=int(d["face"].max()) + 1,
                V=int(d["vert"].max()) + 1, **d)


def make_pool_f64(mesh, log2res, has_mips, kind=0, seed=102):
    """(base, total, level-0 float32 pool) from the seeded generator."""
    base, total = gpool.layout(log2res, has_mips)
    P = gpool.fill_level0_host(kind, seed, log2res, base, total, mesh.boundary_edges(),
                               has_mips)
    return base, total, P


def tiny_meshes():
    """A few small meshes with different structure (closed and with holes)."""
    out = [cube_mesh(), cube_mesh(n=2, seed=7, n_split=3, n_merge=1), load_fig2()]
    # open strip: quads and a triangle fan with boundary
    faces = [[0, 1, 5, 4], [1, 2, 6, 5], [2, 3, 7, 6], [4, 5, 8], [5, 6, 9, 8]]
    out.append(halfedges_from_faces(faces))
    return out


__all__ = ["load_fig2", "make_pool_f64", "tiny_meshes", "uniform_queries", "cube_mesh"]
