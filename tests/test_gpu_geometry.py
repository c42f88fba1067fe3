"""Intrinsic triangles on the GPU (htex_triangle_vertices, Alg. 1) against
the FP64 oracle: v0 and v2 are copies (bit-exact), the centroid v1 within
one float32 rounding of the oracle's FP64 mean and bit-identical across the
triangles of a face; bad vertex ids give NaN rows and count errors."""
import numpy as np
import pytest
import torch

import oracle
import paper_2207_05618_amd as htex
from htexgen.mesh import cube_mesh, sphere_mesh
from tests.fixtures import load_fig2
from tests.gpu_helpers import t

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("which", ["fig2", "cube", "sphere"])
def test_triangle_vertices_match_oracle(which):
    if which == "fig2":
        m = load_fig2()
        pos = np.random.default_rng(1).normal(size=(m.V, 3)).astype(np.float32)
    elif which == "cube":
        m = cube_mesh()
        pos = m.positions.astype(np.float32)
    else:
        m = sphere_mesh(n=40, seed=2)
        pos = m.positions.astype(np.float32)
    dm = htex.Mesh.of(m)
    err = torch.zeros(1, dtype=torch.int32, device="cuda")
    T = htex.htex_triangle_vertices(dm, t(m.vert), t(pos), err_count=err).cpu().numpy()
    assert int(err.item()) == 0
    ref, bad = oracle.triangle_vertices(oracle.Mesh.of(m), m.vert, pos.astype(np.float64))
    assert bad == 0
    np.testing.assert_array_equal(T[:, 0], ref[:, 0].astype(np.float32))
    np.testing.assert_array_equal(T[:, 2], ref[:, 2].astype(np.float32))
    d = np.abs(T[:, 1].astype(np.float64) - ref[:, 1])
    assert (d <= 2.0 ** -24 * np.abs(ref[:, 1]) + 1e-38).all()
    # one centroid per face, bit for bit
    first = np.full(m.F, -1)
    for h in range(m.H):
        f = m.face[h]
        if first[f] < 0:
            first[f] = h
        else:
            np.testing.assert_array_equal(T[h, 1], T[first[f], 1])


def test_bad_vertex_ids_are_counted():
    m = cube_mesh()
    vert = m.vert.copy()
    vert[7] = m.V
    err = torch.zeros(1, dtype=torch.int32, device="cuda")
    T = htex.htex_triangle_vertices(htex.Mesh.of(m), t(vert), t(m.positions.astype(np.float32)),
                                    err_count=err).cpu().numpy()
    # every halfedge of the face of h7 walks over the bad id
    face = m.face == m.face[7]
    assert int(err.item()) == int(face.sum())
    assert np.isnan(T[face]).all() and np.isfinite(T[~face]).all()
