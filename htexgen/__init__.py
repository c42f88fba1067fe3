"""Seeded synthetic inputs (meshes, texel pools, query batches).

Shared by the tests, the bench and the parity checks; it contains no part of
the sampling arithmetic.
"""
from .mesh import Mesh, halfedges_from_faces, cube_mesh, sphere_mesh  # noqa: F401
