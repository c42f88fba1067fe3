"""A rasterized frame (htexgen/raster.py on the oracle's intrinsic
triangles) sampled on the GPU: trilinear with each pixel's isotropic
footprint and anisotropic with its derivatives, in scanline order and in
halfedge order, against the FP64 oracle (integer trace bit-exact, probe
counts bit-exact, colours within 1e-5)."""
import numpy as np
import pytest
import torch

import oracle
import paper_2207_05618_amd as htex
from htexgen.mesh import sphere_mesh
from htexgen.raster import rasterize, sphere_view
from tests.gpu_helpers import Setup, assert_debug_equal, assert_rel, t

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def scene():
    m = sphere_mesh(n=40, seed=2)
    lr = np.random.default_rng(3).integers(3, 7, m.E)
    s = Setup(m, lr, has_mips=True, kind=1, seed=4)
    T, bad = oracle.triangle_vertices(s.omesh, m.vert, m.positions)
    assert bad == 0
    fr = rasterize(T, sphere_view(960, 540))
    return s, fr


def test_raster_frame_trilinear(scene):
    s, fr = scene
    f = fr.footprint()
    out, dbg = htex.htex_sample(s.dmesh, s.pool, t(fr.h), t(fr.u), t(fr.v), t(f),
                                filter=htex.HTEX_TRILINEAR, debug=True)
    torch.cuda.synchronize()
    got = out.cpu().numpy()
    ref, errs, do = oracle.sample(s.omesh, s.opool, fr.h, fr.u, fr.v, f, filter=oracle.TRILINEAR,
                                  debug=True)
    assert errs == 0
    assert_debug_equal(htex.debug_records(dbg), do)
    assert_rel(got, ref, 1e-5)
    # the same fragments in halfedge order give the same bits per fragment
    order = np.argsort(fr.h, kind="stable")
    prep = htex.Prepared(s.dmesh, s.pool)
    o2 = htex.htex_sample_prepared(prep, s.pool, t(fr.h[order]), t(fr.u[order]), t(fr.v[order]),
                                   t(f[order]), filter=htex.HTEX_TRILINEAR,
                                   flags=htex.HTEX_QUERIES_SORTED)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(o2.cpu().numpy(), got[order])


def test_raster_frame_anisotropic(scene):
    s, fr = scene
    out, n = htex.htex_sample_aniso(s.dmesh, s.pool, t(fr.h), t(fr.u), t(fr.v), t(fr.jac),
                                    max_aniso=16, nprobe=True)
    torch.cuda.synchronize()
    ref, errs, nref = oracle.sample_aniso(s.omesh, s.opool, fr.h, fr.u, fr.v, fr.jac,
                                          max_aniso=16)
    assert errs == 0
    np.testing.assert_array_equal(n.cpu().numpy(), nref)
    assert nref.max() > 4          # grazing views near the silhouette
    assert_rel(out.cpu().numpy(), ref, 1e-5)
