"""Builders shared by the GPU tests: the same seeded inputs handed to the HIP
path (through the C ABI) and to the FP64 oracle."""
import numpy as np
import torch

import oracle
import paper_2207_05618_amd as htex
from htexgen import pool as gpool
from htexgen.queries import uniform_queries

INT_FIELDS = ("next", "prev", "edge", "flip", "level", "i0", "j0", "inb")


def t(a, dtype=None):
    a = np.ascontiguousarray(a if dtype is None else np.asarray(a, dtype=dtype))
    return torch.from_numpy(a).to("cuda")


class Setup:
    """A mesh with a seeded float32 pool, on the device and in the oracle."""

    def __init__(self, mesh, log2res, has_mips, kind=0, seed=102, channels=4):
        self.m = mesh
        self.log2res = np.asarray(log2res, np.uint8)
        self.has_mips = has_mips
        base, total = gpool.layout(self.log2res, has_mips)
        lvl0 = gpool.fill_level0_host(kind, seed, self.log2res, base, total,
                                      mesh.boundary_edges(), has_mips, channels=channels)
        self.dmesh = htex.Mesh.of(mesh)
        self.pool = htex.Pool(self.log2res, has_mips, htex.HTEX_F32, texels=t(lvl0),
                              channels=channels)
        if has_mips:
            htex.htex_build_mips(self.pool)
        op = oracle.Pool(self.log2res, base, lvl0.astype(np.float64), has_mips)
        if has_mips:
            op = oracle.Pool(self.log2res, base, oracle.build_mips(op), True)
        self.opool = op
        self.omesh = oracle.Mesh.of(mesh)
        torch.cuda.synchronize()

    def gpu(self, q, filt=htex.HTEX_BILINEAR, debug=False, pool=None, err=None):
        f = t(q.f) if q.f is not None else None
        out, dbg = htex.htex_sample(self.dmesh, pool or self.pool, t(q.h), t(q.u), t(q.v), f,
                                    filter=filt, debug=debug, err_count=err)
        torch.cuda.synchronize()
        return out.cpu().numpy(), (htex.debug_records(dbg) if debug else None)

    def ref(self, q, filt=oracle.BILINEAR, debug=False, opool=None):
        out, errs, d = oracle.sample(self.omesh, opool or self.opool, q.h, q.u, q.v, q.f,
                                     filter=filt, debug=debug)
        return out, errs, d


def assert_rel(got, ref, tol, floor=1e-6):
    got = np.asarray(got, np.float64)
    ref = np.asarray(ref, np.float64)
    nan_g, nan_r = np.isnan(got), np.isnan(ref)
    np.testing.assert_array_equal(nan_g, nan_r)
    ok = ~nan_r
    err = np.abs(got[ok] - ref[ok]) / np.maximum(np.abs(ref[ok]), floor)
    worst = float(err.max()) if err.size else 0.0
    assert worst <= tol, f"max relative error {worst:.3e} > {tol:.1e}"
    return worst


def assert_debug_equal(dg, do, wtol=1e-5):
    for f in INT_FIELDS:
        a, b = dg[f], do[f]
        if not np.array_equal(a, b):
            bad = np.argwhere(a != b)[:5]
            raise AssertionError(f"debug field {f} differs at {bad.tolist()}: "
                                 f"gpu {a[tuple(bad[0])]} oracle {b[tuple(bad[0])]}")
    valid = dg["next"] >= 0
    np.testing.assert_allclose(dg["W"][valid], do["W"][valid], rtol=wtol, atol=1e-6)
    np.testing.assert_allclose(dg["wf"][valid], do["wf"][valid], rtol=wtol, atol=1e-6)
    # phi = log2(m) from a float32 series on s = (m - 1) rcp(m + 1): the
    # rounding of m + 1 (2^-24), the hardware reciprocal (1 ulp, 2^-23), the
    # product (2^-24) and the Horner evaluation (about 2.5 2^-24) bound its
    # error by ~3.9e-7 relative, and phi < 1 (it enters the colour linearly,
    # far inside 1e-5)
    np.testing.assert_allclose(dg["phi"][valid], do["phi"][valid], rtol=0, atol=4e-7)


__all__ = ["Setup", "assert_rel", "assert_debug_equal", "t", "uniform_queries"]
