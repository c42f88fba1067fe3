"""FP64 CPU oracle for batched Htex sampling -- TEST INFRASTRUCTURE ONLY.

Only the test suite, the package smoke check and the benchmark's CPU-baseline
leg may import this package.  The product library never calls it.

Thin numpy/ctypes wrapper over ``htex_oracle.c`` (plain C, FP64).  Built with
gcc on first use if the shared library is missing.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np

from . import build as _build

_lib = None

BILINEAR = 0
TRILINEAR = 1

DEBUG_DTYPE = np.dtype([
    ("next", "<i4"), ("prev", "<i4"),
    ("edge", "<i4", (3,)), ("flip", "<i4", (3,)),
    ("level", "<i4", (3, 2)), ("i0", "<i4", (3, 2)), ("j0", "<i4", (3, 2)),
    ("inb", "<i4", (3, 2)),
    ("phi", "<f8"), ("W", "<f8"), ("wf", "<f8", (3,)),
], align=True)


class _Mesh(C.Structure):
    _fields_ = [("H", C.c_int32), ("E", C.c_int32),
                ("twin", C.c_void_p), ("next", C.c_void_p),
                ("prev", C.c_void_p), ("edge", C.c_void_p)]


class _Pool(C.Structure):
    _fields_ = [("E", C.c_int32), ("has_mips", C.c_int32),
                ("channels", C.c_int32), ("pad", C.c_int32),
                ("log2res", C.c_void_p), ("base", C.c_void_p),
                ("texels", C.c_void_p)]


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_build.LIB):
            _build.build()
        L = C.CDLL(_build.LIB)
        p = C.c_void_p
        L.ora_sample.restype = C.c_int64
        L.ora_sample.argtypes = [p, p, C.c_int64, p, p, p, p, C.c_int, p, p, C.c_int]
        L.ora_sample_aniso.restype = C.c_int64
        L.ora_sample_aniso.argtypes = [p, p, C.c_int64, p, p, p, p, C.c_int, p, p, C.c_int]
        L.ora_backward.restype = C.c_int64
        L.ora_backward.argtypes = [p, p, C.c_int64, p, p, p, p, C.c_int, p, p, p]
        L.ora_build_mips.restype = None
        L.ora_build_mips.argtypes = [p, p]
        L.ora_mip_backward.restype = None
        L.ora_mip_backward.argtypes = [p, p]
        L.ora_f32_to_bf16.restype = C.c_uint16
        L.ora_f32_to_bf16.argtypes = [C.c_float]
        L.ora_bf16_to_f64.restype = C.c_double
        L.ora_bf16_to_f64.argtypes = [C.c_uint16]
        L.ora_e4m3_to_f64.restype = C.c_double
        L.ora_e4m3_to_f64.argtypes = [C.c_uint8]
        L.ora_f64_to_e4m3_sat.restype = C.c_uint8
        L.ora_f64_to_e4m3_sat.argtypes = [C.c_double]
        L.ora_quantize_bf16.restype = None
        L.ora_quantize_bf16.argtypes = [p, C.c_int64, p]
        L.ora_quantize_e4m3.restype = None
        L.ora_quantize_e4m3.argtypes = [p, p, C.c_int64, p, p]
        L.ora_dequantize_bf16.restype = None
        L.ora_dequantize_bf16.argtypes = [p, C.c_int64, p]
        L.ora_dequantize_e4m3.restype = None
        L.ora_dequantize_e4m3.argtypes = [p, p, p, p]
        L.ora_texture_fetch.restype = None
        L.ora_texture_fetch.argtypes = [p, C.c_int32, C.c_int, C.c_double, C.c_double,
                                        C.c_double, p, p]
        L.ora_triangle_vertices.restype = C.c_int64
        L.ora_triangle_vertices.argtypes = [p, p, C.c_int32, p, p]
        L.ora_texel_positions.restype = None
        L.ora_texel_positions.argtypes = [p, p, p, p]
        L.ora_corner_average.restype = None
        L.ora_corner_average.argtypes = [p, p, p, C.c_int32, C.c_int32, p, p]
        L.ora_validate.restype = C.c_int
        L.ora_validate.argtypes = [p, p, p]
        _lib = L
    return _lib


def _ptr(a):
    return None if a is None else a.ctypes.data


def _c(a, dt):
    return None if a is None else np.ascontiguousarray(a, dtype=dt)


class Mesh:
    """Halfedge arrays held for the oracle (copies, int32)."""

    def __init__(self, twin, next, prev, edge, E, vert=None):
        self.twin = _c(twin, np.int32)
        self.next = _c(next, np.int32)
        self.prev = _c(prev, np.int32)
        self.edge = _c(edge, np.int32)
        self.vert = _c(vert, np.int32)
        self.H = len(self.twin)
        self.E = int(E)
        self._s = _Mesh(self.H, self.E, _ptr(self.twin), _ptr(self.next),
                        _ptr(self.prev), _ptr(self.edge))

    @classmethod
    def of(cls, m):
        return cls(m.twin, m.next, m.prev, m.edge, m.E, getattr(m, "vert", None))


class Pool:
    """Texel pool for the oracle: float64 [total, C] (C = 4 RGBA channels or
    1, e.g. a displacement map) plus per-edge layout."""

    def __init__(self, log2res, base, texels, has_mips):
        self.log2res = _c(log2res, np.uint8)
        self.base = _c(base, np.int64)
        self.texels = _c(texels, np.float64)
        if self.texels.ndim != 2 or self.texels.shape[1] not in (1, 4):
            raise ValueError("texels must be [total, 4] or [total, 1]")
        self.channels = int(self.texels.shape[1])
        self.has_mips = int(bool(has_mips))
        self.E = len(self.log2res)
        self._s = _Pool(self.E, self.has_mips, self.channels, 0, _ptr(self.log2res),
                        _ptr(self.base), _ptr(self.texels))


def sample(mesh: Mesh, pool: Pool, h, u, v, f=None, filter=BILINEAR,
           debug=False, nthreads=0):
    """Alg. 3 for every query.  Returns (out float64 [Q, C], errors, debug)."""
    h = _c(h, np.int32)
    u = _c(u, np.float32)
    v = _c(v, np.float32)
    f = _c(f, np.float32)
    Q = len(h)
    out = np.empty((Q, pool.channels), dtype=np.float64)
    dbg = np.zeros(Q, dtype=DEBUG_DTYPE) if debug else None
    errs = lib().ora_sample(C.byref(mesh._s), C.byref(pool._s), Q, _ptr(h), _ptr(u),
                            _ptr(v), _ptr(f), int(filter), _ptr(out), _ptr(dbg),
                            int(nthreads))
    if errs < 0:
        raise ValueError("oracle rejected the call (trilinear on a pool without mips)")
    return out, int(errs), dbg


def sample_aniso(mesh: Mesh, pool: Pool, h, u, v, jac, max_aniso=16, nthreads=0):
    """Anisotropic Alg. 3 (Section 5.1 reading): jac is float32 [Q, 4] =
    (du/dx, dv/dx, du/dy, dv/dy).  Returns (out float64 [Q, C], errors,
    probes int32 [Q])."""
    h = _c(h, np.int32)
    u = _c(u, np.float32)
    v = _c(v, np.float32)
    jac = _c(jac, np.float32).reshape(-1, 4)
    Q = len(h)
    out = np.empty((Q, pool.channels), dtype=np.float64)
    n = np.zeros(Q, dtype=np.int32)
    errs = lib().ora_sample_aniso(C.byref(mesh._s), C.byref(pool._s), Q, _ptr(h), _ptr(u),
                                  _ptr(v), _ptr(jac), int(max_aniso), _ptr(out), _ptr(n),
                                  int(nthreads))
    if errs < 0:
        raise ValueError("oracle rejected the call (needs mips and max_aniso >= 1)")
    return out, int(errs), n


def backward(mesh: Mesh, pool: Pool, h, u, v, dout, f=None, filter=BILINEAR,
             with_abs=False):
    """Gradient of sum(out * dout) with respect to the texels (float64, pool-shaped)."""
    h = _c(h, np.int32)
    u = _c(u, np.float32)
    v = _c(v, np.float32)
    f = _c(f, np.float32)
    dout = _c(dout, np.float64)
    dtex = np.zeros_like(pool.texels)
    dabs = np.zeros_like(pool.texels) if with_abs else None
    errs = lib().ora_backward(C.byref(mesh._s), C.byref(pool._s), len(h), _ptr(h),
                              _ptr(u), _ptr(v), _ptr(f), int(filter), _ptr(dout),
                              _ptr(dtex), _ptr(dabs))
    if errs < 0:
        raise ValueError("oracle rejected the call")
    return (dtex, dabs) if with_abs else dtex


def build_mips(pool: Pool) -> np.ndarray:
    """Box-filtered mip chain in FP64 from level 0 of `pool` (returns a copy)."""
    tex = pool.texels.copy()
    p2 = Pool(pool.log2res, pool.base, tex, pool.has_mips)
    lib().ora_build_mips(C.byref(p2._s), _ptr(tex))
    return tex


def mip_backward(pool: Pool, dtex) -> np.ndarray:
    """Transpose of build_mips: gradients of every level folded into level 0
    (returns a copy; see ora_mip_backward)."""
    d = np.array(dtex, dtype=np.float64, copy=True, order="C")
    p2 = Pool(pool.log2res, pool.base, np.zeros((1, d.shape[1])), pool.has_mips)
    lib().ora_mip_backward(C.byref(p2._s), _ptr(d))
    return d


def f32_to_bf16(x):
    x = np.ascontiguousarray(x, dtype=np.float32).reshape(-1)
    out = np.empty(len(x), dtype=np.uint16)
    lib().ora_quantize_bf16(_ptr(x), len(x), _ptr(out))
    return out


def bf16_to_f64(codes):
    c = np.ascontiguousarray(codes, dtype=np.uint16)
    out = np.empty(c.shape, dtype=np.float64)
    lib().ora_dequantize_bf16(_ptr(c), c.size, _ptr(out))
    return out


def e4m3_pool_to_f64(log2res, base, has_mips, codes, scale):
    """float64 [total,4] texel values of an FP8 pool (decoded code x edge scale)."""
    c = np.ascontiguousarray(codes, dtype=np.uint8)
    s = np.ascontiguousarray(scale, dtype=np.float32)
    p = Pool(log2res, base, np.zeros((1, c.shape[1])), has_mips)
    out = np.zeros(c.shape, dtype=np.float64)
    lib().ora_dequantize_e4m3(C.byref(p._s), _ptr(c), _ptr(s), _ptr(out))
    return out


def e4m3_table() -> np.ndarray:
    """float64 value of each of the 256 E4M3 codes (NaN for the NaN codes)."""
    L = lib()
    return np.array([L.ora_e4m3_to_f64(c) for c in range(256)])


def f64_to_e4m3(x) -> np.ndarray:
    L = lib()
    return np.array([L.ora_f64_to_e4m3_sat(float(a)) for a in np.asarray(x).reshape(-1)],
                    dtype=np.uint8)


def quantize_e4m3(log2res, base, has_mips, texels_f32):
    """(codes uint8 [total, C], scale float32 [E]) for a float32 pool."""
    t = np.ascontiguousarray(texels_f32, dtype=np.float32)
    p = Pool(log2res, base, np.zeros((1, t.shape[1])), has_mips)
    codes = np.zeros(t.shape, dtype=np.uint8)
    scale = np.zeros(p.E, dtype=np.float32)
    lib().ora_quantize_e4m3(C.byref(p._s), _ptr(t), t.shape[0], _ptr(codes), _ptr(scale))
    return codes, scale


def triangle_vertices(mesh: Mesh, vert, positions):
    """Alg. 1 for every halfedge: float64 [H, 3, 3] = (v0, v1, v2) per
    intrinsic triangle, and the number of halfedges that could not be
    resolved (NaN rows)."""
    vt = _c(vert, np.int32)
    pos = _c(positions, np.float64).reshape(-1, 3)
    out = np.empty((mesh.H, 3, 3), dtype=np.float64)
    bad = lib().ora_triangle_vertices(C.byref(mesh._s), _ptr(vt), len(pos), _ptr(pos), _ptr(out))
    return out, int(bad)


def texel_positions(mesh: Mesh, tri, pool: Pool) -> np.ndarray:
    """Surface point of every texel centre (Section 4.2 read backwards,
    Alg. 1 triangles `tri` [H, 3, 3]): float64 [total, 3], NaN on padding."""
    T = _c(tri, np.float64)
    out = np.full((len(pool.texels), 3), np.nan)
    lib().ora_texel_positions(C.byref(mesh._s), _ptr(T), C.byref(pool._s), _ptr(out))
    return out


def corner_average(mesh: Mesh, pool: Pool, vert, face, V: int, F: int) -> np.ndarray:
    """Section 4.4 corner pre-processing in FP64 (returns a copy of the
    texels): corner texels on one mesh vertex or one face centroid take
    their mean, per resolution n >= 2."""
    tex = pool.texels.copy()
    p2 = Pool(pool.log2res, pool.base, tex, pool.has_mips)
    vt = _c(vert, np.int32)
    fc = _c(face, np.int32)
    lib().ora_corner_average(C.byref(mesh._s), _ptr(vt), _ptr(fc), int(V), int(F),
                             C.byref(p2._s), _ptr(tex))
    return tex


def validate(mesh: Mesh):
    """(status, first_bad_halfedge): 0 when every halfedge invariant holds."""
    bad = np.zeros(1, dtype=np.int32)
    rc = lib().ora_validate(C.byref(mesh._s), _ptr(mesh.vert), _ptr(bad))
    return int(rc), int(bad[0])


def texture_fetch(pool: Pool, e: int, x: float, y: float, f: float = 0.0,
                  filter=BILINEAR):
    """One filtered fetch (Alg. 3's Texture): (colour float64[C], weight)."""
    out = np.zeros(4, dtype=np.float64)
    w = np.zeros(1, dtype=np.float64)
    lib().ora_texture_fetch(C.byref(pool._s), int(e), int(filter), float(f), float(x),
                            float(y), _ptr(out), _ptr(w))
    return out[:pool.channels], float(w[0])
