"""MI355X-native batched Htex sampling (per-halfedge texturing, Barbier &
Dupuy 2022): a thin Python binding over libhtex's C ABI (include/htex.h).

Names follow the C entry points.  This layer only marshals arguments: torch
supplies device memory and the current stream; every step of the sampling
path runs in the HIP kernels of libhtex.  Tensors must live on the GPU; there
is no CPU path.
"""
from __future__ import annotations

import ctypes as C
import hashlib

import numpy as np
import torch

from . import _lib
from ._lib import (DEBUG_FIELDS, HTEX_BF16, HTEX_BILINEAR, HTEX_F32, HTEX_FP8_E4M3,  # noqa: F401
                   HTEX_QUERIES_SCATTERED, HTEX_QUERIES_SORTED, HTEX_TRILINEAR, HtexError,
                   check, load)

__all__ = ["Mesh", "Pool", "htex_pool_layout", "htex_mesh_validate", "htex_build_mips",
           "htex_corner_average", "htex_mip_backward", "htex_triangle_vertices",
           "htex_quantize", "htex_sample", "htex_sample_backward", "HtexSample",
           "htex_prepare", "htex_sample_prepared", "Prepared",
           "htex_sample_aniso", "htex_sample_aniso_prepared",
           "htex_sort_queries", "htex_sort_batch", "htex_permute_queries",
           "htex_unpermute_results",
           "debug_records", "HtexError"]

DEBUG_DTYPE = np.dtype(DEBUG_FIELDS)
_TEXEL_TORCH = {HTEX_F32: torch.float32, HTEX_BF16: torch.int16, HTEX_FP8_E4M3: torch.uint8}


def _stream(stream=None) -> int:
    s = torch.cuda.current_stream() if stream is None else stream
    return s.cuda_stream


def _dev(t: torch.Tensor, dtype: torch.dtype, name: str) -> torch.Tensor:
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA (HIP) tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return t


class Mesh:
    """Halfedge operators Twin/Next/Prev/Edge (Section 2) as device int32 arrays."""

    def __init__(self, twin, next, prev, edge, E: int, device="cuda"):
        as_t = lambda a: torch.as_tensor(np.ascontiguousarray(a, np.int32)).to(device)
        self.twin, self.next, self.prev, self.edge = (as_t(twin), as_t(next), as_t(prev),
                                                      as_t(edge))
        self.H = int(self.twin.numel())
        self.E = int(E)
        self.c = _lib.htex_mesh(self.H, self.E, self.twin.data_ptr(), self.next.data_ptr(),
                                self.prev.data_ptr(), self.edge.data_ptr())

    @classmethod
    def of(cls, m, device="cuda"):
        return cls(m.twin, m.next, m.prev, m.edge, m.E, device)


def htex_pool_layout(log2res, has_mips: bool):
    """(base int64[E], total_texels) for the pool format of htex.h (host)."""
    lr = np.ascontiguousarray(log2res, dtype=np.uint8)
    E = len(lr)
    base = np.zeros(max(E, 1), dtype=np.int64)
    total = np.zeros(1, dtype=np.int64)
    check(load().htex_pool_layout(E, lr.ctypes.data, int(bool(has_mips)), base.ctypes.data,
                                  total.ctypes.data))
    return base[:E], int(total[0])


def layout_key(log2res, has_mips: bool, total: int):
    """What prepared records depend on: the pool's texel layout (edge count,
    size, mips, per-edge resolutions) -- not the texels, their storage type
    or their channel count."""
    lr = np.ascontiguousarray(log2res, dtype=np.uint8)
    return (len(lr), int(total), bool(has_mips), hashlib.sha256(lr.tobytes()).hexdigest())


class Pool:
    """Per-edge texel pool on the device (layout of htex.h).

    texels: float32 [total, C] (HTEX_F32), int16 [total, C] holding bfloat16
    bits (HTEX_BF16) or uint8 [total, C] holding E4M3 codes (HTEX_FP8_E4M3,
    with float32 scale [E]); C = 4 (RGBA) or 1 (e.g. displacement)."""

    def __init__(self, log2res, has_mips: bool, dtype: int = HTEX_F32, texels=None,
                 scale=None, device="cuda", channels: int = 4):
        lr = np.ascontiguousarray(log2res, dtype=np.uint8)
        self.E = len(lr)
        self.has_mips = bool(has_mips)
        self.dtype = int(dtype)
        if channels not in (1, 4):
            raise ValueError("channels must be 1 or 4")
        self.channels = int(channels)
        self.max_log2res = int(lr.max()) if self.E else 0
        base, total = htex_pool_layout(lr, has_mips)
        self.base_host = base
        self.log2res_host = lr
        self.total = total
        self.log2res = torch.as_tensor(lr).to(device)
        self.base = torch.as_tensor(base).to(device)
        if texels is None:
            texels = torch.zeros((total, self.channels), dtype=_TEXEL_TORCH[self.dtype],
                                 device=device)
        self.texels = _dev(texels, _TEXEL_TORCH[self.dtype], "texels")
        if self.texels.shape != (total, self.channels):
            raise ValueError(f"texels must have shape ({total}, {self.channels})")
        self.scale = scale
        self.layout_key = layout_key(lr, self.has_mips, total)
        if self.dtype == HTEX_FP8_E4M3:
            self.scale = _dev(scale, torch.float32, "scale") if scale is not None else \
                torch.zeros(self.E, dtype=torch.float32, device=device)
        self._sync_c()

    def _sync_c(self):
        self.c = _lib.htex_pool(self.E, self.dtype, int(self.has_mips), self.max_log2res,
                                self.channels, 0, self.total, self.log2res.data_ptr(),
                                self.base.data_ptr(),
                                self.texels.data_ptr(),
                                self.scale.data_ptr() if self.scale is not None else None)

    def nbytes(self) -> int:
        return self.texels.numel() * self.texels.element_size()


def htex_mesh_validate(mesh: Mesh, stream=None):
    """(ok, first_bad_halfedge): checks the halfedge invariants on the device."""
    bad = C.c_int32(-1)
    st = load().htex_mesh_validate(C.byref(mesh.c), C.byref(bad), _stream(stream))
    if st == -2:
        return False, int(bad.value)
    check(st)
    return True, -1


def htex_build_mips(pool: Pool, stream=None):
    check(load().htex_build_mips(C.byref(pool.c), pool.texels.data_ptr(), _stream(stream)))


def htex_triangle_vertices(mesh: Mesh, vert, positions, err_count=None, stream=None):
    """Alg. 1 on the device -> float32 [H, 3, 3] = (v0, v1, v2) per halfedge."""
    vert = _dev(vert, torch.int32, "vert")
    positions = _dev(positions, torch.float32, "positions")
    if positions.dim() != 2 or positions.shape[1] != 3:
        raise ValueError("positions must be [V, 3]")
    out = torch.empty((mesh.H, 3, 3), dtype=torch.float32, device=vert.device)
    err = None if err_count is None else _dev(err_count, torch.int32, "err_count").data_ptr()
    check(load().htex_triangle_vertices(C.byref(mesh.c), vert.data_ptr(), positions.shape[0],
                                        positions.data_ptr(), out.data_ptr(), err,
                                        _stream(stream)))
    return out


def htex_mip_backward(pool: Pool, dtexels: torch.Tensor, clear_coarse: bool = False,
                      stream=None) -> torch.Tensor:
    """Transpose of htex_build_mips on a pool-shaped float32 gradient, in
    place: level 0 receives the gradient through every coarser level."""
    _dev(dtexels, torch.float32, "dtexels")
    if dtexels.shape != (pool.total, pool.channels):
        raise ValueError("dtexels must have the pool's shape")
    check(load().htex_mip_backward(C.byref(pool.c), dtexels.data_ptr(), int(bool(clear_coarse)),
                                   _stream(stream)))
    return dtexels


def htex_corner_average(mesh: Mesh, pool: Pool, err_count: torch.Tensor | None = None,
                        stream=None):
    """Corner pre-processing (Section 4.4) of a float32 pool, in place: corner
    texels on one mesh vertex or one face centroid take their mean, on every
    level of at least 2x2 texels.  Run after htex_build_mips."""
    err = None if err_count is None else _dev(err_count, torch.int32, "err_count").data_ptr()
    check(load().htex_corner_average(C.byref(mesh.c), C.byref(pool.c), pool.texels.data_ptr(),
                                     err, _stream(stream)))


def htex_quantize(pool: Pool, dtype: int, stream=None) -> Pool:
    """New pool holding `pool` (float32) converted to HTEX_BF16 or HTEX_FP8_E4M3."""
    q = Pool(pool.log2res_host, pool.has_mips, dtype, device=pool.texels.device,
             channels=pool.channels)
    scale_ptr = q.scale.data_ptr() if q.scale is not None else None
    check(load().htex_quantize(C.byref(pool.c), int(dtype), q.texels.data_ptr(), scale_ptr,
                               _stream(stream)))
    return q


def _queries(h, u, v, footprint):
    h = _dev(h, torch.int32, "h")
    u = _dev(u, torch.float32, "u")
    v = _dev(v, torch.float32, "v")
    if footprint is not None:
        footprint = _dev(footprint, torch.float32, "footprint")
    Q = h.numel()
    if u.numel() != Q or v.numel() != Q or (footprint is not None and footprint.numel() != Q):
        raise ValueError("query arrays differ in length")
    q = _lib.htex_queries(Q, h.data_ptr(), u.data_ptr(), v.data_ptr(),
                          footprint.data_ptr() if footprint is not None else None)
    return q, Q


def _rows(t, name, n, C_):
    """Checks a float32 [n, C_] device tensor (a [n] vector when C_ == 1 is
    accepted too)."""
    _dev(t, torch.float32, name)
    if t.numel() != n * C_ or (t.dim() == 2 and tuple(t.shape) != (n, C_)) or t.dim() > 2:
        raise ValueError(f"{name} must have shape ({n}, {C_}), got {tuple(t.shape)}")
    return t


def _out(out, Q, pool, device):
    if out is None:
        return torch.empty((Q, pool.channels), dtype=torch.float32, device=device)
    return _rows(out, "out", Q, pool.channels)


def htex_sample(mesh: Mesh, pool: Pool, h, u, v, footprint=None, filter=HTEX_BILINEAR,
                flags=0, out=None, debug=False, err_count=None, stream=None):
    """Alg. 3 for every query -> (out float32 [Q, C], debug int32 [Q, 40] or None)."""
    q, Q = _queries(h, u, v, footprint)
    out = _out(out, Q, pool, h.device)
    dbg = torch.zeros((Q, 40), dtype=torch.int32, device=h.device) if debug else None
    if err_count is not None:
        _dev(err_count, torch.int32, "err_count")
    check(load().htex_sample(C.byref(mesh.c), C.byref(pool.c), C.byref(q), int(filter),
                             int(flags), out.data_ptr(),
                             dbg.data_ptr() if dbg is not None else None,
                             err_count.data_ptr() if err_count is not None else None,
                             _stream(stream)))
    return out, dbg


class Prepared:
    """Per-halfedge fetch records of one (mesh, pool layout) pair (device).
    Keeps the layout it was built for (edge count, pool size, mips, the
    per-edge resolutions): a pool of another layout is refused."""

    def __init__(self, mesh: Mesh, pool: Pool, stream=None):
        self.H = mesh.H
        n = max(mesh.H, 1) * _lib.HTEX_PREP_BYTES // 16
        self.buf = torch.empty((n, 4), dtype=torch.int32, device=mesh.twin.device)
        htex_prepare(mesh, pool, self, stream)

    def check_pool(self, pool: Pool):
        if pool.layout_key != self.layout_key:
            raise ValueError("prepared records were built for another pool layout "
                             f"(E, texels, mips = {self.layout_key[:3]}; the pool has "
                             f"{pool.layout_key[:3]}); rebuild them with Prepared(mesh, pool)")


def htex_prepare(mesh: Mesh, pool: Pool, prep: "Prepared", stream=None):
    check(load().htex_prepare(C.byref(mesh.c), C.byref(pool.c), prep.buf.data_ptr(),
                              _stream(stream)))
    prep.layout_key = pool.layout_key


def htex_sample_prepared(prep: "Prepared", pool: Pool, h, u, v, footprint=None,
                         filter=HTEX_BILINEAR, flags=0, out=None, err_count=None,
                         stream=None):
    """htex_sample from prepared records (bit-identical results) -> out [Q, C]."""
    prep.check_pool(pool)
    q, Q = _queries(h, u, v, footprint)
    out = _out(out, Q, pool, h.device)
    if err_count is not None:
        _dev(err_count, torch.int32, "err_count")
    check(load().htex_sample_prepared(prep.H, prep.buf.data_ptr(), C.byref(pool.c), C.byref(q),
                                      int(filter), int(flags), out.data_ptr(),
                                      err_count.data_ptr() if err_count is not None else None,
                                      _stream(stream)))
    return out


def htex_sample_prepared_reordered(prep: "Prepared", pool: Pool, h, u, v, footprint=None,
                                   filter=HTEX_BILINEAR, out=None, err_count=None, stream=None):
    """htex_sample_prepared for a batch in any order: the library puts it in
    halfedge order, samples it there and writes the results in the batch's
    own order (the same bits) -> out [Q, C]."""
    prep.check_pool(pool)
    q, Q = _queries(h, u, v, footprint)
    out = _out(out, Q, pool, h.device)
    if err_count is not None:
        _dev(err_count, torch.int32, "err_count")
    nbytes = int(load().htex_sample_reordered_workspace_bytes(prep.H, Q, pool.channels))
    ws = torch.empty(max(nbytes, 1), dtype=torch.uint8, device=h.device)
    check(load().htex_sample_prepared_reordered(
        prep.H, prep.buf.data_ptr(), C.byref(pool.c), C.byref(q), int(filter), out.data_ptr(),
        ws.data_ptr(), nbytes, err_count.data_ptr() if err_count is not None else None,
        _stream(stream)))
    return out


def htex_sample_aniso(mesh: Mesh, pool: Pool, h, u, v, jac, max_aniso: int = 16, flags=0,
                      out=None, nprobe=False, err_count=None, stream=None):
    """Anisotropic Alg. 3 (the OpenGL anisotropic filter on every fetch);
    jac: float32 [Q, 4] = (du/dx, dv/dx, du/dy, dv/dy).
    -> (out float32 [Q, C], probes int32 [Q] or None)."""
    q, Q = _queries(h, u, v, None)
    _dev(jac, torch.float32, "jac")
    if jac.numel() != 4 * Q:
        raise ValueError("jac must hold 4 floats per query")
    out = _out(out, Q, pool, h.device)
    n = torch.zeros(Q, dtype=torch.int32, device=h.device) if nprobe else None
    if err_count is not None:
        _dev(err_count, torch.int32, "err_count")
    check(load().htex_sample_aniso(C.byref(mesh.c), C.byref(pool.c), C.byref(q), jac.data_ptr(),
                                   int(max_aniso), int(flags), out.data_ptr(),
                                   n.data_ptr() if n is not None else None,
                                   err_count.data_ptr() if err_count is not None else None,
                                   _stream(stream)))
    return out, n


def htex_sample_aniso_prepared(prep: "Prepared", pool: Pool, h, u, v, jac, max_aniso: int = 16,
                               flags=0, out=None, err_count=None, stream=None):
    """htex_sample_aniso from prepared records (bit-identical) -> out [Q, C]."""
    prep.check_pool(pool)
    q, Q = _queries(h, u, v, None)
    _dev(jac, torch.float32, "jac")
    if jac.numel() != 4 * Q:
        raise ValueError("jac must hold 4 floats per query")
    out = _out(out, Q, pool, h.device)
    if err_count is not None:
        _dev(err_count, torch.int32, "err_count")
    check(load().htex_sample_aniso_prepared(prep.H, prep.buf.data_ptr(), C.byref(pool.c),
                                            C.byref(q), jac.data_ptr(), int(max_aniso),
                                            int(flags), out.data_ptr(),
                                            err_count.data_ptr() if err_count is not None
                                            else None, _stream(stream)))
    return out


def _sort_ws(H, Q, device):
    nbytes = int(load().htex_sort_workspace_bytes(int(H), Q))
    return torch.empty(max(nbytes, 1), dtype=torch.uint8, device=device), nbytes


def htex_sort_queries(H: int, h, stream=None):
    """perm (int32 [Q], device): the stable order of the queries by halfedge."""
    h = _dev(h, torch.int32, "h")
    Q = h.numel()
    perm = torch.empty(Q, dtype=torch.int32, device=h.device)
    ws, nbytes = _sort_ws(H, Q, h.device)
    check(load().htex_sort_queries(int(H), Q, h.data_ptr(), perm.data_ptr(), ws.data_ptr(),
                                   nbytes, _stream(stream)))
    return perm


def htex_sort_batch(H: int, h, u, v, footprint=None, stream=None, key=None, nkeys=None):
    """(perm, h, u, v, footprint) of the batch in halfedge order, in one call:
    the last radix pass gathers each sorted row's query as one 16-byte
    record.  With `key` (device int32 [H]) and `nkeys`, the batch is ordered
    by key[h] instead (keys 0 .. nkeys - 1; e.g. a Mesh's `edge` and E, so
    that both halfedges of an edge come together)."""
    q, Q = _queries(h, u, v, footprint)
    perm = torch.empty(Q, dtype=torch.int32, device=h.device)
    ho, uo, vo = torch.empty_like(h), torch.empty_like(u), torch.empty_like(v)
    fo = torch.empty_like(footprint) if footprint is not None else None
    fp = fo.data_ptr() if fo is not None else None
    if key is None:
        ws, nbytes = _sort_ws(H, Q, h.device)
        check(load().htex_sort_batch(int(H), C.byref(q), perm.data_ptr(), ho.data_ptr(),
                                     uo.data_ptr(), vo.data_ptr(), fp, ws.data_ptr(), nbytes,
                                     _stream(stream)))
    else:
        key = _dev(key, torch.int32, "key")
        if key.numel() != H:
            raise ValueError(f"key must hold one value per halfedge ({H}), got {key.numel()}")
        if nkeys is None or int(nkeys) < 1:
            raise ValueError("nkeys (the number of distinct keys, >= 1) is required with key")
        ws, nbytes = _sort_ws(int(nkeys), Q, h.device)
        check(load().htex_sort_batch_by_key(int(H), int(nkeys), key.data_ptr(), C.byref(q),
                                            perm.data_ptr(), ho.data_ptr(), uo.data_ptr(),
                                            vo.data_ptr(), fp, ws.data_ptr(), nbytes,
                                            _stream(stream)))
    return perm, ho, uo, vo, fo


def htex_permute_queries(perm, h, u, v, footprint=None, stream=None):
    """(h, u, v, footprint) gathered into the order `perm`."""
    q, Q = _queries(h, u, v, footprint)
    _dev(perm, torch.int32, "perm")
    if perm.numel() != Q:
        raise ValueError("perm must hold one index per query")
    ho = torch.empty_like(h)
    uo = torch.empty_like(u)
    vo = torch.empty_like(v)
    fo = torch.empty_like(footprint) if footprint is not None else None
    check(load().htex_permute_queries(C.byref(q), perm.data_ptr(), ho.data_ptr(), uo.data_ptr(),
                                      vo.data_ptr(), fo.data_ptr() if fo is not None else None,
                                      _stream(stream)))
    return ho, uo, vo, fo


def htex_unpermute_results(perm, out_sorted, out=None, stream=None):
    """Results of a permuted batch back in input order (rows of 1 or 4
    floats)."""
    _dev(perm, torch.int32, "perm")
    _dev(out_sorted, torch.float32, "out_sorted")
    Q = perm.numel()
    if out_sorted.dim() != 2 or out_sorted.shape[0] != Q or out_sorted.shape[1] not in (1, 4):
        raise ValueError(f"out_sorted must have shape ({Q}, 1) or ({Q}, 4)")
    ch = int(out_sorted.shape[1])
    if out is None:
        out = torch.empty_like(out_sorted)
    _rows(out, "out", Q, ch)
    check(load().htex_unpermute_results(Q, ch, perm.data_ptr(), out_sorted.data_ptr(),
                                        out.data_ptr(), _stream(stream)))
    return out


def debug_records(dbg: torch.Tensor) -> np.ndarray:
    """Device debug output -> numpy structured array (fields of htex_debug_rec)."""
    a = dbg.cpu().numpy()
    return a.view(DEBUG_DTYPE).reshape(-1)


def htex_sample_backward(mesh: Mesh, pool: Pool, h, u, v, dout, footprint=None,
                         filter=HTEX_BILINEAR, flags=0, dtexels=None, stream=None):
    """dtexels (float32, pool-shaped) += transpose of htex_sample applied to dout."""
    q, Q = _queries(h, u, v, footprint)
    _rows(dout, "dout", Q, pool.channels)
    if dtexels is None:
        dtexels = torch.zeros_like(pool.texels, dtype=torch.float32)
    _rows(dtexels, "dtexels", pool.total, pool.channels)
    check(load().htex_sample_backward(C.byref(mesh.c), C.byref(pool.c), C.byref(q),
                                      int(filter), int(flags), dout.data_ptr(),
                                      dtexels.data_ptr(), _stream(stream)))
    return dtexels


class HtexSample(torch.autograd.Function):
    """Differentiable sampling with respect to a float32 pool's texels.

    forward(texels, mesh, pool, h, u, v, footprint, filter, flags,
    mips_from_level0, prep) -> [Q, C]; the gradient flows to `texels` (which
    must be pool.texels).  With mips_from_level0 the pool's coarser levels
    are taken to be box means of level 0 (rebuild them with htex_build_mips
    after each update): the gradient is folded into level 0 through the
    transposed mip chain and is zero on the coarser levels.  With `prep`
    (htex.Prepared of the mesh and pool) the forward pass reads prepared
    records (same results, faster)."""

    @staticmethod
    def forward(ctx, texels, mesh, pool, h, u, v, footprint=None, filter=HTEX_BILINEAR,
                flags=0, mips_from_level0=False, prep=None):
        if texels.data_ptr() != pool.texels.data_ptr():
            raise ValueError("texels must be pool.texels")
        if prep is not None:
            out = htex_sample_prepared(prep, pool, h, u, v, footprint, filter, flags)
        else:
            out, _ = htex_sample(mesh, pool, h, u, v, footprint, filter, flags)
        ctx.save_for_backward(h, u, v, footprint)
        ctx.mesh, ctx.pool, ctx.filter, ctx.flags = mesh, pool, filter, flags
        ctx.mips = bool(mips_from_level0)
        return out

    @staticmethod
    def backward(ctx, gout):
        h, u, v, footprint = ctx.saved_tensors
        d = htex_sample_backward(ctx.mesh, ctx.pool, h, u, v, gout.contiguous(), footprint,
                                 ctx.filter, ctx.flags)
        if ctx.mips:
            htex_mip_backward(ctx.pool, d, clear_coarse=True)
        return d, None, None, None, None, None, None, None, None, None, None
