"""Texel-pool layout and host-side fills (input generator).

Pool format: one square RGBA texture per edge, resolution n_e = 2^k_e.
Edge e starts at texel offset base[e]; its mip levels follow each other from
the finest (level 0, n_e x n_e) to the coarsest (1 x 1).  Each level is stored
row-major: texel (row j, column i) at j * n + i, 4 channels per texel.
Every base is a multiple of `align` texels.
"""
from __future__ import annotations

import numpy as np

from .texels import texel_values

ALIGN = 16  # texels (256 bytes of float32 RGBA)


def edge_texel_count(k, has_mips: bool):
    k = np.asarray(k, dtype=np.int64)
    if has_mips:
        return ((np.int64(4) << (2 * k)) - 1) // 3
    return np.int64(1) << (2 * k)


def layout(log2res, has_mips: bool, align: int = ALIGN):
    """(base int64[E], total_texels) for the pool format above."""
    cnt = edge_texel_count(log2res, has_mips)
    cnt = (cnt + align - 1) // align * align
    base = np.zeros(len(cnt), dtype=np.int64)
    if len(cnt) > 1:
        np.cumsum(cnt[:-1], out=base[1:])
    total = int(cnt.sum()) if len(cnt) else 0
    return base, total


def fill_level0_host(kind: int, seed: int, log2res, base, total: int,
                     boundary, has_mips: bool, edges=None, channels: int = 4) -> np.ndarray:
    """float32 [total, channels] pool with level 0 of every edge (or of
    `edges`) filled; mip levels and padding are left at zero.  A one-channel
    pool holds channel 0 of the four-channel values."""
    pool = np.zeros((total, channels), dtype=np.float32)
    log2res = np.asarray(log2res)
    es = np.arange(len(log2res)) if edges is None else np.asarray(edges)
    for k in np.unique(log2res[es]):
        sel = es[log2res[es] == k]
        n = 1 << int(k)
        jj, ii = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
        jj = jj.reshape(-1)
        ii = ii.reshape(-1)
        for chunk in np.array_split(sel, max(1, len(sel) * n * n // (1 << 20))):
            if len(chunk) == 0:
                continue
            E_ = chunk[:, None, None]
            vals = texel_values(kind, seed, E_, n, boundary[chunk][:, None, None],
                                ii[None, :, None], jj[None, :, None],
                                np.arange(channels)[None, None, :])
            rows = base[chunk][:, None] + (jj * n + ii)[None, :]
            pool[rows.reshape(-1)] = vals.reshape(-1, channels)
    return pool
