"""Device-side texel fill (same values as htexgen.texels, written on the GPU).

torch is imported before libhtexgen is loaded so both share torch's HIP
runtime.
"""
from __future__ import annotations

import ctypes as C
import os

import numpy as np
import torch

from . import build as _build

_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_build.LIB):
            raise ImportError(f"{_build.LIB} missing: run `python -m htexgen.build`")
        L = C.CDLL(_build.LIB)
        L.htexgen_fill_level0.restype = C.c_int
        L.htexgen_fill_level0.argtypes = [C.c_int, C.c_uint64, C.c_int32, C.c_void_p,
                                          C.c_void_p, C.c_void_p, C.c_void_p, C.c_int,
                                          C.c_void_p]
        _lib = L
    return _lib


def fill_level0(texels: torch.Tensor, kind: int, seed: int, log2res: torch.Tensor,
                base: torch.Tensor, boundary) -> None:
    """Write level 0 of every edge into `texels` (float32 [total, C], C = 4 or
    1, device)."""
    assert texels.is_cuda and texels.dtype == torch.float32 and texels.is_contiguous()
    assert texels.dim() == 2 and texels.shape[1] in (1, 4)
    bnd = torch.as_tensor(np.ascontiguousarray(boundary, dtype=np.uint8)).to(texels.device)
    E = int(log2res.numel())
    rc = _load().htexgen_fill_level0(int(kind), int(seed), E, log2res.data_ptr(),
                                     base.data_ptr(), bnd.data_ptr(), texels.data_ptr(),
                                     int(texels.shape[1]), torch.cuda.current_stream().cuda_stream)
    if rc != 0:
        raise RuntimeError(f"htexgen_fill_level0 failed ({rc})")
    torch.cuda.current_stream().synchronize()
