"""ctypes declarations of libhtex's C ABI (include/htex.h).

torch is imported before the library is loaded so that libhtex binds to the
HIP runtime torch already loaded (same soname): device pointers and stream
handles from torch are then valid inside libhtex.  There is no fallback: a
missing library raises.
"""
from __future__ import annotations

import ctypes as C
import os

import torch  # noqa: F401  (must precede loading libhtex, see above)

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libhtex.so")

HTEX_OK = 0
STATUS = {0: "HTEX_OK", -1: "HTEX_E_ARG", -2: "HTEX_E_TOPOLOGY", -3: "HTEX_E_RANGE",
          -4: "HTEX_E_DEVICE", -5: "HTEX_E_UNSUPPORTED", -6: "HTEX_E_BUSY", -7: "HTEX_E_NOMEM"}

HTEX_F32, HTEX_BF16, HTEX_FP8_E4M3 = 0, 1, 2
HTEX_BILINEAR, HTEX_TRILINEAR = 0, 1
HTEX_QUERIES_SORTED = 1
HTEX_QUERIES_SCATTERED = 2


class htex_mesh(C.Structure):
    _fields_ = [("H", C.c_int32), ("E", C.c_int32),
                ("twin", C.c_void_p), ("next", C.c_void_p),
                ("prev", C.c_void_p), ("edge", C.c_void_p)]


class htex_pool(C.Structure):
    _fields_ = [("E", C.c_int32), ("dtype", C.c_int32), ("has_mips", C.c_int32),
                ("max_log2res", C.c_int32), ("channels", C.c_int32), ("reserved", C.c_int32),
                ("total_texels", C.c_int64),
                ("log2res", C.c_void_p), ("base", C.c_void_p),
                ("texels", C.c_void_p), ("scale", C.c_void_p)]


class htex_queries(C.Structure):
    _fields_ = [("Q", C.c_int64), ("h", C.c_void_p), ("u", C.c_void_p),
                ("v", C.c_void_p), ("footprint", C.c_void_p)]


DEBUG_FIELDS = [("next", "<i4"), ("prev", "<i4"), ("edge", "<i4", (3,)),
                ("flip", "<i4", (3,)), ("level", "<i4", (3, 2)), ("i0", "<i4", (3, 2)),
                ("j0", "<i4", (3, 2)), ("inb", "<i4", (3, 2)), ("phi", "<f4"),
                ("W", "<f4"), ("wf", "<f4", (3,)), ("pad", "<i4", (3,))]
DEBUG_BYTES = 160

# every entry point of include/htex.h: name -> (restype, argtypes)
_P = C.c_void_p
SIGNATURES = {
    "htex_last_error": (C.c_char_p, []),
    "htex_status_string": (C.c_char_p, [C.c_int32]),
    "htex_pool_layout": (C.c_int32, [C.c_int32, _P, C.c_int32, _P, _P]),
    "htex_mesh_validate": (C.c_int32, [_P, _P, _P]),
    "htex_build_mips": (C.c_int32, [_P, _P, _P]),
    "htex_corner_average": (C.c_int32, [_P, _P, _P, _P, _P]),
    "htex_mip_backward": (C.c_int32, [_P, _P, C.c_int32, _P]),
    "htex_triangle_vertices": (C.c_int32, [_P, _P, C.c_int32, _P, _P, _P, _P]),
    "htex_quantize": (C.c_int32, [_P, C.c_int32, _P, _P, _P]),
    "htex_sample": (C.c_int32, [_P, _P, _P, C.c_int32, C.c_uint32, _P, _P, _P, _P]),
    "htex_sample_backward": (C.c_int32, [_P, _P, _P, C.c_int32, C.c_uint32, _P, _P, _P]),
    "htex_prepare": (C.c_int32, [_P, _P, _P, _P]),
    "htex_sort_workspace_bytes": (C.c_size_t, [C.c_int32, C.c_int64]),
    "htex_sort_queries": (C.c_int32, [C.c_int32, C.c_int64, _P, _P, _P, C.c_size_t, _P]),
    "htex_sort_batch": (C.c_int32, [C.c_int32, _P, _P, _P, _P, _P, _P, _P, C.c_size_t, _P]),
    "htex_sort_batch_by_key": (C.c_int32, [C.c_int32, C.c_int32, _P, _P, _P, _P, _P, _P, _P, _P,
                                           C.c_size_t, _P]),
    "htex_sort_batch_noalloc": (C.c_int32, [C.c_int32, _P, _P, _P, _P, _P, _P, _P]),
    "htex_permute_queries": (C.c_int32, [_P, _P, _P, _P, _P, _P, _P]),
    "htex_unpermute_results": (C.c_int32, [C.c_int64, C.c_int32, _P, _P, _P, _P]),
    "htex_sample_prepared": (C.c_int32, [C.c_int32, _P, _P, _P, C.c_int32, C.c_uint32, _P, _P,
                                         _P]),
    "htex_sample_reordered_workspace_bytes": (C.c_size_t, [C.c_int32, C.c_int64, C.c_int32]),
    "htex_sample_prepared_reordered": (C.c_int32, [C.c_int32, _P, _P, _P, C.c_int32, _P, _P,
                                                   C.c_size_t, _P, _P]),
    "htex_sample_aniso": (C.c_int32, [_P, _P, _P, _P, C.c_int32, C.c_uint32, _P, _P, _P, _P]),
    "htex_sample_aniso_prepared": (C.c_int32, [C.c_int32, _P, _P, _P, _P, C.c_int32, C.c_uint32,
                                               _P, _P, _P]),
}
HTEX_PREP_BYTES = 48
HTEX_SORT_NOALLOC_MAX_Q = 1 << 20
HTEX_MAX_ANISO = 16


class htex_server_config(C.Structure):
    _fields_ = [("dtype", C.c_int32), ("filter", C.c_int32), ("max_inflight", C.c_int32),
                ("compute_streams", C.c_int32), ("arena_bytes", C.c_int64),
                ("max_batch_queries", C.c_int64), ("grid_blocks", C.c_int32),
                ("max_meshes", C.c_int32), ("copy_streams", C.c_int32), ("channels", C.c_int32),
                ("copy_chunk_queries", C.c_int32), ("reserved", C.c_int32)]


class htex_server_stats(C.Structure):
    _fields_ = [("submitted", C.c_int64), ("completed", C.c_int64), ("rejected", C.c_int64),
                ("batches", C.c_int64), ("queries_done", C.c_int64),
                ("arena_peak_bytes", C.c_int64), ("invalid_queries", C.c_int32),
                ("pad", C.c_int32)]


SIGNATURES.update({
    "htex_server_create": (C.c_int32, [_P, _P]),
    "htex_server_add_mesh": (C.c_int32, [_P, C.c_int32, _P, _P, _P]),
    "htex_server_submit": (C.c_int32, [_P, C.c_int32, C.c_int64, _P, _P, _P, _P, _P, _P]),
    "htex_server_poll": (C.c_int32, [_P, C.c_int32, _P, _P, _P]),
    "htex_server_drain": (C.c_int32, [_P, C.c_double]),
    "htex_server_stats_get": (C.c_int32, [_P, _P]),
    "htex_server_destroy": (C.c_int32, [_P]),
})

_lib = None


class HtexError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


def load() -> C.CDLL:
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(
                f"libhtex.so not found at {LIB_PATH}: build it with "
                "`python -m paper_2207_05618_amd.build` (there is no fallback)")
        L = C.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def check(status: int):
    if status != HTEX_OK:
        msg = load().htex_last_error().decode()
        raise HtexError(status, msg)
