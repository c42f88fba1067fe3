"""Host-side checks of the C ABI: the library loads, exports every entry
point declared in include/htex.h, computes the pool layout, and rejects bad
arguments before launching anything (no GPU needed)."""
import ctypes as C
import os
import re

import numpy as np
import pytest

from htexgen import pool as gpool
from tests.conftest import ROOT

import paper_2207_05618_amd as htex
from paper_2207_05618_amd import _lib


def declared_symbols():
    src = open(os.path.join(ROOT, "include", "htex.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(htex_[a-z_]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    L = _lib.load()
    names = declared_symbols()
    assert len(names) >= 8
    for n in names:
        assert hasattr(L, n), n
    assert set(names) == set(_lib.SIGNATURES)


def test_generator_library_exports_fill():
    import ctypes
    from htexgen import build as gb
    assert ctypes.CDLL(gb.LIB).htexgen_fill_level0


def test_status_strings():
    L = _lib.load()
    for code in range(0, -8, -1):
        assert L.htex_status_string(code).decode() not in ("", "unknown status")
    assert L.htex_status_string(-99).decode() == "unknown status"


@pytest.mark.parametrize("mips", [False, True])
def test_pool_layout_matches_format(mips):
    rng = np.random.default_rng(0)
    lr = rng.integers(0, 8, 500).astype(np.uint8)
    base, total = htex.htex_pool_layout(lr, mips)
    b2, t2 = gpool.layout(lr, mips)
    np.testing.assert_array_equal(base, b2)
    assert total == t2
    assert (base % 16 == 0).all()
    cnt = ((4 << (2 * lr.astype(np.int64))) - 1) // 3 if mips else (1 << (2 * lr.astype(np.int64)))
    assert (np.diff(np.append(base, total)) >= cnt).all()


def test_pool_layout_rejects_oversized_resolution():
    lr = np.array([3, 16], np.uint8)
    with pytest.raises(_lib.HtexError) as ei:
        htex.htex_pool_layout(lr, True)
    assert ei.value.status == -3


def _mesh(H=4, E=2, null=False):
    return _lib.htex_mesh(H, E, None if null else 8, 8, 8, 8)


def _pool(E=2, dtype=0, tex=16, mips=1, maxk=2, scale=None, channels=4, reserved=0):
    return _lib.htex_pool(E, dtype, mips, maxk, channels, reserved, 64, 8, 8, tex, scale)


def _q(Q=1, f=None):
    return _lib.htex_queries(Q, 8, 8, 8, f)


@pytest.mark.parametrize("case, status", [
    ("null_mesh_array", -1), ("E_mismatch", -1), ("bad_dtype", -1), ("misaligned_texels", -1),
    ("fp8_no_scale", -1), ("bad_filter", -1), ("tri_no_footprint", -1), ("tri_no_mips", -1),
    ("neg_Q", -1), ("misaligned_out", -1), ("bad_flags", -1), ("big_k", -3),
    ("bad_channels", -1), ("reserved_set", -1), ("one_channel_misaligned_out", -1),
    ("one_channel_misaligned_texels", -1), ("contradictory_hints", -1),
])
def test_sample_rejects_bad_arguments_without_launching(case, status):
    L = _lib.load()
    mesh, pool, q = _mesh(), _pool(), _q()
    filt, flags, out = 0, 0, 16
    if case == "null_mesh_array":
        mesh = _mesh(null=True)
    elif case == "E_mismatch":
        pool = _pool(E=3)
    elif case == "bad_dtype":
        pool = _pool(dtype=7)
    elif case == "misaligned_texels":
        pool = _pool(tex=24)
    elif case == "fp8_no_scale":
        pool = _pool(dtype=2)
    elif case == "bad_filter":
        filt = 5
    elif case == "tri_no_footprint":
        filt = 1
    elif case == "tri_no_mips":
        filt, pool, q = 1, _pool(mips=0), _q(f=8)
    elif case == "neg_Q":
        q = _q(Q=-1)
    elif case == "misaligned_out":
        out = 20
    elif case == "bad_flags":
        flags = 1 << 7
    elif case == "contradictory_hints":
        flags = _lib.HTEX_QUERIES_SORTED | _lib.HTEX_QUERIES_SCATTERED
    elif case == "big_k":
        pool = _pool(maxk=16)
    elif case == "bad_channels":
        pool = _pool(channels=2)
    elif case == "reserved_set":
        pool = _pool(reserved=1)
    elif case == "one_channel_misaligned_out":
        pool, out = _pool(channels=1), 18
    elif case == "one_channel_misaligned_texels":
        pool = _pool(channels=1, tex=18)
    st = L.htex_sample(C.byref(mesh), C.byref(pool), C.byref(q), filt, flags, out, None, None,
                       None)
    assert st == status
    assert L.htex_last_error().decode() != ""


def test_backward_rejects_quantized_pool():
    L = _lib.load()
    st = L.htex_sample_backward(C.byref(_mesh()), C.byref(_pool(dtype=1, tex=8)),
                                C.byref(_q()), 0, 0, 16, 16, None)
    assert st == -5


def test_quantize_and_mips_argument_checks():
    L = _lib.load()
    assert L.htex_quantize(C.byref(_pool()), 9, 16, 16, None) == -1
    assert L.htex_quantize(C.byref(_pool(dtype=1, tex=8)), 1, 16, None, None) == -1
    assert L.htex_build_mips(C.byref(_pool(mips=0)), 16, None) == -1
    assert L.htex_build_mips(C.byref(_pool()), 32, None) == -1
    assert L.htex_build_mips(C.byref(_pool(dtype=1, tex=8)), 8, None) == -5
    # corner pre-processing: float32 only, in place, pool and mesh must agree
    m = _mesh()
    assert L.htex_corner_average(C.byref(m), C.byref(_pool(dtype=1, tex=8)), 8, None, None) == -5
    assert L.htex_corner_average(C.byref(m), C.byref(_pool()), 32, None, None) == -1
    assert L.htex_corner_average(C.byref(m), C.byref(_pool(E=3)), 16, None, None) == -1
    assert L.htex_corner_average(C.byref(_mesh(null=True)), C.byref(_pool()), 16, None,
                                 None) == -1


def test_product_path_refuses_cpu_tensors():
    import torch
    m = htex
    with pytest.raises(TypeError):
        m._dev(torch.zeros(3, dtype=torch.int32), torch.int32, "h")


def test_aniso_argument_checks():
    L = _lib.load()
    m, q = _mesh(), _q()
    ok_pool = _pool()
    # max_aniso outside [1, 16], no mips, misaligned derivatives, bad flags
    assert L.htex_sample_aniso(C.byref(m), C.byref(ok_pool), C.byref(q), 16, 0, 0, 16, None, None,
                               None) == -1
    assert L.htex_sample_aniso(C.byref(m), C.byref(ok_pool), C.byref(q), 16, 17, 0, 16, None, None,
                               None) == -1
    assert L.htex_sample_aniso(C.byref(m), C.byref(_pool(mips=0)), C.byref(q), 16, 4, 0, 16, None,
                               None, None) == -1
    assert L.htex_sample_aniso(C.byref(m), C.byref(ok_pool), C.byref(q), 24, 4, 0, 16, None, None,
                               None) == -1
    assert L.htex_sample_aniso(C.byref(m), C.byref(ok_pool), C.byref(q), 16, 4, 1 << 5, 16, None,
                               None, None) == -1
    assert L.htex_sample_aniso_prepared(4, 16, C.byref(ok_pool), C.byref(q), 16, 0, 0, 16, None,
                                        None) == -1
    assert L.htex_sample_aniso_prepared(4, 24, C.byref(ok_pool), C.byref(q), 16, 4, 0, 16, None,
                                        None) == -1


@pytest.mark.parametrize("field, value", [("copy_chunk_queries", -1), ("reserved", 1),
                                          ("max_inflight", 0), ("copy_streams", 5),
                                          ("channels", 2)])
def test_server_config_is_checked_before_any_device_call(field, value):
    """A bad serving configuration is refused by argument checks alone."""
    import ctypes as C
    L = _lib.load()
    cfg = _lib.htex_server_config(0, 1, 8, 1, 1 << 20, 1 << 16, 0, 4, 1, 4, 0, 0)
    setattr(cfg, field, value)
    h = C.c_void_p()
    assert L.htex_server_create(C.byref(cfg), C.byref(h)) == -1
    assert not h.value
    assert L.htex_last_error().decode() != ""


def test_sort_argument_checks():
    """Sorting refuses a short or misaligned workspace, outputs that overlap
    the input batch, and oversized batches, before launching."""
    L = _lib.load()
    H, Q = 392, 1000
    need = L.htex_sort_workspace_bytes(H, Q)
    assert need > 0
    # larger H needs more digit passes, hence at least as much workspace
    assert L.htex_sort_workspace_bytes(1 << 30, Q) >= need
    ws = 1 << 20
    assert L.htex_sort_queries(H, Q, 16, 16 << 20, ws, need - 1, None) == -1
    assert L.htex_sort_queries(H, Q, 16, 16 << 20, ws + 4, need, None) == -1
    assert L.htex_sort_queries(H, Q, 16, 16 << 20, None, need, None) == -1
    assert L.htex_sort_queries(H, 1 << 31, 16, 16 << 20, ws, 1 << 40, None) == -3
    # perm inside the workspace
    assert L.htex_sort_queries(H, Q, 16, ws + 256, ws, need, None) == -1
    q = _lib.htex_queries(Q, 1 << 24, 2 << 24, 3 << 24, None)
    outs = [5 << 24, 6 << 24, 7 << 24, 8 << 24]
    # an output aliasing an input array is refused
    assert L.htex_sort_batch(H, C.byref(q), 5 << 24, 1 << 24, 7 << 24, 8 << 24, None, ws, need,
                             None) == -1
    # two outputs overlapping each other
    assert L.htex_sort_batch(H, C.byref(q), 5 << 24, 5 << 24, 7 << 24, 8 << 24, None, ws, need,
                             None) == -1
    # a footprint without f_out
    qf = _lib.htex_queries(Q, 1 << 24, 2 << 24, 3 << 24, 4 << 24)
    assert L.htex_sort_batch(H, C.byref(qf), *outs, None, ws, need, None) == -1
    assert L.htex_last_error().decode() != ""


def test_sort_by_key_argument_checks():
    """The keyed sort refuses a missing or misaligned key map, nkeys < 1,
    outputs that overlap the key map, and a workspace sized for fewer keys,
    before launching."""
    L = _lib.load()
    H, Q, K = 392, 1000, 196
    need = L.htex_sort_workspace_bytes(K, Q)
    ws, key = 1 << 20, 9 << 24
    q = _lib.htex_queries(Q, 1 << 24, 2 << 24, 3 << 24, None)
    outs = [5 << 24, 6 << 24, 7 << 24, 8 << 24]
    f = L.htex_sort_batch_by_key
    assert f(H, 0, key, C.byref(q), *outs, None, ws, need, None) == -1
    assert f(H, K, None, C.byref(q), *outs, None, ws, need, None) == -1
    assert f(H, K, key + 2, C.byref(q), *outs, None, ws, need, None) == -1
    assert f(H, K, 5 << 24, C.byref(q), *outs, None, ws, need, None) == -1
    assert f(H, K, key, C.byref(q), *outs, None, ws, need - 1, None) == -1
    assert f(H, K, key, None, *outs, None, ws, need, None) == -1
    assert "key" in L.htex_last_error().decode() or L.htex_last_error().decode() != ""
    # an empty batch needs nothing
    q0 = _lib.htex_queries(0, None, None, None, None)
    assert f(H, K, key, C.byref(q0), *outs, None, None, 0, None) == 0


def test_sample_reordered_argument_checks():
    """The reordered sampler refuses a short or misaligned workspace, one
    that overlaps the output or the query arrays, and oversized batches,
    before launching; its workspace grows with the batch."""
    L = _lib.load()
    H, Q = 392, 1000
    assert L.htex_sample_reordered_workspace_bytes(H, Q, 3) == 0
    need = L.htex_sample_reordered_workspace_bytes(H, Q, 4)
    assert need >= L.htex_sample_reordered_workspace_bytes(H, Q, 1) > 0
    assert L.htex_sample_reordered_workspace_bytes(H, 10 * Q, 4) > need
    lr = np.full(196, 4, np.uint8)
    base, total = gpool.layout(lr, True)
    pool = _lib.htex_pool(196, 0, 1, 4, 4, 0, total, 1 << 30, 2 << 30, 3 << 30, None)
    q = _lib.htex_queries(Q, 1 << 24, 2 << 24, 3 << 24, 4 << 24)
    f = L.htex_sample_prepared_reordered
    prep, out, ws = 5 << 24, 6 << 24, 8 << 24
    assert f(H, prep, C.byref(pool), C.byref(q), 1, out, ws, need - 1, None, None) == -1
    assert f(H, prep, C.byref(pool), C.byref(q), 1, out, ws + 16, need, None, None) == -1
    assert f(H, prep, C.byref(pool), C.byref(q), 1, out, None, need, None, None) == -1
    assert f(H, prep, C.byref(pool), C.byref(q), 1, ws + 256, ws, need, None, None) == -1
    assert f(H, prep, C.byref(pool), C.byref(q), 1, out, 2 << 24, need, None, None) == -1
    big = _lib.htex_queries(1 << 31, 1 << 24, 2 << 24, 3 << 24, 4 << 24)
    assert f(H, prep, C.byref(pool), C.byref(big), 1, out, ws, 1 << 45, None, None) == -3
    assert L.htex_last_error().decode() != ""


def test_unpermute_checks():
    L = _lib.load()
    # channels must be 1 or 4; rows aligned to their width; no overlap
    assert L.htex_unpermute_results(10, 2, 16, 1 << 20, 2 << 20, None) == -1
    assert L.htex_unpermute_results(10, 4, 16, (1 << 20) + 4, 2 << 20, None) == -1
    assert L.htex_unpermute_results(10, 1, 16, 1 << 20, (1 << 20) + 8, None) == -1
    assert L.htex_last_error().decode() != ""


def test_prepared_records_remember_their_layout():
    """Prepared records are refused for a pool of another layout: the key
    changes with the per-edge resolutions, the mips and the size, but not
    with the storage type."""
    import types
    lr = np.array([4, 5, 4], np.uint8)
    base, total = htex.htex_pool_layout(lr, True)
    k = htex.layout_key(lr, True, total)
    assert k == htex.layout_key(lr.copy(), True, total)
    lr2 = np.array([5, 4, 4], np.uint8)
    assert htex.layout_key(lr2, True, htex.htex_pool_layout(lr2, True)[1]) != k
    assert htex.layout_key(lr, False, htex.htex_pool_layout(lr, False)[1]) != k
    prep = htex.Prepared.__new__(htex.Prepared)
    prep.layout_key = k
    prep.check_pool(types.SimpleNamespace(layout_key=k))
    with pytest.raises(ValueError, match="another pool layout"):
        prep.check_pool(types.SimpleNamespace(layout_key=htex.layout_key(lr2, True, total)))


def test_noalloc_sort_refuses_oversized_batches_on_the_host():
    """The allocation-free sort rejects batches above its scratch limit
    before touching the device."""
    L = _lib.load()
    q = _lib.htex_queries(_lib.HTEX_SORT_NOALLOC_MAX_Q + 1, 1 << 24, 2 << 24, 3 << 24, None)
    assert L.htex_sort_batch_noalloc(392, C.byref(q), 5 << 24, 6 << 24, 7 << 24, 8 << 24, None,
                                     None) == -3
    assert "at most" in L.htex_last_error().decode()
    assert L.htex_sort_batch_noalloc(392, None, 16, 16, 16, 16, None, None) == -1
