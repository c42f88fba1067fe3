#!/usr/bin/env python3
"""Throughput of batched Htex sampling on one MI355X.

Workload (default, "frame4k"): a seeded closed-sphere polygon mesh of about
194k faces (70% quads, 20% triangles, 10% 5-8-gons, 1% of the faces removed
as holes so 2% of the edges are boundary edges), one 64x64 RGBA float32
texture per edge with its full mip chain (34.8 GB resident in HBM), texels
from seeded Perlin gradient noise; 3840 x 2160 = 8,294,400 queries per step
(uniform halfedge, uniform barycentric point, log2 footprint ~ U[-3.2, -1.2])
sorted by halfedge, trilinear filtering.  A step is one htex_sample call over
one frame batch; eight distinct seeded batches rotate, so each batch comes
back only after seven others have streamed several GB of texel lines through
the caches.  All inputs are resident in HBM before the
timed region.

Printed: one JSON line with samples/s, the roofline of the sampling kernel
(algorithmic bytes per launch / average kernel time from HIP events on the
launch stream, against 8 TB/s), the FP64 CPU oracle's rate on a bounded
sample of the same workload, and extra rates (unsorted queries, BF16 and
FP8 storage of the same pool).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import re
import statistics
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# HIP maps a process's streams onto GPU_MAX_HW_QUEUES hardware queues (4 by
# default) and streams that share a queue run one after the other.  The
# serving leg drives an upload, a download and a compute stream beside
# torch's own, so it asks for 8 (measured: 2.0e9 samples/s with 8 queues,
# 1.27e9 with 4, on the same requests).  Set before anything starts HIP.
if int(os.environ.get("GPU_MAX_HW_QUEUES", "4")) < 8:
    os.environ["GPU_MAX_HW_QUEUES"] = "8"

HBM_PEAK_GBS = 8000.0
METRIC = "Htex filtered samples/s + % HBM roofline; serving p50/p99 request latency"


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def parse():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="frame4k", choices=["frame4k", "tiny"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extra", action="store_true")
    ap.add_argument("--no-bytes", action="store_true",
                    help="skip the exact algorithmic-byte count (roofline left null)")
    ap.add_argument("--no-serve", action="store_true",
                    help="skip the serving benchmark (200 GB of resident meshes)")
    ap.add_argument("--serve-chunk", type=int, default=0,
                    help="serving: copy requests in round-robin chunks of this many queries "
                         "(0: whole requests in arrival order)")
    ap.add_argument("--copy-probe", action="store_true",
                    help="also run a 1 GiB device copy (HBM counter calibration)")
    ap.add_argument("--storage", default="f32", choices=["f32", "bf16", "fp8_e4m3"],
                    help="texel storage of the timed frame's pool (bf16 and fp8_e4m3 "
                         "quantize the float32 pool before timing; the extra legs, whose "
                         "ratios are taken against the float32 frame, are then left out)")
    return ap.parse_args()


# ---------------------------------------------------------------- inputs --

def build_workload(name):
    import numpy as np
    from htexgen.mesh import cube_mesh, sphere_mesh
    from htexgen.queries import uniform_queries
    if name == "frame4k":
        mesh = sphere_mesh(n=183, seed=201)
        k, Q, log2f, kind, tex_seed = 6, 3840 * 2160, (-3.2, -1.2), 2, 202
        qseeds = [203 + 10 * i for i in range(8)]
    else:
        mesh = cube_mesh()
        k, Q, log2f, kind, tex_seed = 4, 65536, (-6.0, 0.0), 0, 102
        qseeds = [103 + 10 * i for i in range(8)]
    batches = [uniform_queries(mesh.H, Q, s, log2f=log2f, sort=True) for s in qseeds]
    unsorted = uniform_queries(mesh.H, Q, qseeds[0], log2f=log2f, sort=False,
                               shuffle_seed=204)
    return mesh, np.full(mesh.E, k, np.uint8), batches, unsorted, kind, tex_seed


def to_dev(q):
    import numpy as np
    import torch
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).to("cuda")
    return (t(q.h), t(q.u), t(q.v), t(q.f))


# ------------------------------------------------------ algorithmic bytes --

def algorithmic_bytes(dbg, h, log2res, base, total, Q, qbytes=16, obytes=16, tbytes=16):
    """Exact bytes one launch must move: queries in (h, u, v and f when
    filtering trilinearly: qbytes), result out (obytes), each distinct
    halfedge/edge record it reads, and each distinct texel (tbytes) under an
    in-bounds filter tap.  Also the distinct 64-byte segments and 128-byte
    lines those texels occupy."""
    import numpy as np
    rec = dbg.view(np.dtype([("next", "<i4"), ("prev", "<i4"), ("edge", "<i4", (3,)),
                             ("flip", "<i4", (3,)), ("level", "<i4", (3, 2)),
                             ("i0", "<i4", (3, 2)), ("j0", "<i4", (3, 2)),
                             ("inb", "<i4", (3, 2)), ("phi", "<f4"), ("W", "<f4"),
                             ("wf", "<f4", (3,)), ("pad", "<i4", (3,))])).reshape(-1)
    mark = np.zeros(total, dtype=np.bool_)
    k_all = log2res.astype(np.int64)
    for s in range(3):
        e = rec["edge"][:, s].astype(np.int64)
        k = k_all[e]
        eb = base[e]
        for sl in range(2):
            lv = rec["level"][:, s, sl].astype(np.int64)
            use = lv >= 0
            lvc = np.where(use, lv, 0)
            n = np.left_shift(1, k - lvc)
            lofs = ((4 << (2 * k)) - (4 << (2 * (k - lvc)))) // 3
            i0 = rec["i0"][:, s, sl].astype(np.int64)
            j0 = rec["j0"][:, s, sl].astype(np.int64)
            inb = rec["inb"][:, s, sl]
            for dj in range(2):
                for di in range(2):
                    ok = use & ((inb >> (dj * 2 + di)) & 1).astype(bool)
                    idx = eb + lofs + (j0 + dj) * n + (i0 + di)
                    mark[idx[ok]] = True
    texels = int(np.count_nonzero(mark))
    nz = np.nonzero(mark)[0] * tbytes
    segments = int(len(np.unique(nz >> 6)))      # 64-byte segments
    lines128 = int(len(np.unique(nz >> 7)))      # 128-byte lines
    # Next/Prev of each distinct h; Twin/Edge of each distinct h, Next h, Prev h;
    # log2res/base of each distinct edge
    n_h = len(np.unique(h))
    n_g = len(np.unique(np.concatenate([h, rec["next"], rec["prev"]])))
    n_e = len(np.unique(rec["edge"].reshape(-1)))
    topo = 8 * n_h + 8 * n_g + 9 * n_e
    io = (qbytes + obytes) * Q
    total_bytes = io + topo + tbytes * texels
    return {"bytes": int(total_bytes), "bytes_per_query": total_bytes / Q,
            "io_bytes": int(io), "topo_bytes": int(topo), "distinct_edges": int(n_e),
            "texel_bytes_per_query": tbytes * texels / Q, "unique_texels": texels,
            "unique_64B_segments": segments, "unique_128B_lines": lines128,
            "segment_bytes_per_query": (io + topo + 64 * segments) / Q,
            "line128_bytes_per_query": (io + topo + 128 * lines128) / Q}


def storage_bytes(alg, Q, tbytes, scaled):
    """Algorithmic bytes of the same launch with texels stored in `tbytes`
    bytes each (BF16: 8, FP8: 4 for RGBA), plus one float32 scale per
    distinct edge for FP8."""
    b = alg["io_bytes"] + alg["topo_bytes"] + tbytes * alg["unique_texels"]
    if scaled:
        b += 4 * alg["distinct_edges"]
    return {"bytes": int(b), "bytes_per_query": b / Q,
            "texel_bytes_per_query": tbytes * alg["unique_texels"] / Q}


def kernel_seconds(fn, n=10, warm=3):
    """Average time of one call of fn(i) (one kernel launch) from HIP events
    recorded around each call on the launch stream."""
    import torch
    stream = torch.cuda.current_stream()
    for i in range(warm):
        fn(i)
    torch.cuda.synchronize()
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in range(n)]
    t0 = time.perf_counter()
    for i in range(n):
        evs[i][0].record(stream)
        fn(i)
        evs[i][1].record(stream)
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) / n
    return sum(a.elapsed_time(b) for a, b in evs) / n / 1e3, wall


def roofline_entry(kernel, nbytes, seconds, bound="hbm"):
    achieved = nbytes / seconds / 1e9
    return {"bound": bound, "kernel": kernel, "achieved": achieved, "peak": HBM_PEAK_GBS,
            "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "avg_kernel_us": seconds * 1e6}


# ----------------------------------------------------------- CPU oracle --

def cpu_baseline(mesh, log2res, base, pool_dev, batch, has_mips=True, want_s=10.0):
    """FP64 oracle on a contiguous slice of the sorted frame batch: level-0
    texels of the touched edges come from the generator's device fill, the
    oracle builds their mips itself; median of 5 timed runs after a warm-up,
    on every host core."""
    import numpy as np
    import torch
    import oracle
    cores = len(os.sched_getaffinity(0))
    Qs = min(batch.Q, 200_000)
    lo = (batch.Q - Qs) // 2
    sl = batch.take(np.arange(lo, lo + Qs))
    hs = np.unique(np.concatenate([sl.h, mesh.next[sl.h], mesh.prev[sl.h]]))
    edges = np.unique(mesh.edge[hs])
    remap = np.full(mesh.E, -1, np.int32)
    remap[edges] = np.arange(len(edges), dtype=np.int32)
    lr = log2res[edges]
    from htexgen import pool as gpool
    cbase, ctotal = gpool.layout(lr, has_mips)
    n0 = (1 << lr.astype(np.int64)) ** 2
    T = np.zeros((ctotal, 4), np.float64)
    rows = np.concatenate([base[e] + np.arange(c) for e, c in zip(edges, n0)])
    lvl0 = pool_dev[torch.from_numpy(rows).to(pool_dev.device)].cpu().numpy()
    dst = np.concatenate([cb + np.arange(c) for cb, c in zip(cbase, n0)])
    T[dst] = lvl0
    op = oracle.Pool(lr, cbase, T, has_mips)
    if has_mips:
        op = oracle.Pool(lr, cbase, oracle.build_mips(op), True)
    om = oracle.Mesh(mesh.twin, mesh.next, mesh.prev, remap[mesh.edge], len(edges))
    filt = oracle.TRILINEAR if has_mips else oracle.BILINEAR
    oracle.sample(om, op, sl.h, sl.u, sl.v, sl.f, filter=filt, nthreads=cores)
    t0 = time.perf_counter()
    oracle.sample(om, op, sl.h, sl.u, sl.v, sl.f, filter=filt, nthreads=cores)
    one = time.perf_counter() - t0
    reps = max(1, min(5, int(want_s / max(one, 1e-3))))
    times = [one]
    for _ in range(reps - 1):
        t0 = time.perf_counter()
        oracle.sample(om, op, sl.h, sl.u, sl.v, sl.f, filter=filt, nthreads=cores)
        times.append(time.perf_counter() - t0)
    med = statistics.median(times)
    # and on one core (a fifth of the sample)
    q1 = sl.take(np.arange(Qs // 5))
    one_times = []
    for _ in range(3):
        t0 = time.perf_counter()
        oracle.sample(om, op, q1.h, q1.u, q1.v, q1.f, filter=filt, nthreads=1)
        one_times.append(time.perf_counter() - t0)
    return {"value": Qs / med, "unit": "samples/s", "cores": cores, "kind": "oracle",
            "sample": f"{Qs} consecutive queries of the sorted frame batch "
                      f"({len(edges)} edges, FP64, median of {len(times)} runs)",
            "single_core_value": q1.Q / statistics.median(one_times)}


# ------------------------------------------------------------ precision --

def precision_config3(n_iter=20):
    """Config 3: the tiny cube's 16x16 RGBA float32 pool (no mips) stored as
    float32, BF16 and FP8-E4M3 (per-edge scale), 2^20 seeded queries,
    bilinear, blended in float32.  Per storage type: kernel time from HIP
    events, samples/s and the algorithmic bytes per launch (the 0.2-0.8 MB
    pool stays in the caches, so HBM is not what bounds these launches;
    the roofline entry is reported for completeness)."""
    import numpy as np
    import torch

    import paper_2207_05618_amd as htex
    from htexgen import pool as gpool
    from htexgen.mesh import cube_mesh
    from htexgen.queries import uniform_queries

    m = cube_mesh()
    lr = np.full(m.E, 4, np.uint8)
    base, total = gpool.layout(lr, False)
    T = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    pool = htex.Pool(lr, False, texels=T(gpool.fill_level0_host(0, 102, lr, base, total,
                                                                m.boundary_edges(), False)))
    q = uniform_queries(m.H, 1 << 20, 301)
    dm = htex.Mesh.of(m)
    prep = htex.Prepared(dm, pool)
    h, u, v = T(q.h), T(q.u), T(q.v)
    _, dbg = htex.htex_sample(dm, pool, h, u, v, debug=True)
    alg = algorithmic_bytes(dbg.cpu().numpy(), q.h, lr, base, total, q.Q, qbytes=12)
    del dbg
    out = torch.empty((q.Q, 4), dtype=torch.float32, device="cuda")
    res = {"queries": q.Q, "pool_texels": int(total), "filter": "bilinear"}
    for name, dt, tb in (("f32", htex.HTEX_F32, 16), ("bf16", htex.HTEX_BF16, 8),
                         ("fp8_e4m3", htex.HTEX_FP8_E4M3, 4)):
        p = pool if dt == htex.HTEX_F32 else htex.htex_quantize(pool, dt)
        ks, wall = kernel_seconds(lambda i: htex.htex_sample_prepared(prep, p, h, u, v, out=out),
                                  n=n_iter)
        b = storage_bytes(alg, q.Q, tb, dt == htex.HTEX_FP8_E4M3)
        res[name] = {"samples_per_s": q.Q / ks, "kernel_us": ks * 1e6, "wall_us": wall * 1e6,
                     "pool_bytes": p.nbytes(), "alg_bytes_per_query": b["bytes_per_query"],
                     "roofline": roofline_entry(f"htex::k_sample_prep<{name},bilinear>",
                                                b["bytes"], ks)}
    for name in ("bf16", "fp8_e4m3"):
        res[name]["speedup_vs_f32"] = res[name]["samples_per_s"] / res["f32"]["samples_per_s"]
    return res


# ------------------------------------------------------- differentiation --

def grad_benchmark(steps=200):
    """Differentiation form: the tiny cube with 32x32 RGBA float32 textures,
    8,294,400 queries sorted by halfedge; forward and backward rates with
    N(0,1) upstream gradients, then Adam fitting the textures (start 0.5) to
    the samples of a seeded smooth target pool (MSE)."""
    import numpy as np
    import torch

    import paper_2207_05618_amd as htex
    from htexgen import pool as gpool
    from htexgen.mesh import cube_mesh
    from htexgen.queries import uniform_queries

    m = cube_mesh()
    lr = np.full(m.E, 5, np.uint8)
    dm = htex.Mesh.of(m)
    base, total = gpool.layout(lr, False)
    target = htex.Pool(lr, False, texels=torch.from_numpy(
        gpool.fill_level0_host(2, 401, lr, base, total, m.boundary_edges(), False)).cuda())
    q = uniform_queries(m.H, 3840 * 2160, 405, sort=True)
    T = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    h, u, v = T(q.h), T(q.u), T(q.v)
    y, _ = htex.htex_sample(dm, target, h, u, v)
    tex = torch.full((total, 4), 0.5, dtype=torch.float32, device="cuda")
    pool = htex.Pool(lr, False, texels=tex)
    g = torch.from_numpy(np.random.default_rng(403).standard_normal((q.Q, 4)).astype(
        np.float32)).cuda()
    out = torch.empty_like(y)
    dtex = torch.zeros_like(tex)

    def timed(fn, n=10):
        for _ in range(2):
            fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(n):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / n / 1e3

    S = htex.HTEX_QUERIES_SORTED
    prep = htex.Prepared(dm, pool)
    t_fwd = timed(lambda: htex.htex_sample_prepared(prep, pool, h, u, v, flags=S, out=out))
    t_fwd_plain = timed(lambda: htex.htex_sample(dm, pool, h, u, v, flags=S, out=out))
    t_bwd = timed(lambda: htex.htex_sample_backward(dm, pool, h, u, v, g, flags=S, dtexels=dtex))
    t_bwd_plain = timed(lambda: htex.htex_sample_backward(dm, pool, h, u, v, g, dtexels=dtex))
    tex.requires_grad_(True)
    opt = torch.optim.Adam([tex], lr=0.02)
    losses = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for it in range(steps):
        opt.zero_grad(set_to_none=False)
        o = htex.HtexSample.apply(tex, dm, pool, h, u, v, None, htex.HTEX_BILINEAR, S, False,
                                  prep)
        loss = ((o - y) ** 2).mean()
        loss.backward()
        opt.step()
        if it % 20 == 0 or it == steps - 1:
            losses.append(float(loss.item()))
    torch.cuda.synchronize()
    fit_s = time.perf_counter() - t0
    tex.requires_grad_(False)
    tri = grad_trilinear(m, dm, q, timed, steps)
    return {"queries": q.Q, "edges": int(m.E), "texels": int(total),
            "backward_roofline": backward_roofline(q.Q, total, t_bwd, trilinear=False),
            "forward_samples_per_s": q.Q / t_fwd, "backward_samples_per_s": q.Q / t_bwd,
            "forward_us": t_fwd * 1e6, "forward_plain_us": t_fwd_plain * 1e6,
            "backward_us": t_bwd * 1e6,
            "backward_plain_atomics_us": t_bwd_plain * 1e6,
            "adam_steps": steps, "adam_seconds": fit_s, "loss_first": losses[0],
            "loss_last": losses[-1], "loss_reduction": losses[0] / max(losses[-1], 1e-30),
            "loss_curve_every_20": losses, "trilinear_level0": tri}


def backward_roofline(Q, texels, seconds, trilinear):
    """The backward launch against HBM: per query it reads h, u, v (and the
    footprint) and dL/dout (16 B); the gradient pool is read and written
    once (every texel of these small pools is touched).  The launch is
    bound by LDS float atomics, not by these bytes."""
    per_query = (16 if trilinear else 12) + 16
    b = Q * per_query + 2 * 16 * texels
    achieved = b / seconds / 1e9
    return {"bound": "lds_atomics", "alg_bytes_per_query": b / Q, "alg_bytes": int(b),
            "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS, "avg_kernel_us": seconds * 1e6}


def grad_trilinear(m, dm, q, timed, steps):
    """Trilinear training of level 0: the same cube and queries with 32x32
    textures and their mips, log2 footprints ~ U[-8, 0]; forward, backward,
    the mip-chain transpose, and Adam on level 0 with the mips rebuilt from
    it before every step."""
    import numpy as np
    import torch

    import paper_2207_05618_amd as htex
    from htexgen import pool as gpool

    lr = np.full(m.E, 5, np.uint8)
    base, total = gpool.layout(lr, True)
    T = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    target = htex.Pool(lr, True, texels=T(gpool.fill_level0_host(2, 401, lr, base, total,
                                                                  m.boundary_edges(), True)))
    htex.htex_build_mips(target)
    f = T(np.exp2(np.random.default_rng(406).uniform(-8, 0, q.Q)).astype(np.float32))
    h, u, v = T(q.h), T(q.u), T(q.v)
    S, TRI = htex.HTEX_QUERIES_SORTED, htex.HTEX_TRILINEAR
    y, _ = htex.htex_sample(dm, target, h, u, v, f, filter=TRI)
    tex = torch.full((total, 4), 0.5, dtype=torch.float32, device="cuda")
    pool = htex.Pool(lr, True, texels=tex)
    htex.htex_build_mips(pool)
    g = torch.from_numpy(np.random.default_rng(407).standard_normal((q.Q, 4)).astype(
        np.float32)).cuda()
    out = torch.empty_like(y)
    dtex = torch.zeros_like(tex)
    prep = htex.Prepared(dm, pool)
    t_fwd = timed(lambda: htex.htex_sample_prepared(prep, pool, h, u, v, f, filter=TRI, flags=S,
                                                    out=out))
    t_fwd_plain = timed(lambda: htex.htex_sample(dm, pool, h, u, v, f, filter=TRI, flags=S,
                                                 out=out))
    t_bwd = timed(lambda: htex.htex_sample_backward(dm, pool, h, u, v, g, f, filter=TRI, flags=S,
                                                    dtexels=dtex))
    t_mip = timed(lambda: htex.htex_mip_backward(pool, dtex))
    t_mips = timed(lambda: htex.htex_build_mips(pool))
    tex.requires_grad_(True)
    opt = torch.optim.Adam([tex], lr=0.02)
    losses = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for it in range(steps):
        with torch.no_grad():
            htex.htex_build_mips(pool)
        opt.zero_grad(set_to_none=False)
        o = htex.HtexSample.apply(tex, dm, pool, h, u, v, f, TRI, S, True, prep)
        loss = ((o - y) ** 2).mean()
        loss.backward()
        opt.step()
        if it % 20 == 0 or it == steps - 1:
            losses.append(float(loss.item()))
    torch.cuda.synchronize()
    fit_s = time.perf_counter() - t0
    tex.requires_grad_(False)
    return {"texels": int(total), "forward_us": t_fwd * 1e6,
            "forward_plain_us": t_fwd_plain * 1e6, "backward_us": t_bwd * 1e6,
            "backward_roofline": backward_roofline(q.Q, total, t_bwd, trilinear=True),
            "mip_backward_us": t_mip * 1e6, "build_mips_us": t_mips * 1e6,
            "adam_steps": steps, "adam_seconds": fit_s, "loss_first": losses[0],
            "loss_last": losses[-1], "loss_reduction": losses[0] / max(losses[-1], 1e-30),
            "loss_curve_every_20": losses}


# ---------------------------------------------------------- displacement --

def displacement_benchmark(mesh, dmesh, rgb_step, Q_rgb, T=4, n_iter=10, with_bytes=True):
    """The paper's "RGB + disp" configuration on the frame mesh: besides the
    4K fragment batch (RGBA, trilinear), a vertex stage tessellates every
    intrinsic triangle into T^2 sub-triangles and reads a one-channel 64x64
    float32 displacement map per edge at each patch vertex (bilinear, level
    0), with corners pre-processed so the displaced surface has no cracks.
    Reports the one-off corner pass, the vertex stage alone, and the frame
    with and without it."""
    import numpy as np
    import torch

    import paper_2207_05618_amd as htex
    from htexgen import device as gdev
    from htexgen.queries import tessellated_queries

    lr = np.full(mesh.E, 6, np.uint8)
    disp = htex.Pool(lr, False, htex.HTEX_F32, channels=1)
    gdev.fill_level0(disp.texels, 1, 501, disp.log2res, disp.base, mesh.boundary_edges())
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    htex.htex_corner_average(dmesh, disp)
    e1.record()
    torch.cuda.synchronize()
    corner_ms = e0.elapsed_time(e1)
    prep = htex.Prepared(dmesh, disp)
    q = tessellated_queries(mesh.H, T)
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    h, u, v = dev(q.h), dev(q.u), dev(q.v)
    out = torch.empty((q.Q, 1), dtype=torch.float32, device="cuda")

    def disp_step():
        htex.htex_sample_prepared(prep, disp, h, u, v, None, filter=htex.HTEX_BILINEAR,
                                  flags=htex.HTEX_QUERIES_SORTED, out=out)

    def timed(fn):
        for i in range(3):
            fn(i)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for i in range(n_iter):
            fn(i)
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / n_iter

    t_disp = timed(lambda i: disp_step())
    t_rgb = timed(rgb_step)

    def both(i):
        disp_step()
        rgb_step(i)

    t_both = timed(both)
    # kernel time of the vertex stage alone (HIP events on the launch stream)
    stream = torch.cuda.current_stream()
    e0.record(stream)
    for _ in range(n_iter):
        disp_step()
    e1.record(stream)
    torch.cuda.synchronize()
    k_disp = e0.elapsed_time(e1) / n_iter / 1e3
    # the same vertices in edge order: both triangles of an intrinsic quad (a
    # halfedge and its twin read one texture) back to back, each in patch
    # order (a stable sort, outside the timed region)
    eo = np.argsort(mesh.edge[q.h], kind="stable")
    he, ue, ve = dev(q.h[eo]), dev(q.u[eo]), dev(q.v[eo])
    for _ in range(3):
        htex.htex_sample_prepared(prep, disp, he, ue, ve, None, filter=htex.HTEX_BILINEAR,
                                  flags=htex.HTEX_QUERIES_SORTED, out=out)
    torch.cuda.synchronize()
    e0.record(stream)
    for _ in range(n_iter):
        htex.htex_sample_prepared(prep, disp, he, ue, ve, None, filter=htex.HTEX_BILINEAR,
                                  flags=htex.HTEX_QUERIES_SORTED, out=out)
    e1.record(stream)
    torch.cuda.synchronize()
    k_disp_edge = e0.elapsed_time(e1) / n_iter / 1e3
    del he, ue, ve
    res = {"tessellation": T, "vertex_queries": int(q.Q), "fragment_queries": int(Q_rgb),
           "displacement_pool_bytes": disp.nbytes(), "corner_preprocess_ms": corner_ms,
           "vertex_stage_ms": t_disp * 1e3, "vertex_stage_kernel_us": k_disp * 1e6,
           "vertex_samples_per_s": q.Q / t_disp, "rgb_only_ms": t_rgb * 1e3,
           "rgb_plus_disp_ms": t_both * 1e3, "rgb_plus_disp_over_rgb": t_both / t_rgb,
           "vertex_stage_edge_order_kernel_us": k_disp_edge * 1e6}
    if with_bytes:
        _, dbg = htex.htex_sample(dmesh, disp, h, u, v, None, filter=htex.HTEX_BILINEAR,
                                  debug=True)
        dbg_host = dbg.cpu().numpy()
        del dbg
        alg = algorithmic_bytes(dbg_host, q.h, lr, disp.base_host, disp.total, q.Q,
                                qbytes=12, obytes=4, tbytes=4)
        achieved = alg["bytes"] / k_disp / 1e9
        res["roofline"] = {"bound": "hbm", "kernel": "htex::k_sample_prep<f32,1ch,bilinear>",
                           "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                           "frac": achieved / HBM_PEAK_GBS,
                           "alg_bytes_per_query": alg["bytes_per_query"],
                           "alg_texel_bytes_per_query": alg["texel_bytes_per_query"],
                           "line128_bytes_per_query": alg["line128_bytes_per_query"],
                           "edge_order_frac": alg["bytes"] / k_disp_edge / 1e9 / HBM_PEAK_GBS}
    del disp, prep, h, u, v, out
    torch.cuda.empty_cache()
    return res


# ------------------------------------------------------- rasterized view --

def raster_benchmark(mesh, dmesh, prep, pool, n_iter=10):
    """A rendered 4K view of the frame mesh instead of synthetic queries:
    the intrinsic triangles (Alg. 1) on the device, then a software
    rasterizer on the host gives one query per covered pixel with its
    perspective-correct (u, v) and screen derivatives.  Trilinear (footprint
    = the longer derivative) and anisotropic sampling, in scanline order and
    in halfedge order."""
    import numpy as np
    import torch

    import paper_2207_05618_amd as htex
    from htexgen.raster import rasterize, sphere_view

    T = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    vert, pos = T(mesh.vert), T(mesh.positions.astype(np.float32))
    htex.htex_triangle_vertices(dmesh, vert, pos)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    tri = htex.htex_triangle_vertices(dmesh, vert, pos)
    e1.record()
    torch.cuda.synchronize()
    alg1_us = e0.elapsed_time(e1) * 1e3
    t0 = time.perf_counter()
    cam = sphere_view()
    fr = rasterize(tri.cpu().numpy().astype(np.float64), cam)
    raster_s = time.perf_counter() - t0
    f = fr.footprint()
    order = np.argsort(fr.h, kind="stable")
    scan = (T(fr.h), T(fr.u), T(fr.v), T(f), T(fr.jac))
    srt = (T(fr.h[order]), T(fr.u[order]), T(fr.v[order]), T(f[order]), T(fr.jac[order]))
    out = torch.empty((fr.Q, 4), dtype=torch.float32, device="cuda")
    TRI, S = htex.HTEX_TRILINEAR, htex.HTEX_QUERIES_SORTED

    def timed(fn, n=20):
        # two HIP events around n launches queued back to back: a launch
        # takes about 0.1 ms here, and events around each launch (or a host
        # clock) also count the time the host spends issuing it
        for _ in range(3):
            fn()
        torch.cuda.synchronize()
        stream = torch.cuda.current_stream()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(n):
            fn()
        e1.record(stream)
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / n / 1e3

    res = {"width": cam.width, "height": cam.height, "queries": int(fr.Q),
           "coverage": fr.Q / (cam.width * cam.height),
           "visible_halfedges": int(len(np.unique(fr.h))), "alg1_kernel_us": alg1_us,
           "host_raster_s": raster_s,
           "log2_footprint_p5_p50_p95": [float(x) for x in np.percentile(np.log2(f), [5, 50, 95])]}
    for name, (h, u, v, ff, jac), flags in (("scanline", scan, 0), ("halfedge_order", srt, S)):
        t_tri = timed(lambda: htex.htex_sample_prepared(prep, pool, h, u, v, ff, filter=TRI,
                                                        flags=flags, out=out))
        t_an = timed(lambda: htex.htex_sample_aniso_prepared(prep, pool, h, u, v, jac,
                                                             flags=flags, out=out))
        res[name] = {"trilinear_samples_per_s": fr.Q / t_tri, "trilinear_ms": t_tri * 1e3,
                     "aniso_samples_per_s": fr.Q / t_an, "aniso_ms": t_an * 1e3}
    j = fr.jac.astype(np.float64)
    px, py = np.hypot(j[:, 0], j[:, 1]), np.hypot(j[:, 2], j[:, 3])
    with np.errstate(divide="ignore"):
        res["mean_probes"] = float(np.minimum(np.ceil(np.maximum(px, py) / np.minimum(px, py)),
                                              16).mean())
    del scan, srt, out, tri
    return res


# ------------------------------------------------------------ anisotropy --

def aniso_benchmark(prep, pool, batches, dev_batches, Q, max_aniso=16, n_iter=10):
    """Anisotropic filtering on the frame (Section 5.1, Fig. 7): the frame's
    queries with elliptic footprints whose minor axis is the query's
    isotropic footprint and whose major axis is longer by a log-uniform
    factor in [1, 16] (grazing views), up to 16 probes per query."""
    import numpy as np
    import torch

    import paper_2207_05618_amd as htex
    from htexgen.queries import aniso_jacobians

    jacs = [torch.from_numpy(aniso_jacobians(b.Q, 601 + i, b.f)).cuda()
            for i, b in enumerate(batches)]
    out = torch.empty((Q, 4), dtype=torch.float32, device="cuda")

    def step(i):
        h, u, v, _ = dev_batches[i % len(dev_batches)]
        htex.htex_sample_aniso_prepared(prep, pool, h, u, v, jacs[i % len(jacs)],
                                        max_aniso=max_aniso, flags=htex.HTEX_QUERIES_SORTED,
                                        out=out)

    for i in range(3):
        step(i)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(n_iter):
        step(i)
    torch.cuda.synchronize()
    t = (time.perf_counter() - t0) / n_iter
    # mean probe count of the batches (the filter's rule: ceil of the axis
    # ratio, at most max_aniso)
    n_sum = 0.0
    for jb in jacs:
        px = torch.sqrt(jb[:, 0] * jb[:, 0] + jb[:, 1] * jb[:, 1])
        py = torch.sqrt(jb[:, 2] * jb[:, 2] + jb[:, 3] * jb[:, 3])
        r = torch.maximum(px, py) / torch.minimum(px, py)
        n_sum += float(torch.clamp(torch.ceil(r), max=max_aniso).mean())
    n_mean = n_sum / len(jacs)
    res = {"max_aniso": max_aniso, "ratio_range": [1, 16], "queries": Q,
           "ms_per_frame": t * 1e3, "samples_per_s": Q / t, "mean_probes": n_mean,
           "probe_samples_per_s": Q * n_mean / t}
    del jacs, out
    return res


# -------------------------------------------------------------- serving --

def _gen_sphere(args):
    n, seed = args
    from htexgen.mesh import sphere_mesh
    m = sphere_mesh(n=n, seed=seed)
    return (m.twin, m.next, m.prev, m.edge, m.E, m.F, m.boundary_edges())


def _bf16_pool_chunked(htex, gdev, log2res, boundary, seed, chunk_texels=1 << 29):
    """BF16 pool with mips filled on the device in float32 chunks of edges
    (fill, box mips, quantize, copy), so the float32 copy never exists
    whole."""
    import numpy as np
    import torch
    big = htex.Pool(log2res, True, htex.HTEX_BF16)
    E = len(log2res)
    base = big.base_host
    e0 = 0
    ci = 0
    while e0 < E:
        e1 = max(e0 + 1, int(np.searchsorted(base, base[e0] + chunk_texels)))
        e1 = min(e1, E)
        sub = htex.Pool(log2res[e0:e1], True, htex.HTEX_F32)
        gdev.fill_level0(sub.texels, 1, seed * 4096 + ci, sub.log2res, sub.base, boundary[e0:e1])
        htex.htex_build_mips(sub)
        q = htex.htex_quantize(sub, htex.HTEX_BF16)
        big.texels[base[e0]:base[e0] + sub.total].copy_(q.texels)
        del sub, q
        e0 = e1
        ci += 1
    torch.cuda.synchronize()
    return big


def serve_meshes(seed=501):
    """The 16 serving meshes (5k-500k faces, log-uniform), generated in worker
    processes; called before this process touches the GPU."""
    import multiprocessing as mp
    from concurrent.futures import ProcessPoolExecutor

    import numpy as np
    rng = np.random.default_rng(seed)
    faces = np.exp(rng.uniform(np.log(5e3), np.log(5e5), 16))
    ns = np.maximum(4, np.round(np.sqrt(faces * 1.025 / 6 / 0.99))).astype(int)
    workers = max(1, min(16, len(os.sched_getaffinity(0))))
    with ProcessPoolExecutor(max_workers=workers, mp_context=mp.get_context("spawn")) as ex:
        return list(ex.map(_gen_sphere, [(int(n), seed * 100 + i) for i, n in enumerate(ns)]))


def serve_benchmark(meshes, seed=501, target_bytes=200e9, rates=(0.3, 0.6, 0.9), run_s=2.0,
                    chunk=0):
    """Serving form: 16 resident meshes (5k-500k faces, log-uniform) with
    BF16 textures + mips sized to about 200 GB, Poisson streams of requests
    of 4k-2M queries (log-uniform, frame-like, sorted by halfedge) to random
    meshes at 0.3 / 0.6 / 0.9 of the measured capacity (the smaller of a burst's
    rate and the rate sustained under overload)."""
    import numpy as np
    import torch

    import paper_2207_05618_amd as htex
    from htexgen import device as gdev
    from htexgen.queries import uniform_queries
    from paper_2207_05618_amd.serve import Server

    t0 = time.perf_counter()
    rng = np.random.default_rng(seed + 1)
    # per-mesh resolution from 16^2 .. 128^2, downgraded on the largest
    # meshes to reach the budget
    ks = rng.choice([4, 5, 6, 7], 16)

    def bytes_of(i, k):
        return htex.htex_pool_layout(np.full(meshes[i][4], k, np.uint8), True)[1] * 8

    while sum(bytes_of(i, ks[i]) for i in range(16)) > target_bytes * 1.05:
        i = int(np.argmax([bytes_of(i, ks[i]) if ks[i] > 4 else -1 for i in range(16)]))
        ks[i] -= 1
    while True:
        tot = sum(bytes_of(i, ks[i]) for i in range(16))
        cands = [i for i in range(16) if ks[i] < 7
                 and tot - bytes_of(i, ks[i]) + bytes_of(i, ks[i] + 1) <= target_bytes * 1.05]
        if tot >= target_bytes * 0.95 or not cands:
            break
        i = min(cands, key=lambda j: bytes_of(j, ks[j]))
        ks[i] += 1
    resident = []
    for i, (tw, nx, pv, ed, E, F, bnd) in enumerate(meshes):
        dm = htex.Mesh(tw, nx, pv, ed, E)
        pool = _bf16_pool_chunked(htex, gdev, np.full(E, ks[i], np.uint8), bnd, seed * 100 + i)
        prep = htex.Prepared(dm, pool)
        resident.append((dm, pool, prep, len(tw)))
    torch.cuda.synchronize()
    pool_bytes = sum(r[1].nbytes() for r in resident)
    log(f"serve: {pool_bytes / 1e9:.1f} GB BF16 resident ({time.perf_counter() - t0:.1f}s)")

    # request payloads (page-locked), reused by the streams
    P = Server.pinned
    payloads = []
    for j in range(48):
        mid = int(rng.integers(0, 16))
        Q = int(np.exp(rng.uniform(np.log(4096), np.log(2097152))))
        q = uniform_queries(resident[mid][3], Q, seed * 1000 + j, log2f=(-3.2, -1.2), sort=True)
        payloads.append((mid, Q, P(q.h, torch.int32), P(q.u, torch.float32),
                         P(q.v, torch.float32), P(q.f, torch.float32),
                         torch.empty((Q, 4), dtype=torch.float32, pin_memory=True)))
    mean_q = float(np.mean([p[1] for p in payloads]))
    log(f"serve: 48 payloads, mean {mean_q:.0f} queries ({time.perf_counter() - t0:.1f}s)")

    def sequential(js, res):
        """One request at a time: copy in, sample, copy out, wait (no
        batching).  Returns (samples/s, latencies, results)."""
        lat, outs = [], {}
        for j in js:
            mid, Q, h, u, v, f, _ = payloads[j]
            _, pool, prep, _ = res[mid]
            ts = time.perf_counter()
            dh, du, dv, df = (x.to("cuda", non_blocking=True) for x in (h, u, v, f))
            o = htex.htex_sample_prepared(prep, pool, dh, du, dv, df, filter=htex.HTEX_TRILINEAR,
                                          flags=htex.HTEX_QUERIES_SORTED)
            oh = torch.empty((Q, 4), dtype=torch.float32, pin_memory=True)
            oh.copy_(o, non_blocking=True)
            torch.cuda.synchronize()
            lat.append(time.perf_counter() - ts)
            outs[j] = oh
        return sum(payloads[j][1] for j in js) / sum(lat), lat, outs

    seq_rate, seq_lat, alone = sequential(range(16), resident)

    # Against plain FP32 on the same GPU: the same meshes and resolutions
    # with float32 texels take twice the bytes, so the comparison runs on
    # the meshes whose float32 pools fit the same budget (smallest first),
    # with the payloads that name them: BF16 served (capacity) and one at a
    # time, then float32 served and one at a time.
    f32_bytes = [2 * r[1].nbytes() for r in resident]
    subset, acc = [], 0
    for i in np.argsort(f32_bytes):
        if acc + f32_bytes[i] <= target_bytes:
            subset.append(int(i))
            acc += f32_bytes[i]
    js = [j for j in range(48) if payloads[j][0] in subset]
    cmp = {"meshes": subset, "f32_resident_bytes": acc, "requests": len(js)}
    if js:
        cmp["bf16_sequential_samples_per_s"] = sequential(js[:16], resident)[0]

    srv = Server(htex.HTEX_BF16, htex.HTEX_TRILINEAR, arena_bytes=4 << 30, max_inflight=64,
                 compute_streams=1, copy_streams=1, max_batch_queries=1 << 22, max_meshes=16,
                 copy_chunk_queries=chunk)
    for dm, pool, prep, _ in resident:
        srv.add_mesh(prep, pool)

    def submit(j, server=None):
        mid, Q, h, u, v, f, out = payloads[j]
        return (server or srv).submit(mid, h, u, v, f, out)

    def burst(server, js, reps=2):
        """Saturation: the faster of `reps` timed bursts of 3 x js requests,
        after one untimed burst that warms the server (events, arena pages,
        copy queues; the first burst on a fresh box can run slow while the
        host and link settle)."""
        for j in js:
            submit(j, server)
        server.drain(300)
        for rid, _ in server.poll(1 << 16):
            server.release(rid)
        best = 0.0
        for rep in range(reps):
            tb = time.perf_counter()
            for r in range(3):
                for j in js:
                    submit(j, server)
            server.drain(300)
            best = max(best, 3 * sum(payloads[j][1] for j in js) / (time.perf_counter() - tb))
            for rid, _ in server.poll(1 << 16):
                server.release(rid)
        return best

    sat_rate = burst(srv, range(48))
    same = all(np.array_equal(payloads[j][6].numpy(), alone[j].numpy()) for j in range(16))
    log(f"serve: burst {sat_rate:.3e} samples/s; sequential {seq_rate:.3e}; "
        f"mix==alone {same}")

    def poisson(lam):
        """Poisson arrivals at lam requests/s for run_s seconds; returns the
        achieved samples/s (until the last result), the latencies and the
        request sizes (in completion order)."""
        arr = np.cumsum(rng.exponential(1.0 / lam, size=int(lam * run_s) + 1))
        arr = arr[arr < run_s]
        picks = rng.integers(0, 48, size=len(arr))
        start = time.perf_counter()
        nq = 0
        size_of = {}
        for a, j in zip(arr, picks):
            while time.perf_counter() - start < a:
                pass
            size_of[submit(int(j))] = payloads[int(j)][1]
            nq += payloads[int(j)][1]
        srv.drain(300)
        wall = time.perf_counter() - start
        done = srv.poll(1 << 20)
        lat = np.array([l for _, l in done])
        sizes = np.array([size_of[rid] for rid, _ in done])
        for rid, _ in done:
            srv.release(rid)
        return nq / wall, lat, len(arr), sizes

    # request-size classes: deciles of the payloads' sizes (log-uniform
    # over 4k-2M queries)
    size_edges = np.quantile([p[1] for p in payloads], np.linspace(0, 1, 11))

    def by_size(lat, sizes):
        rows = []
        for d in range(10):
            lo, hi = size_edges[d], size_edges[d + 1]
            sel = (sizes >= lo) & ((sizes <= hi) if d == 9 else (sizes < hi))
            if sel.any():
                rows.append({"decile": d + 1, "queries_lo": int(lo), "queries_hi": int(hi),
                             "requests": int(sel.sum()),
                             "p50_ms": float(np.percentile(lat[sel], 50) * 1e3),
                             "p99_ms": float(np.percentile(lat[sel], 99) * 1e3)})
        return rows

    # sustained capacity: arrivals offered 25% above the burst rate keep the
    # server busy for the whole run; a burst of queued requests batches more
    # than a stream of arrivals does, so the loads below are set against the
    # smaller of the two
    sustained, _, _, _ = poisson(1.25 * sat_rate / mean_q)
    capacity = min(sat_rate, sustained)
    log(f"serve: sustained {sustained:.3e} samples/s under overload; capacity {capacity:.3e}")
    out = {"resident_bytes": pool_bytes, "meshes": 16,
           "faces": int(sum(m[5] for m in meshes)), "edges": int(sum(m[4] for m in meshes)),
           "log2res": [int(k) for k in ks], "mean_queries_per_request": mean_q,
           "saturation_samples_per_s": capacity, "burst_samples_per_s": sat_rate,
           "sustained_samples_per_s": sustained, "sequential_samples_per_s": seq_rate,
           "sequential_p50_ms": float(np.percentile(seq_lat, 50) * 1e3),
           "speedup_vs_sequential": capacity / seq_rate, "results_mix_equal_alone": bool(same),
           "rates": []}
    lam_sat = capacity / mean_q
    for frac in rates:
        lam = frac * lam_sat
        achieved, lat, nreq, sizes = poisson(lam)
        rec = {"load": frac, "requests": int(nreq), "offered_req_per_s": lam,
               "achieved_samples_per_s": achieved,
               "p50_ms": float(np.percentile(lat, 50) * 1e3),
               "p99_ms": float(np.percentile(lat, 99) * 1e3),
               "by_request_size": by_size(lat, sizes)}
        out["rates"].append(rec)
        log(f"serve: load {frac}: {nreq} requests, p50 {rec['p50_ms']:.2f} ms, "
            f"p99 {rec['p99_ms']:.2f} ms, {rec['achieved_samples_per_s']:.3e} samples/s")
    st = srv.stats()
    out["batches"] = st["batches"]
    out["arena_peak_bytes"] = st["arena_peak_bytes"]
    out["copy_chunk_queries"] = chunk

    if js:
        cmp["bf16_served_samples_per_s"] = burst(srv, js)
    srv.close()
    srv = None      # the server object kept its meshes' pools alive
    del alone
    for i in range(16):
        if i not in subset:
            resident[i] = None
    torch.cuda.empty_cache()
    for i in subset:
        dm, pool, prep, H = resident[i]
        resident[i] = None
        del pool, prep
        torch.cuda.empty_cache()
        E = meshes[i][4]
        p32 = htex.Pool(np.full(E, ks[i], np.uint8), True, htex.HTEX_F32)
        gdev.fill_level0(p32.texels, 1, seed * 100 + i, p32.log2res, p32.base, meshes[i][6])
        htex.htex_build_mips(p32)
        resident[i] = (dm, p32, htex.Prepared(dm, p32), H)
    torch.cuda.synchronize()
    if js:
        srv32 = Server(htex.HTEX_F32, htex.HTEX_TRILINEAR, arena_bytes=4 << 30, max_inflight=64,
                       compute_streams=1, copy_streams=1, max_batch_queries=1 << 22,
                       max_meshes=16, copy_chunk_queries=chunk)
        ids = {}
        for i in subset:
            ids[i] = srv32.add_mesh(resident[i][2], resident[i][1])
        # the server numbers meshes in registration order: remap the payloads
        remapped = {j: (ids[payloads[j][0]],) + payloads[j][1:] for j in js}
        saved = {j: payloads[j] for j in js}
        for j in js:
            payloads[j] = remapped[j]
        cmp["f32_served_samples_per_s"] = burst(srv32, js)
        srv32.close()
        for j in js:
            payloads[j] = saved[j]
        cmp["f32_sequential_samples_per_s"] = sequential(js[:16], resident)[0]
        cmp["served_bf16_over_sequential_f32"] = (cmp["bf16_served_samples_per_s"] /
                                                   cmp["f32_sequential_samples_per_s"])
        cmp["served_f32_over_sequential_f32"] = (cmp["f32_served_samples_per_s"] /
                                                  cmp["f32_sequential_samples_per_s"])
        log(f"serve vs plain f32: {json.dumps(cmp)}")
    out["vs_plain_f32"] = cmp
    del resident, payloads
    torch.cuda.empty_cache()
    return out


# ------------------------------------------------------------- profiles --

def kernel_source_sha256():
    """Hash of the sources the frame kernel is built from (its file and the
    device building blocks it includes)."""
    h = hashlib.sha256()
    for f in ("htex_sample.hip", "htex_filter.h"):
        h.update(open(os.path.join(ROOT, "paper_2207_05618_amd", "csrc", f), "rb").read())
    return h.hexdigest()


def recorded_traffic():
    """HBM traffic per launch from the committed rocprofv3 counter summary,
    if it was taken on the current kernel sources; else None."""
    path = os.path.join(ROOT, "profiles", "k_sample_prep_frame4k_pmc.md")
    if not os.path.exists(path):
        return None
    txt = open(path).read()
    m = re.search(r"kernel_source_sha256:\s*([0-9a-f]{64})", txt)
    b = re.search(r"traffic_bytes_per_launch:\s*([0-9.e+]+)", txt)
    if not m or not b:
        return None
    return float(b.group(1)) if kernel_source_sha256() == m.group(1) else None


# ----------------------------------------------------------------- main --

def main():
    args = parse()
    if args.storage != "f32":
        args.no_extra = True
    if args.gpus != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path; "
              "run with --gpus 1", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch
    import paper_2207_05618_amd as htex
    from htexgen import device as gdev

    t_start = time.perf_counter()
    smeshes = None
    if not args.no_serve and args.workload == "frame4k":
        smeshes = serve_meshes()
        log(f"serve meshes: {sum(m[5] for m in smeshes)} faces "
            f"({time.perf_counter() - t_start:.1f}s)")
    mesh, log2res, batches, unsorted, kind, tex_seed = build_workload(args.workload)
    log(f"mesh H={mesh.H} E={mesh.E} F={mesh.F}; {len(batches)} batches of {batches[0].Q}"
        f" queries ({time.perf_counter() - t_start:.1f}s)")
    dmesh = htex.Mesh.of(mesh)
    pool = htex.Pool(log2res, True, htex.HTEX_F32)
    gdev.fill_level0(pool.texels, kind, tex_seed, pool.log2res, pool.base,
                     mesh.boundary_edges())
    htex.htex_build_mips(pool)
    torch.cuda.synchronize()
    log(f"pool {pool.nbytes() / 1e9:.2f} GB filled + mips ({time.perf_counter() - t_start:.1f}s)")
    prep = htex.Prepared(dmesh, pool)       # per (mesh, pool layout), like the mips
    STORAGE = {"f32": (htex.HTEX_F32, 16), "bf16": (htex.HTEX_BF16, 8),
               "fp8_e4m3": (htex.HTEX_FP8_E4M3, 4)}
    st_dtype, st_texel_bytes = STORAGE[args.storage]
    tpool = pool if args.storage == "f32" else htex.htex_quantize(pool, st_dtype)
    torch.cuda.synchronize()
    dev_batches = [to_dev(b) for b in batches]
    Q = batches[0].Q
    out = torch.empty((Q, 4), dtype=torch.float32, device="cuda")
    stream = torch.cuda.current_stream()

    # device-to-device copy rate of 1 GiB (the practical HBM ceiling, and the
    # calibration kernel of the committed counter summaries)
    x = torch.empty(1 << 28, dtype=torch.float32, device="cuda")
    y = torch.empty_like(x)
    y.copy_(x)
    torch.cuda.synchronize()
    if args.copy_probe:
        copy_gbs = None
    else:
        ce0, ce1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        for _ in range(5):
            y.copy_(x)
        ce0.record(stream)
        for _ in range(30):
            y.copy_(x)
        ce1.record(stream)
        torch.cuda.synchronize()
        copy_gbs = 30 * 2 * x.numel() * 4 / (ce0.elapsed_time(ce1) / 1e3) / 1e9
    del x, y

    def step(i, p=tpool, bs=dev_batches, flags=htex.HTEX_QUERIES_SORTED):
        h, u, v, f = bs[i % len(bs)]
        htex.htex_sample_prepared(prep, p, h, u, v, f, filter=htex.HTEX_TRILINEAR,
                                  flags=flags, out=out)

    for i in range(args.warmup):
        step(i)
    torch.cuda.synchronize()
    evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
           for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for i in range(args.steps):
        evs[i][0].record(stream)
        step(i)
        evs[i][1].record(stream)
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t0
    kern_ms = [a.elapsed_time(b) for a, b in evs]
    avg_kernel_s = sum(kern_ms) / len(kern_ms) / 1e3
    median_kernel_s = statistics.median(kern_ms) / 1e3
    value = args.steps * Q / elapsed
    log(f"{args.steps} steps in {elapsed * 1e3:.2f} ms; kernel avg {avg_kernel_s * 1e6:.1f} us")

    alg = None
    if not args.no_bytes:
        h, u, v, f = dev_batches[0]
        _, dbg = htex.htex_sample(dmesh, pool, h, u, v, f, filter=htex.HTEX_TRILINEAR,
                                  debug=True)
        dbg_host = dbg.cpu().numpy()
        del dbg
        alg = algorithmic_bytes(dbg_host, batches[0].h, log2res, pool.base_host, pool.total, Q)
        del dbg_host
        torch.cuda.empty_cache()

    def rate(p, bs, n=10, flags=htex.HTEX_QUERIES_SORTED):
        for i in range(3):
            step(i, p, bs, flags)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        for i in range(n):
            step(i, p, bs, flags)
        torch.cuda.synchronize()
        return n * Q / (time.perf_counter() - t1)

    extra = {}
    if not args.no_extra:
        # the unsorted batch with the scattered hint: the kernel that reads
        # in-bounds taps only
        extra["unsorted_samples_per_s"] = rate(pool, [to_dev(unsorted)],
                                               flags=htex.HTEX_QUERIES_SCATTERED)
        if args.workload == "frame4k":
            # footprints over the whole mip range, log2 f ~ U[-8, 0]
            from htexgen.queries import uniform_queries
            stress = [to_dev(uniform_queries(mesh.H, Q, 205 + i, log2f=(-8.0, 0.0), sort=True))
                      for i in range(2)]
            extra["full_mip_range_samples_per_s"] = rate(pool, stress)
            del stress
            # one GPU's share of the frame on eight GPUs: a contiguous eighth
            # of each sorted batch
            share = [tuple(a[:Q // 8].contiguous() if a is not None else None for a in b)
                     for b in dev_batches]
            out8 = out[:Q // 8]

            def share_step(i):
                h, u, v, f = share[i % len(share)]
                htex.htex_sample_prepared(prep, pool, h, u, v, f, filter=htex.HTEX_TRILINEAR,
                                          flags=htex.HTEX_QUERIES_SORTED, out=out8)

            for i in range(3):
                share_step(i)
            torch.cuda.synchronize()
            t1 = time.perf_counter()
            for i in range(20):
                share_step(i)
            torch.cuda.synchronize()
            t_share = (time.perf_counter() - t1) / 20
            extra["one_of_eight_share"] = {"queries": Q // 8, "us": t_share * 1e6,
                                           "samples_per_s": (Q // 8) / t_share}
            del share, out8
        # unsorted batch put in halfedge order first: as three calls (one
        # sorts the batch with its queries, one samples it with the sorted
        # kernel, one puts the results back in input order), timed as a
        # whole, then step by step, and as a whole in edge order (sorted by
        # the edge of each halfedge, so that both triangles of an intrinsic
        # quad come together); then as the library's one call
        hu, uu, vu, fu = to_dev(unsorted)
        sorted_out = torch.empty_like(out)
        keep = {}
        by = {}

        def sort_step(i=0):
            keep["b"] = htex.htex_sort_batch(mesh.H, hu, uu, vu, fu, **by)

        def sample_sorted(i=0):
            perm, h2, u2, v2, f2 = keep["b"]
            htex.htex_sample_prepared(prep, pool, h2, u2, v2, f2, filter=htex.HTEX_TRILINEAR,
                                      flags=htex.HTEX_QUERIES_SORTED, out=sorted_out)

        def unpermute(i=0):
            htex.htex_unpermute_results(keep["b"][0], sorted_out, out=out)

        def sorted_step():
            sort_step()
            sample_sorted()
            unpermute()

        for _ in range(2):
            sorted_step()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        for _ in range(5):
            sorted_step()
        torch.cuda.synchronize()
        extra["unsorted_via_sort_batch_samples_per_s"] = 5 * Q / (time.perf_counter() - t1)
        extra["sort_path_us"] = {"order": "halfedge",
                                 "sort_batch": kernel_seconds(sort_step, n=5)[0] * 1e6,
                                 "sample_sorted": kernel_seconds(sample_sorted, n=5)[0] * 1e6,
                                 "unpermute": kernel_seconds(unpermute, n=5)[0] * 1e6}
        by = {"key": dmesh.edge, "nkeys": mesh.E}
        for _ in range(2):
            sorted_step()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        for _ in range(5):
            sorted_step()
        torch.cuda.synchronize()
        extra["unsorted_via_edge_sort_samples_per_s"] = 5 * Q / (time.perf_counter() - t1)
        extra["edge_sort_path_us"] = {"sort_batch": kernel_seconds(sort_step, n=5)[0] * 1e6,
                                      "sample_sorted": kernel_seconds(sample_sorted, n=5)[0] * 1e6}
        # the library's one call for a batch in any order: sorted to a
        # permutation and records, sampled in halfedge order through the
        # permutation, written back in the batch's order
        def reordered(i=0):
            htex.htex_sample_prepared_reordered(prep, pool, hu, uu, vu, fu,
                                                filter=htex.HTEX_TRILINEAR, out=out)

        for _ in range(2):
            reordered()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        for _ in range(5):
            reordered()
        torch.cuda.synchronize()
        # the headline sort path: the one call
        extra["unsorted_via_sort_samples_per_s"] = 5 * Q / (time.perf_counter() - t1)
        extra["sort_path_us"]["reordered_call"] = kernel_seconds(reordered, n=5)[0] * 1e6
        del hu, uu, vu, fu, sorted_out, keep
        # the frame with its pool stored as BF16 and FP8-E4M3: kernel time
        # from HIP events per launch, and the roofline against the bytes the
        # launch needs at 8 and 4 bytes per texel
        for name, dt, tb in (("bf16", htex.HTEX_BF16, 8), ("fp8_e4m3", htex.HTEX_FP8_E4M3, 4)):
            qp = htex.htex_quantize(pool, dt)
            extra[f"{name}_samples_per_s"] = rate(qp, dev_batches)
            ks, _ = kernel_seconds(lambda i: step(i, qp, dev_batches), n=20)
            rec = {"kernel_us": ks * 1e6, "samples_per_s_kernel": Q / ks,
                   "pool_bytes": qp.nbytes()}
            if alg is not None:
                b = storage_bytes(alg, Q, tb, dt == htex.HTEX_FP8_E4M3)
                rec["alg_bytes_per_query"] = b["bytes_per_query"]
                rec["alg_texel_bytes_per_query"] = b["texel_bytes_per_query"]
                rec["roofline"] = roofline_entry(f"htex::k_sample_prep<{name},trilinear>",
                                                 b["bytes"], ks)
            extra[f"{name}_frame"] = rec
            del qp
            torch.cuda.empty_cache()
        extra["config3_precision"] = precision_config3()
        log(f"config3 {json.dumps(extra['config3_precision'])}")
        for kk in list(extra):
            if kk.endswith("samples_per_s"):
                extra[kk.replace("samples_per_s", "speedup_vs_f32")] = extra[kk] / value
        log(f"extra {json.dumps(extra)}")
        if args.workload == "frame4k":
            extra["rgb_plus_displacement"] = displacement_benchmark(
                mesh, dmesh, step, Q, with_bytes=not args.no_bytes)
            extra["rasterized_view"] = raster_benchmark(mesh, dmesh, prep, pool)
            log(f"raster {json.dumps(extra['rasterized_view'])}")
            extra["anisotropic"] = aniso_benchmark(prep, pool, batches, dev_batches, Q)
            a = extra["anisotropic"]
            a["cost_vs_trilinear"] = value / a["samples_per_s"]
            log(f"aniso {json.dumps(a)}")
            log(f"rgb+disp {json.dumps(extra['rgb_plus_displacement'])}")

    roofline = None
    if alg is not None:
        if args.storage != "f32":
            # the line and segment figures below count float32 texels
            alg = dict(alg, segment_bytes_per_query=float("nan"),
                       line128_bytes_per_query=None, unique_128B_lines=None,
                       **storage_bytes(alg, Q, st_texel_bytes, st_dtype == htex.HTEX_FP8_E4M3))
        achieved = alg["bytes"] / avg_kernel_s / 1e9
        traffic = recorded_traffic() if args.storage == "f32" else None
        roofline = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS,
                    "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                    "kernel": f"htex::k_sample_prep<{args.storage},trilinear>",
                    "avg_kernel_us": avg_kernel_s * 1e6,
                    "median_kernel_us": median_kernel_s * 1e6,
                    "copy_GBs": copy_gbs,
                    # the other two readings of the roofline: counted traffic
                    # between the L2 and the memory fabric (HBM plus hits in
                    # the fabric-side cache; when the counters match this
                    # source) and 64-byte-segment-granular unique bytes
                    "l2_fabric_GBs": traffic / avg_kernel_s / 1e9 if traffic else None,
                    "l2_fabric_frac": (traffic / avg_kernel_s / 1e9 / HBM_PEAK_GBS
                                       if traffic else None),
                    "l2_fabric_vs_copy": (traffic / avg_kernel_s / 1e9 / copy_gbs
                                          if traffic and copy_gbs else None),
                    "segment64_frac": (alg["segment_bytes_per_query"] * Q / avg_kernel_s / 1e9
                                       / HBM_PEAK_GBS if args.storage == "f32" else None),
                    "alg_bytes_per_query": alg["bytes_per_query"],
                    "alg_texel_bytes_per_query": alg["texel_bytes_per_query"],
                    "segment64_bytes_per_query": (alg["segment_bytes_per_query"]
                                                  if args.storage == "f32" else None),
                    "line128_bytes_per_query": alg["line128_bytes_per_query"],
                    "unique_128B_texel_lines": alg["unique_128B_lines"]}
        log(f"algorithmic bytes/query {alg['bytes_per_query']:.1f} "
            f"(texels {alg['texel_bytes_per_query']:.1f}); achieved {achieved:.0f} GB/s")

    if not args.no_extra:
        extra["differentiation"] = grad_benchmark()
        d = extra["differentiation"]
        log(f"grad: fwd {d['forward_us']:.0f} us, bwd {d['backward_us']:.0f} us, Adam loss "
            f"{d['loss_first']:.3e} -> {d['loss_last']:.3e}")

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(mesh, log2res, pool.base_host, pool.texels, batches[0])
        log(f"cpu oracle {cpu['value']:.3e} samples/s on {cpu['cores']} cores")

    pool_bytes = tpool.nbytes()
    serving = None
    if not args.no_serve and args.workload == "frame4k":
        del prep, out, dev_batches, pool, tpool
        torch.cuda.empty_cache()
        serving = serve_benchmark(smeshes, chunk=args.serve_chunk)

    fs = mesh.face_sizes()
    rec = {
        "metric": METRIC, "value": value, "unit": "samples/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": elapsed / args.steps * 1e3, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {
            "workload": ("4K frame: 3840x2160 queries sorted by halfedge, trilinear, "
                         "64x64 RGBA f32 per edge + mips on a seeded ~194k-face "
                         "mixed-polygon sphere with 2% boundary edges")
            if args.workload == "frame4k" else "tiny cube, 16x16 RGBA f32 + mips, trilinear",
            "faces": int(mesh.F), "halfedges": int(mesh.H), "edges": int(mesh.E),
            "face_mix": {"tri": float((fs == 3).mean()), "quad": float((fs == 4).mean()),
                         "5to8": float((fs >= 5).mean())},
            "boundary_edge_frac": float(mesh.boundary_edges().mean()),
            "queries_per_step": Q, "pool_bytes": pool_bytes, "filter": "trilinear",
            "texel_storage": args.storage,
            "log2_footprint": [-3.2, -1.2] if args.workload == "frame4k" else [-6, 0],
            "sorted": True, "batches_rotated": len(batches)},
        "roofline": roofline, "cpu_baseline": cpu, "extra": extra, "serving": serving,
    }
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
