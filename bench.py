#!/usr/bin/env python3
"""Throughput of batched Htex sampling on one MI355X.

Workload (default, "frame4k"): a seeded closed-sphere polygon mesh of about
194k faces (70% quads, 20% triangles, 10% 5-8-gons, 1% of the faces removed
as holes so 2% of the edges are boundary edges), one 64x64 RGBA float32
texture per edge with its full mip chain (34.8 GB resident in HBM), texels
from seeded smooth lattice noise; 3840 x 2160 = 8,294,400 queries per step
(uniform halfedge, uniform barycentric point, log2 footprint ~ U[-3.2, -1.2])
sorted by halfedge, trilinear filtering.  A step is one htex_sample call over
one frame batch; four distinct seeded batches rotate so consecutive steps do
not replay the same addresses.  All inputs are resident in HBM before the
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
    ap.add_argument("--copy-probe", action="store_true",
                    help="also run a 1 GiB device copy (HBM counter calibration)")
    return ap.parse_args()


# ---------------------------------------------------------------- inputs --

def build_workload(name):
    import numpy as np
    from htexgen.mesh import cube_mesh, sphere_mesh
    from htexgen.queries import uniform_queries
    if name == "frame4k":
        mesh = sphere_mesh(n=183, seed=201)
        k, Q, log2f, kind, tex_seed = 6, 3840 * 2160, (-3.2, -1.2), 1, 202
        qseeds = [203, 213, 223, 233]
    else:
        mesh = cube_mesh()
        k, Q, log2f, kind, tex_seed = 4, 65536, (-6.0, 0.0), 0, 102
        qseeds = [103, 113, 123, 133]
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

def algorithmic_bytes(dbg, h, log2res, base, total, Q):
    """Exact bytes one launch must move: queries in (h, u, v, f: 16 B), result
    out (16 B), each distinct halfedge/edge record it reads, and each distinct
    texel (16 B) under an in-bounds filter tap.  Also the distinct 64-byte
    segments those texels occupy."""
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
    nz = np.nonzero(mark)[0]
    segments = int(len(np.unique(nz >> 2)))      # 64-byte segments
    lines128 = int(len(np.unique(nz >> 3)))      # 128-byte lines
    # Next/Prev of each distinct h; Twin/Edge of each distinct h, Next h, Prev h;
    # log2res/base of each distinct edge
    n_h = len(np.unique(h))
    n_g = len(np.unique(np.concatenate([h, rec["next"], rec["prev"]])))
    n_e = len(np.unique(rec["edge"].reshape(-1)))
    topo = 8 * n_h + 8 * n_g + 9 * n_e
    total_bytes = 16 * Q + 16 * Q + topo + 16 * texels
    return {"bytes": int(total_bytes), "bytes_per_query": total_bytes / Q,
            "texel_bytes_per_query": 16 * texels / Q, "unique_texels": texels,
            "unique_64B_segments": segments, "unique_128B_lines": lines128,
            "segment_bytes_per_query": (32 * Q + topo + 64 * segments) / Q,
            "line128_bytes_per_query": (32 * Q + topo + 128 * lines128) / Q}


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
    return {"value": Qs / med, "unit": "samples/s", "cores": cores, "kind": "oracle",
            "sample": f"{Qs} consecutive queries of the sorted frame batch "
                      f"({len(edges)} edges, FP64, median of {len(times)} runs)"}


# ------------------------------------------------------------- profiles --

def recorded_traffic():
    """HBM traffic per launch from the committed rocprofv3 counter summary,
    if it was taken on the current kernel source; else None."""
    path = os.path.join(ROOT, "profiles", "htex_sample_frame4k_pmc.md")
    src = os.path.join(ROOT, "paper_2207_05618_amd", "csrc", "htex_sample.hip")
    if not os.path.exists(path):
        return None
    txt = open(path).read()
    m = re.search(r"kernel_source_sha256:\s*([0-9a-f]{64})", txt)
    b = re.search(r"traffic_bytes_per_launch:\s*([0-9.e+]+)", txt)
    if not m or not b:
        return None
    sha = hashlib.sha256(open(src, "rb").read()).hexdigest()
    return float(b.group(1)) if sha == m.group(1) else None


# ----------------------------------------------------------------- main --

def main():
    args = parse()
    if args.gpus != 1:
        print("bench.py measures one GPU only: this build has no multi-GPU path "
              "(see the sharding notes in DESIGN.md); run with --gpus 1", file=sys.stderr)
        sys.exit(2)
    import numpy as np
    import torch
    import paper_2207_05618_amd as htex
    from htexgen import device as gdev

    t_start = time.perf_counter()
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
    torch.cuda.synchronize()
    dev_batches = [to_dev(b) for b in batches]
    Q = batches[0].Q
    out = torch.empty((Q, 4), dtype=torch.float32, device="cuda")
    stream = torch.cuda.current_stream()

    if args.copy_probe:
        x = torch.empty(1 << 28, dtype=torch.float32, device="cuda")
        y = torch.empty_like(x)
        y.copy_(x)
        torch.cuda.synchronize()
        del x, y

    def step(i, p=pool, bs=dev_batches):
        h, u, v, f = bs[i % len(bs)]
        htex.htex_sample_prepared(prep, p, h, u, v, f, filter=htex.HTEX_TRILINEAR,
                                  flags=htex.HTEX_QUERIES_SORTED, out=out)

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
    value = args.steps * Q / elapsed
    log(f"{args.steps} steps in {elapsed * 1e3:.2f} ms; kernel avg {avg_kernel_s * 1e6:.1f} us")

    def rate(p, bs, n=10):
        for i in range(3):
            step(i, p, bs)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        for i in range(n):
            step(i, p, bs)
        torch.cuda.synchronize()
        return n * Q / (time.perf_counter() - t1)

    extra = {}
    if not args.no_extra:
        extra["unsorted_samples_per_s"] = rate(pool, [to_dev(unsorted)])
        qb = htex.htex_quantize(pool, htex.HTEX_BF16)
        extra["bf16_samples_per_s"] = rate(qb, dev_batches)
        del qb
        q8 = htex.htex_quantize(pool, htex.HTEX_FP8_E4M3)
        extra["fp8_e4m3_samples_per_s"] = rate(q8, dev_batches)
        del q8
        torch.cuda.empty_cache()
        for kk in list(extra):
            extra[kk.replace("samples_per_s", "speedup_vs_f32")] = extra[kk] / value
        log(f"extra {json.dumps({k: round(v, 3) for k, v in extra.items()})}")

    roofline = None
    alg = None
    if not args.no_bytes:
        h, u, v, f = dev_batches[0]
        _, dbg = htex.htex_sample(dmesh, pool, h, u, v, f, filter=htex.HTEX_TRILINEAR,
                                  debug=True)
        dbg_host = dbg.cpu().numpy()
        del dbg
        alg = algorithmic_bytes(dbg_host, batches[0].h, log2res, pool.base_host, pool.total, Q)
        del dbg_host
        achieved = alg["bytes"] / avg_kernel_s / 1e9
        traffic = recorded_traffic()
        roofline = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS,
                    "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                    "kernel": "htex::k_sample_prep<f32,trilinear>",
                    "avg_kernel_us": avg_kernel_s * 1e6,
                    "alg_bytes_per_query": alg["bytes_per_query"],
                    "alg_texel_bytes_per_query": alg["texel_bytes_per_query"],
                    "segment64_bytes_per_query": alg["segment_bytes_per_query"],
                    "line128_bytes_per_query": alg["line128_bytes_per_query"],
                    "unique_128B_texel_lines": alg["unique_128B_lines"]}
        log(f"algorithmic bytes/query {alg['bytes_per_query']:.1f} "
            f"(texels {alg['texel_bytes_per_query']:.1f}); achieved {achieved:.0f} GB/s")

    cpu = None
    if not args.no_cpu_baseline:
        cpu = cpu_baseline(mesh, log2res, pool.base_host, pool.texels, batches[0])
        log(f"cpu oracle {cpu['value']:.3e} samples/s on {cpu['cores']} cores")

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
            "queries_per_step": Q, "pool_bytes": pool.nbytes(), "filter": "trilinear",
            "log2_footprint": [-3.2, -1.2] if args.workload == "frame4k" else [-6, 0],
            "sorted": True, "batches_rotated": len(batches)},
        "roofline": roofline, "cpu_baseline": cpu, "extra": extra,
    }
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
