// htex_sample.hip -- batched Htex sampling (forward) for gfx950: the plain
// and prepared batch kernels, the serving kernel and the preparation of
// per-halfedge records.
//
// One lane per query.  Per query: the halfedge operators Next/Prev/Twin/Edge
// (Section 2), Alg. 2's reflection for each of the three fetches of Alg. 3
// (own quad at (u, v), Next quad at (v, -u), Prev quad at (-v, u)), the
// OpenGL level pair for trilinear filtering, the bilinear taps of each level
// with a zero border, and the float32 blend normalized by the summed
// border-normalization channel (computed from the in-bounds tap weights, so
// it costs no memory).  This is a gather bound by HBM bandwidth: no MFMA.
// The building blocks live in htex_filter.h.
#include <hip/hip_runtime.h>

#include "htex_filter.h"

namespace htex {
namespace {

template <int DT, int CH, bool TRI, bool DBG>
__global__ void __launch_bounds__(kBlock) k_sample(SampleArgs a)
{
    const int64_t q = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (q >= a.Q) return;
    // queries and results stream through once: keep them out of the caches
    const int32_t h = __builtin_nontemporal_load(a.qh + q);
    const float u = __builtin_nontemporal_load(a.qu + q);
    const float v = __builtin_nontemporal_load(a.qv + q);
    if (!((uint32_t)h < (uint32_t)a.H) || !isfinite(u) || !isfinite(v)) {
        const float nan = __uint_as_float(0x7fc00000u);
        store_row<CH>(a.out, q, nan, nan, nan, nan);
        if (a.err) atomicAdd(a.err, 1);
        if constexpr (DBG) {
            htex_debug_rec d = {};
            d.next = d.prev = -1;
            for (int s = 0; s < 3; ++s) {
                d.edge[s] = -1;
                d.level[s][0] = d.level[s][1] = -1;
            }
            a.dbg[q] = d;
        }
        return;
    }
    const int32_t n1 = a.next[h], p1 = a.prev[h];
    Lod L{0, 0, 0.0f, 1.0f};
    if constexpr (TRI) L = lod_of(__builtin_nontemporal_load(a.qf + q));
    FetchSpec fs[3];
    fetch_specs(h, n1, p1, u, v, fs);
    htex_debug_rec d;
    if constexpr (DBG) {
        d = {};
        d.next = n1;
        d.prev = p1;
        d.phi = L.phi;
    }
    // Alg. 3: c <- c + Texture(...) for the own quad, then Next, then Prev
    float4 C = make_float4(0.f, 0.f, 0.f, 0.f);
    float W = 0.0f;
#pragma unroll
    for (int s = 0; s < 3; ++s) {
        float4 Cf = make_float4(0.f, 0.f, 0.f, 0.f);
        float Wf = 0.0f;
        fetch<DT, CH, TRI, DBG>(a, L, fs[s], resolve_plain<DT, CH>(a, fs[s].g), Cf, Wf, &d, s);
        C.x += Cf.x;
        C.y += Cf.y;
        C.z += Cf.z;
        C.w += Cf.w;
        W += Wf;
    }
    const float r = __builtin_amdgcn_rcpf(W);
    store_row<CH>(a.out, q, C.x * r, C.y * r, C.z * r, C.w * r);
    if constexpr (DBG) {
        d.W = W;
        a.dbg[q] = d;
    }
}

// The prepared record of halfedge h, read once per run of lanes with the
// same halfedge: in a sorted batch about ten neighbouring lanes share one,
// and a 48-byte load on every lane costs the texture data unit, which
// bounds the sampler, time in proportion to its active lanes.  The first
// lane of each run loads it (an invalid h loads nothing and reads zeros),
// the others take its words through ds_bpermute.  Every lane of the
// wavefront that is still active must call this; a lane's run starts at or
// below it, so lanes past the end of a batch (the high lanes) are never read.
__device__ __forceinline__ PrepRec run_shared_record(const SampleArgs &a, int32_t h)
{
    const int lane = __lane_id();
    // every lane shuffles (a lane left out of a ds_bpermute gives it no data)
    const int32_t hp = __shfl_up(h, 1);
    const bool first = (lane == 0) | (hp != h);
    const uint64_t firsts = __ballot(first);
    const int src = 63 - __builtin_clzll(firsts & ((2ull << lane) - 1ull));
    constexpr int NW = 11;   // the record's words before its padding
    static_assert(sizeof(PrepRec) == 4 * (NW + 1), "record words");
    uint32_t w[NW + 1] = {};
    if (first && (uint32_t)h < (uint32_t)a.H) {
        const PrepRec r = static_cast<const PrepRec *>(a.prep)[h];
        __builtin_memcpy(w, &r, sizeof(PrepRec));
    }
#pragma unroll
    for (int i = 0; i < NW; ++i) w[i] = (uint32_t)__shfl((int)w[i], src);
    w[NW] = 0u;
    PrepRec rec;
    __builtin_memcpy(&rec, w, sizeof(PrepRec));
    return rec;
}

// Fast path: the same arithmetic as k_sample with the navigation read from
// one prepared record per query (bit-identical results).  Shared by the
// batch kernel and the serving kernel, so a query's result does not depend
// on which launch, batch or tile computes it.
// SCATTERED selects the per-tap predicated fetch for batches in random
// order (same results); SHARE reads the record once per run of lanes on one
// halfedge (the batch kernel for sorted batches; same results).  A record
// that does not fit the pool (prepared for another layout) makes its query
// invalid.
template <int DT, int CH, bool TRI, bool SCATTERED, bool GATHER = false, bool SHARE = false>
__device__ __forceinline__ void sample_one_prepared(const SampleArgs &a, int64_t q)
{
    int32_t h;
    float u, v, fq = 0.0f;
    if constexpr (GATHER) {
        // query q of a batch sampled in another order: record order[q]
        const float4 r = static_cast<const float4 *>(a.qrec)[__builtin_nontemporal_load(a.order + q)];
        h = __float_as_int(r.x);
        u = r.y;
        v = r.z;
        fq = r.w;
    } else {
        h = __builtin_nontemporal_load(a.qh + q);
        u = __builtin_nontemporal_load(a.qu + q);
        v = __builtin_nontemporal_load(a.qv + q);
    }
    PrepRec rec;
    bool valid = ((uint32_t)h < (uint32_t)a.H) && isfinite(u) && isfinite(v);
    if constexpr (SHARE) {
        rec = run_shared_record(a, h);
        if (valid) valid = record_in_pool(rec, a.total_texels, a.has_mips != 0);
    } else if (valid) {
        rec = static_cast<const PrepRec *>(a.prep)[h];
        valid = record_in_pool(rec, a.total_texels, a.has_mips != 0);
    }
    if (!valid) {
        const float nan = __uint_as_float(0x7fc00000u);
        store_row<CH>(a.out, q, nan, nan, nan, nan);
        if (a.err) atomicAdd(a.err, 1);
        return;
    }
    Lod L{0, 0, 0.0f, 1.0f};
    if constexpr (TRI) L = lod_of(GATHER ? fq : __builtin_nontemporal_load(a.qf + q));
    FetchSpec fs[3];
    fetch_specs(h, rec.next, rec.prev, u, v, fs);
    float4 C = make_float4(0.f, 0.f, 0.f, 0.f);
    float W = 0.0f;
#pragma unroll
    for (int s = 0; s < 3; ++s) {
        float4 Cf = make_float4(0.f, 0.f, 0.f, 0.f);
        float Wf = 0.0f;
        const Resolved R = resolve_prepared<DT, CH>(a, rec.w[s], rec.e[s]);
        if constexpr (SCATTERED) fetch_in_bounds<DT, CH, TRI>(a, L, fs[s], R, Cf, Wf);
        else fetch<DT, CH, TRI, false>(a, L, fs[s], R, Cf, Wf, nullptr, s);
        C.x += Cf.x;
        C.y += Cf.y;
        C.z += Cf.z;
        C.w += Cf.w;
        W += Wf;
    }
    const float r = __builtin_amdgcn_rcpf(W);
    store_row<CH>(a.out, q, C.x * r, C.y * r, C.z * r, C.w * r);
}

// Whether fetch s (Next or Prev) of a query may have an in-bounds tap: the
// Next quad's y coordinate is -u (1 + u when reflected) and the Prev quad's
// x coordinate is -v (1 + v), so a tap row or column of a level with n
// texels lies inside only when c n <= 1/2; the test uses the coarsest level
// the fetch samples, so it holds whenever any level has an in-bounds tap.
__device__ __forceinline__ bool neighbour_may_touch(const Lod &L, int k, float c)
{
    int lv[2];
    float om[2];
    const int nl = fetch_levels(L, k, lv, om);
    return ldexpf(c, k - (nl == 2 ? lv[1] : lv[0])) <= 0.5f;
}

__device__ __forceinline__ int32_t bperm(int32_t byte_addr, int32_t x)
{
    return __builtin_amdgcn_ds_bpermute(byte_addr, x);
}
__device__ __forceinline__ float bperm(int32_t byte_addr, float x)
{
    return __int_as_float(__builtin_amdgcn_ds_bpermute(byte_addr, __float_as_int(x)));
}

// A Next or Prev fetch dealt out to another lane of the wavefront: the
// owner's coordinates, level selection and the fetch's prepared record word.
struct alignas(16) Task {
    float u, v, phi, om0;
    int32_t lpack;   // E << 2 | mode
    int32_t e;
    uint32_t wlo, whi;
};
constexpr int kTasks = 128;   // per wavefront: at most one Next and one Prev fetch per lane

// The prepared fast path executed by a whole wavefront at once, for
// launches bound by the VALU.  Every lane computes its own quad's fetch;
// the Next and Prev fetches, which only queries near the spokes of their
// triangle need, are compacted: lanes that need one are counted by ballot,
// write the fetch's inputs to consecutive task slots in LDS, the wave works
// through the slots 64 at a time, and each owner pulls its results back by
// ds_bpermute and adds them in Alg. 3's order (a query's Next slot always
// precedes its Prev slot), so the results are those of sample_one_prepared
// bit for bit.  Decoding BF16 and FP8 texels makes their launches
// VALU-bound, and so does a float32 pool small enough to stay in the
// caches; the compaction saves 6-10% there.  A large float32 pool is bound
// by the memory pipeline, and there the compaction costs 2-3%.  All 64
// lanes of the wave must call it; `live` marks lanes that hold a query.
template <int DT, int CH, bool TRI, bool GATHER = false>
__device__ __forceinline__ void sample_wave_prepared(const SampleArgs &a, int64_t q, bool live,
                                                     Task *tasks)
{
    const int lane = (int)__lane_id();
    int32_t h = 0;
    float u = 0.0f, v = 0.0f, f = 0.0f;
    if (live) {
        if constexpr (GATHER) {
            const float4 r =
                static_cast<const float4 *>(a.qrec)[__builtin_nontemporal_load(a.order + q)];
            h = __float_as_int(r.x);
            u = r.y;
            v = r.z;
            if constexpr (TRI) f = r.w;
        } else {
            h = __builtin_nontemporal_load(a.qh + q);
            u = __builtin_nontemporal_load(a.qu + q);
            v = __builtin_nontemporal_load(a.qv + q);
            if constexpr (TRI) f = __builtin_nontemporal_load(a.qf + q);
        }
    }
    bool valid = live && ((uint32_t)h < (uint32_t)a.H) && isfinite(u) && isfinite(v);
    PrepRec rec = PrepRec{};
    if (valid) {
        rec = static_cast<const PrepRec *>(a.prep)[h];
        valid = record_in_pool(rec, a.total_texels, a.has_mips != 0);
        if (!valid) rec = PrepRec{};
    }
    if (live && !valid) {
        const float nan = __uint_as_float(0x7fc00000u);
        store_row<CH>(a.out, q, nan, nan, nan, nan);
        if (a.err) atomicAdd(a.err, 1);
    }
    Lod L{0, 0, 0.0f, 1.0f};
    if constexpr (TRI) L = lod_of(f);
    // the Next and Prev fetches this query may need, posted as tasks
    const bool need1 = valid && neighbour_may_touch(L, (int)((rec.w[1] >> 40) & 31u), u);
    const bool need2 = valid && neighbour_may_touch(L, (int)((rec.w[2] >> 40) & 31u), v);
    const uint64_t b1 = __ballot(need1), b2 = __ballot(need2);
    const int n1 = __popcll(b1), T = n1 + __popcll(b2);
    const int s1 = (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(b1 >> 32),
                                                  __builtin_amdgcn_mbcnt_lo((uint32_t)b1, 0u));
    const int s2 = n1 + (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(b2 >> 32),
                                                       __builtin_amdgcn_mbcnt_lo((uint32_t)b2, 0u));
    if (T > 0) {
        Task t;
        t.u = u;
        t.v = v;
        t.phi = L.phi;
        t.om0 = L.om0;
        t.lpack = (L.E << 2) | L.mode;
        if (need1) {
            t.e = rec.e[1];
            t.wlo = (uint32_t)rec.w[1];
            t.whi = (uint32_t)(rec.w[1] >> 32);
            tasks[s1] = t;
        }
        if (need2) {
            t.e = rec.e[2];
            t.wlo = (uint32_t)rec.w[2];
            t.whi = (uint32_t)(rec.w[2] >> 32);
            tasks[s2] = t;
        }
    }
    // Alg. 3's first fetch: the query's own quad at (u, v)
    float4 C = make_float4(0.f, 0.f, 0.f, 0.f);
    float W = 0.0f;
    if (valid) {
        const FetchSpec f0 = {h, u, v, false, false};
        fetch<DT, CH, TRI, false>(a, L, f0, resolve_prepared<DT, CH>(a, rec.w[0], rec.e[0]), C, W,
                                  nullptr, 0);
    }
    if (T > 0) {
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        for (int base = 0; base < T; base += 64) {
            const int i = base + lane;
            const bool has = i < T;
            const bool nx = i < n1;   // a Next fetch, else a Prev fetch
            float4 Ct = make_float4(0.f, 0.f, 0.f, 0.f);
            float Wt = 0.0f;
            if (has) {
                const Task t = tasks[i];
                Lod tL;
                tL.mode = t.lpack & 3;
                tL.E = t.lpack >> 2;
                tL.phi = t.phi;
                tL.om0 = t.om0;
                // Next quad at (v, -u), Prev quad at (-v, u)
                const FetchSpec tf = {0, t.v, t.u, !nx, nx};
                const uint64_t w = (uint64_t)t.whi << 32 | t.wlo;
                fetch<DT, CH, TRI, false>(a, tL, tf, resolve_prepared<DT, CH>(a, w, t.e), Ct, Wt,
                                          nullptr, nx ? 1 : 2);
            }
            // owners add the fetches of this round, Next before Prev
            const int r1 = s1 - base, r2 = s2 - base;
            const bool got1 = need1 && (uint32_t)r1 < 64u, got2 = need2 && (uint32_t)r2 < 64u;
            const int a1 = (r1 & 63) << 2, a2 = (r2 & 63) << 2;
            const float x1 = bperm(a1, Ct.x), x2 = bperm(a2, Ct.x);
            const float q1 = bperm(a1, Wt), q2 = bperm(a2, Wt);
            if constexpr (CH == 4) {
                const float y1 = bperm(a1, Ct.y), z1 = bperm(a1, Ct.z), w1 = bperm(a1, Ct.w);
                const float y2 = bperm(a2, Ct.y), z2 = bperm(a2, Ct.z), w2 = bperm(a2, Ct.w);
                if (got1) { C.x += x1; C.y += y1; C.z += z1; C.w += w1; W += q1; }
                if (got2) { C.x += x2; C.y += y2; C.z += z2; C.w += w2; W += q2; }
            } else {
                if (got1) { C.x += x1; W += q1; }
                if (got2) { C.x += x2; W += q2; }
            }
        }
    }
    if (valid) {
        const float r = __builtin_amdgcn_rcpf(W);
        store_row<CH>(a.out, q, C.x * r, C.y * r, C.z * r, C.w * r);
    }
}

// Prepared-record kernels: MODE 0 one lane per query, all taps of a
// sampled level read (coherent batches); 1 one lane per query, in-bounds
// taps only (scattered batches); 2 the wavefront-compacted path
// (VALU-bound launches).  All three give the same bits.
// MODE: the kernel (kPrepLane, kPrepScattered, kPrepWave), plus kPrepGather
// for a batch read through an order array (SampleArgs::order, ::qrec).
enum { kPrepLane = 0, kPrepScattered = 1, kPrepWave = 2, kPrepGather = 4 };

template <int DT, int CH, bool TRI, int MODE>
__global__ void __launch_bounds__(kBlock) k_sample_prep(SampleArgs a)
{
    constexpr int KIND = MODE & 3;
    constexpr bool GATHER = (MODE & kPrepGather) != 0;
    const int64_t q = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if constexpr (KIND == kPrepWave) {
        __shared__ Task tasks[kBlock / 64][kTasks];
        if (q - (int64_t)__lane_id() >= a.Q) return;   // the whole wavefront is past the end
        sample_wave_prepared<DT, CH, TRI, GATHER>(a, q, q < a.Q, tasks[threadIdx.x >> 6]);
    } else {
        if (q >= a.Q) return;
        sample_one_prepared<DT, CH, TRI, KIND == kPrepScattered, GATHER, KIND == kPrepLane>(a, q);
    }
}

// Serving: one launch covers a list of tiles, each up to kBlock queries of
// one request on one resident mesh.  A fixed grid walks the list (block b
// takes tiles b, b + G, ...), so every block exits once the list is done.
template <int DT, int CH, bool TRI>
__global__ void __launch_bounds__(kBlock) k_serve(const ServeMesh *meshes, const ServeTile *tiles,
                                                  int32_t ntiles, int32_t *err)
{
    for (int32_t t = blockIdx.x; t < ntiles; t += gridDim.x) {
        const ServeTile T = tiles[t];
        if ((int32_t)threadIdx.x < T.count) {
            const ServeMesh M = meshes[T.mesh];
            SampleArgs a{};
            a.H = M.H;
            a.prep = M.prep;
            a.total_texels = M.total_texels;
            a.has_mips = M.has_mips;
            a.texels = M.texels;
            a.scale = M.scale;
            a.Q = T.q0 + T.count;
            a.qh = T.h;
            a.qu = T.u;
            a.qv = T.v;
            a.qf = T.f;
            a.out = T.out;
            a.err = err;
            sample_one_prepared<DT, CH, TRI, false>(a, T.q0 + threadIdx.x);
        }
    }
}

// One record per halfedge: resolve Next/Prev, the edges, reflections,
// resolutions and texture bases of its three fetches.
__global__ void __launch_bounds__(kBlock) k_prepare(SampleArgs a, PrepRec *out)
{
    const int64_t h = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (h >= a.H) return;
    PrepRec r;
    r.next = a.next[h];
    r.prev = a.prev[h];
    r.pad = 0;
    const int32_t g[3] = {(int32_t)h, r.next, r.prev};
#pragma unroll
    for (int s = 0; s < 3; ++s) {
        const bool flip = !(g[s] > a.twin[g[s]]);
        const int32_t e = a.edge[g[s]];
        r.e[s] = e;
        r.w[s] = (uint64_t)a.base[e] | ((uint64_t)a.log2res[e] << 40) | ((uint64_t)(flip ? 1 : 0) << 45);
    }
    out[h] = r;
}


template <int DT, int CH, bool TRI>
hipError_t launch_fwd(const SampleArgs &a, hipStream_t s)
{
    const uint32_t G = (uint32_t)ceil_div(a.Q, kBlock);
    if (a.dbg)
        hipLaunchKernelGGL((k_sample<DT, CH, TRI, true>), dim3(G), dim3(kBlock), 0, s, a);
    else
        hipLaunchKernelGGL((k_sample<DT, CH, TRI, false>), dim3(G), dim3(kBlock), 0, s, a);
    return hipGetLastError();
}

template <int DT, int CH, bool TRI, int MODE>
hipError_t launch_fwd_prep(const SampleArgs &a, hipStream_t s)
{
    const uint32_t G = (uint32_t)ceil_div(a.Q, kBlock);
    hipLaunchKernelGGL((k_sample_prep<DT, CH, TRI, MODE>), dim3(G), dim3(kBlock), 0, s, a);
    return hipGetLastError();
}

// Calls L<DT, CH, TRI>::run(a, s) for the runtime storage type, channel
// count and filter.
template <template <int, int, bool> class L>
hipError_t dispatch(const SampleArgs &a, int dtype, int filter, hipStream_t s)
{
    const bool tri = filter == HTEX_TRILINEAR;
    const bool one = a.channels == 1;
#define HTEX_DISPATCH_DT(DTV)                                                              \
    return one ? (tri ? L<DTV, 1, true>::run(a, s) : L<DTV, 1, false>::run(a, s))          \
               : (tri ? L<DTV, 4, true>::run(a, s) : L<DTV, 4, false>::run(a, s))
    switch (dtype) {
    case HTEX_F32: HTEX_DISPATCH_DT(HTEX_F32);
    case HTEX_BF16: HTEX_DISPATCH_DT(HTEX_BF16);
    default: HTEX_DISPATCH_DT(HTEX_FP8_E4M3);
    }
#undef HTEX_DISPATCH_DT
}

template <int DT, int CH, bool TRI> struct Fwd {
    static hipError_t run(const SampleArgs &a, hipStream_t s) { return launch_fwd<DT, CH, TRI>(a, s); }
};
template <int DT, int CH, bool TRI> struct FwdPrep {
    static hipError_t run(const SampleArgs &a, hipStream_t s)
    {
        return launch_fwd_prep<DT, CH, TRI, kPrepLane>(a, s);
    }
};
template <int DT, int CH, bool TRI> struct FwdPrepScattered {
    static hipError_t run(const SampleArgs &a, hipStream_t s)
    {
        return launch_fwd_prep<DT, CH, TRI, kPrepScattered>(a, s);
    }
};
template <int DT, int CH, bool TRI> struct FwdPrepWave {
    static hipError_t run(const SampleArgs &a, hipStream_t s)
    {
        return launch_fwd_prep<DT, CH, TRI, kPrepWave>(a, s);
    }
};
template <int DT, int CH, bool TRI> struct FwdPrepGather {
    static hipError_t run(const SampleArgs &a, hipStream_t s)
    {
        return launch_fwd_prep<DT, CH, TRI, kPrepLane | kPrepGather>(a, s);
    }
};
template <int DT, int CH, bool TRI> struct FwdPrepWaveGather {
    static hipError_t run(const SampleArgs &a, hipStream_t s)
    {
        return launch_fwd_prep<DT, CH, TRI, kPrepWave | kPrepGather>(a, s);
    }
};

}  // namespace

hipError_t launch_serve(const ServeMesh *meshes, const ServeTile *tiles, int32_t ntiles,
                        int32_t grid, int dtype, int channels, int filter, int32_t *err,
                        hipStream_t s)
{
    if (ntiles == 0) return hipSuccess;
    const uint32_t G = (uint32_t)(grid < ntiles ? grid : ntiles);
    const bool tri = filter == HTEX_TRILINEAR, one = channels == 1;
#define HTEX_SERVE(DTV, CHV, TRV)                                                          \
    hipLaunchKernelGGL((k_serve<DTV, CHV, TRV>), dim3(G), dim3(kBlock), 0, s, meshes, tiles, \
                       ntiles, err)
#define HTEX_SERVE_DT(DTV)                                                                 \
    if (one) {                                                                             \
        if (tri) HTEX_SERVE(DTV, 1, true); else HTEX_SERVE(DTV, 1, false);                 \
    } else {                                                                               \
        if (tri) HTEX_SERVE(DTV, 4, true); else HTEX_SERVE(DTV, 4, false);                 \
    }
    switch (dtype) {
    case HTEX_F32: HTEX_SERVE_DT(HTEX_F32); break;
    case HTEX_BF16: HTEX_SERVE_DT(HTEX_BF16); break;
    default: HTEX_SERVE_DT(HTEX_FP8_E4M3); break;
    }
#undef HTEX_SERVE_DT
#undef HTEX_SERVE
    return hipGetLastError();
}

hipError_t launch_prepare(const SampleArgs &a, void *prep, hipStream_t s)
{
    if (a.H == 0) return hipSuccess;
    const uint32_t G = (uint32_t)ceil_div(a.H, kBlock);
    hipLaunchKernelGGL(k_prepare, dim3(G), dim3(kBlock), 0, s, a, static_cast<PrepRec *>(prep));
    return hipGetLastError();
}

hipError_t launch_sample_prepared(const SampleArgs &a, int dtype, int filter, bool scattered,
                                  bool cache_resident, hipStream_t s)
{
    if (a.Q == 0) return hipSuccess;
    // VALU-bound: quantized texels, or a pool that stays in the caches
    const bool valu = dtype != HTEX_F32 || cache_resident;
    if (a.order)   // a batch read through an order: its sorted-batch kernels
        return valu ? dispatch<FwdPrepWaveGather>(a, dtype, filter, s)
                    : dispatch<FwdPrepGather>(a, dtype, filter, s);
    if (scattered) return dispatch<FwdPrepScattered>(a, dtype, filter, s);
    if (valu) return dispatch<FwdPrepWave>(a, dtype, filter, s);
    return dispatch<FwdPrep>(a, dtype, filter, s);
}

hipError_t launch_sample(const SampleArgs &a, int dtype, int filter, hipStream_t s)
{
    if (a.Q == 0) return hipSuccess;
    return dispatch<Fwd>(a, dtype, filter, s);
}

}  // namespace htex
