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

// Fast path: the same arithmetic as k_sample with the navigation read from
// one prepared record per query (bit-identical results).  Shared by the
// batch kernel and the serving kernel, so a query's result does not depend
// on which launch, batch or tile computes it.
// SCATTERED selects the per-tap predicated fetch for batches in random
// order (same results).
template <int DT, int CH, bool TRI, bool SCATTERED>
__device__ __forceinline__ void sample_one_prepared(const SampleArgs &a, int64_t q)
{
    const int32_t h = __builtin_nontemporal_load(a.qh + q);
    const float u = __builtin_nontemporal_load(a.qu + q);
    const float v = __builtin_nontemporal_load(a.qv + q);
    if (!((uint32_t)h < (uint32_t)a.H) || !isfinite(u) || !isfinite(v)) {
        const float nan = __uint_as_float(0x7fc00000u);
        store_row<CH>(a.out, q, nan, nan, nan, nan);
        if (a.err) atomicAdd(a.err, 1);
        return;
    }
    const PrepRec rec = static_cast<const PrepRec *>(a.prep)[h];
    Lod L{0, 0, 0.0f, 1.0f};
    if constexpr (TRI) L = lod_of(__builtin_nontemporal_load(a.qf + q));
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

template <int DT, int CH, bool TRI, bool SCATTERED>
__global__ void __launch_bounds__(kBlock) k_sample_prep(SampleArgs a)
{
    const int64_t q = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (q >= a.Q) return;
    sample_one_prepared<DT, CH, TRI, SCATTERED>(a, q);
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

template <int DT, int CH, bool TRI, bool SCATTERED>
hipError_t launch_fwd_prep(const SampleArgs &a, hipStream_t s)
{
    const uint32_t G = (uint32_t)ceil_div(a.Q, kBlock);
    hipLaunchKernelGGL((k_sample_prep<DT, CH, TRI, SCATTERED>), dim3(G), dim3(kBlock), 0, s, a);
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
        return launch_fwd_prep<DT, CH, TRI, false>(a, s);
    }
};
template <int DT, int CH, bool TRI> struct FwdPrepScattered {
    static hipError_t run(const SampleArgs &a, hipStream_t s)
    {
        return launch_fwd_prep<DT, CH, TRI, true>(a, s);
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
                                  hipStream_t s)
{
    if (a.Q == 0) return hipSuccess;
    return scattered ? dispatch<FwdPrepScattered>(a, dtype, filter, s)
                     : dispatch<FwdPrep>(a, dtype, filter, s);
}

hipError_t launch_sample(const SampleArgs &a, int dtype, int filter, hipStream_t s)
{
    if (a.Q == 0) return hipSuccess;
    return dispatch<Fwd>(a, dtype, filter, s);
}

}  // namespace htex
