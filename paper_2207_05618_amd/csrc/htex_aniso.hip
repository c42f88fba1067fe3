// htex_aniso.hip -- anisotropic Htex sampling (Section 5.1, Fig. 7): the
// OpenGL anisotropic filter applied to each of Alg. 3's fetches, from the
// screen-space derivatives of a query's barycentric coordinates.
#include <hip/hip_runtime.h>

#include "htex_filter.h"

namespace htex {
namespace {

// Anisotropic filtering (the OpenGL anisotropic filter applied to each of
// Alg. 3's fetches).  From the screen derivatives of (u, v): axis lengths
// px = |d/dx|, py = |d/dy|; N = ceil(pmax / pmin) probes (at most
// max_aniso) at (u, v) + (i / (N + 1) - 1/2) * major axis, i = 1..N, each a
// trilinear Alg. 3 evaluation at footprint pmax / N; colour and
// normalization are summed over all probes, then divided.  The quad maps
// are isometries, so one plan serves all three fetches.  N and the probe
// coordinates decide integers (probe count, tap bases), so they are formed
// with one IEEE rounding per operation and no fused multiply-add, exactly
// as the specification of the filter is written.
struct AnisoPlan {
    int n;
    float f, au, av;
};

__device__ __forceinline__ AnisoPlan aniso_plan(float4 J, int max_aniso)
{
#pragma clang fp contract(off)
    const float px = __builtin_sqrtf(J.x * J.x + J.y * J.y);
    const float py = __builtin_sqrtf(J.z * J.z + J.w * J.w);
    const bool xmajor = px >= py;
    const float pmax = xmajor ? px : py, pmin = xmajor ? py : px;
    AnisoPlan A;
    A.au = xmajor ? J.x : J.z;
    A.av = xmajor ? J.y : J.w;
    if (pmax == 0.0f) {
        A.n = 1;
        A.f = 0.0f;
        return A;
    }
    const float ratio = pmax / pmin;   // +inf when pmin is 0
    A.n = ratio > (float)max_aniso ? max_aniso : max(1, (int)ceilf(ratio));
    A.f = pmax / (float)A.n;
    return A;
}

__device__ __forceinline__ void aniso_probe(const AnisoPlan &A, int i, float u, float v,
                                            float &ui, float &vi)
{
#pragma clang fp contract(off)
    const float t = (float)i / (float)(A.n + 1) - 0.5f;
    ui = u + t * A.au;
    vi = v + t * A.av;
}

template <int DT, int CH, bool PREP>
__global__ void __launch_bounds__(kBlock) k_aniso(SampleArgs a, const float4 *jac, int max_aniso,
                                                  int32_t *nprobe)
{
    const int64_t q = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (q >= a.Q) return;
    const int32_t h = __builtin_nontemporal_load(a.qh + q);
    const float u = __builtin_nontemporal_load(a.qu + q);
    const float v = __builtin_nontemporal_load(a.qv + q);
    const float4 J = jac[q];
    if (!((uint32_t)h < (uint32_t)a.H) || !isfinite(u) || !isfinite(v) || !isfinite(J.x) ||
        !isfinite(J.y) || !isfinite(J.z) || !isfinite(J.w)) {
        const float nan = __uint_as_float(0x7fc00000u);
        store_row<CH>(a.out, q, nan, nan, nan, nan);
        if (a.err) atomicAdd(a.err, 1);
        if (nprobe) nprobe[q] = 0;
        return;
    }
    int32_t n1, p1;
    Resolved R[3];
    if constexpr (PREP) {
        const PrepRec rec = static_cast<const PrepRec *>(a.prep)[h];
        n1 = rec.next;
        p1 = rec.prev;
#pragma unroll
        for (int s = 0; s < 3; ++s) R[s] = resolve_prepared<DT, CH>(a, rec.w[s], rec.e[s]);
    } else {
        n1 = a.next[h];
        p1 = a.prev[h];
        R[0] = resolve_plain<DT, CH>(a, h);
        R[1] = resolve_plain<DT, CH>(a, n1);
        R[2] = resolve_plain<DT, CH>(a, p1);
    }
    const AnisoPlan A = aniso_plan(J, max_aniso);
    const Lod L = lod_of(A.f);
    float4 C = make_float4(0.f, 0.f, 0.f, 0.f);
    float W = 0.0f;
    for (int i = 1; i <= A.n; ++i) {
        float ui, vi;
        aniso_probe(A, i, u, v, ui, vi);
        FetchSpec fs[3];
        fetch_specs(h, n1, p1, ui, vi, fs);
#pragma unroll
        for (int s = 0; s < 3; ++s) {
            float4 Cf = make_float4(0.f, 0.f, 0.f, 0.f);
            float Wf = 0.0f;
            fetch<DT, CH, true, false>(a, L, fs[s], R[s], Cf, Wf, nullptr, s);
            C.x += Cf.x;
            C.y += Cf.y;
            C.z += Cf.z;
            C.w += Cf.w;
            W += Wf;
        }
    }
    const float r = __builtin_amdgcn_rcpf(W);
    store_row<CH>(a.out, q, C.x * r, C.y * r, C.z * r, C.w * r);
    if (nprobe) nprobe[q] = A.n;
}

template <int DT, int CH, bool PREP>
hipError_t launch_aniso_t(const SampleArgs &a, const float *jac, int max_aniso, int32_t *nprobe,
                          hipStream_t s)
{
    const uint32_t G = (uint32_t)ceil_div(a.Q, kBlock);
    hipLaunchKernelGGL((k_aniso<DT, CH, PREP>), dim3(G), dim3(kBlock), 0, s, a,
                       reinterpret_cast<const float4 *>(jac), max_aniso, nprobe);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_sample_aniso(const SampleArgs &a, int dtype, const float *jac, int max_aniso,
                               int32_t *nprobe, hipStream_t s)
{
    if (a.Q == 0) return hipSuccess;
    const bool prep = a.prep != nullptr, one = a.channels == 1;
#define HTEX_ANISO(DTV)                                                                       \
    return prep ? (one ? launch_aniso_t<DTV, 1, true>(a, jac, max_aniso, nprobe, s)          \
                       : launch_aniso_t<DTV, 4, true>(a, jac, max_aniso, nprobe, s))         \
                : (one ? launch_aniso_t<DTV, 1, false>(a, jac, max_aniso, nprobe, s)         \
                       : launch_aniso_t<DTV, 4, false>(a, jac, max_aniso, nprobe, s))
    switch (dtype) {
    case HTEX_F32: HTEX_ANISO(HTEX_F32);
    case HTEX_BF16: HTEX_ANISO(HTEX_BF16);
    default: HTEX_ANISO(HTEX_FP8_E4M3);
    }
#undef HTEX_ANISO
}

}  // namespace htex
