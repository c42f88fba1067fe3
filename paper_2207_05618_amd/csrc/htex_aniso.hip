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

// What a probe needs of its query, posted to LDS by the query's lane: the
// position and major axis, the level selection and probe count (packed as
// n << 12 | (E + 256) << 2 | mode) and, per fetch, the packed word base |
// k << 40 | flip << 45 and the edge id.
struct alignas(16) AnisoQuery {
    float u, v, au, av;
    float phi, om0;
    int32_t pack;
    int32_t e0;
    uint32_t w[6];
    int32_t e1, e2;
};
static_assert(sizeof(AnisoQuery) == 64, "one query in four 16-byte words");

__device__ __forceinline__ int32_t wave_inclusive_sum(int32_t x)
{
    const int lane = (int)__lane_id();
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const int32_t y = __shfl_up(x, d, 64);
        if (lane >= d) x += y;
    }
    return x;
}

__device__ __forceinline__ void wave_lds_sync()
{
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Whether a fetch at quad coordinates (x, y) (after Alg. 3's map; Alg. 2's
// reflection maps the test region onto itself) can reach a texel: within
// one texel of the coarsest level it samples around the unit square.  Taps
// farther out are out of bounds at both levels, so a fetch ruled out adds
// nothing.
__device__ __forceinline__ bool fetch_may_touch(const Lod &L, int k, float x, float y)
{
    int lv[2];
    float om[2];
    const int nl = fetch_levels(L, k, lv, om);
    const float h = ldexpf(1.0f, (nl == 2 ? lv[1] : lv[0]) - k);
    return (x >= -h) & (x <= 1.0f + h) & (y >= -h) & (y <= 1.0f + h);
}

__device__ __forceinline__ int mbcnt64(uint64_t b)
{
    return (int)__builtin_amdgcn_mbcnt_hi((uint32_t)(b >> 32),
                                          __builtin_amdgcn_mbcnt_lo((uint32_t)b, 0u));
}

__device__ __forceinline__ float bperm(int32_t byte_addr, float x)
{
    return __int_as_float(__builtin_amdgcn_ds_bpermute(byte_addr, __float_as_int(x)));
}
__device__ __forceinline__ int bperm(int32_t byte_addr, int x)
{
    return __builtin_amdgcn_ds_bpermute(byte_addr, x);
}

__device__ __forceinline__ Lod unpack_lod(const AnisoQuery &s)
{
    Lod L;
    L.mode = s.pack & 3;
    L.E = ((s.pack >> 2) & 1023) - 256;
    L.phi = s.phi;
    L.om0 = s.om0;
    return L;
}

__device__ __forceinline__ uint64_t word(const AnisoQuery &s, int f)
{
    return (uint64_t)s.w[2 * f + 1] << 32 | s.w[2 * f];
}

__device__ __forceinline__ int word_k(uint64_t w) { return (int)((w >> 40) & 31u); }

// The probes are dealt out over the wavefront: a query's N probes are N
// consecutive tasks (queries in lane order), the wave works through the
// tasks 64 at a time, and a lane finds the query of its task by binary
// search over the running task counts.  Lanes therefore stay busy whatever
// the spread of N within the wave, instead of all running the wave's
// largest N.  Each probe sums its three fetches in Alg. 3's order; the
// query's lane adds its probes' sums in probe order, so a query's result
// does not depend on the other queries of its wavefront.  Within a round a
// lane runs its probe's own-quad fetch itself; the Next and Prev fetches
// that can reach a texel (a long major axis carries most probes' neighbour
// fetches off their quads) are dealt out over the wavefront once more, and
// each probe pulls their results back by ds_bpermute in Alg. 3's order.
template <int DT, int CH, bool PREP>
__global__ void __launch_bounds__(kBlock) k_aniso(SampleArgs a, const float4 *jac, int max_aniso,
                                                  int32_t *nprobe)
{
    __shared__ AnisoQuery sq[kBlock / 64][64];
    __shared__ int32_t send[kBlock / 64][64];
    __shared__ float4 sc[kBlock / 64][64];
    __shared__ float sw[kBlock / 64][64];
    __shared__ uint8_t tl[kBlock / 64][128];
    const int lane = (int)__lane_id(), wv = threadIdx.x >> 6;
    const int64_t q = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (q - lane >= a.Q) return;   // the whole wavefront is past the end
    const bool live = q < a.Q;
    int32_t h = 0;
    float u = 0.0f, v = 0.0f;
    float4 J = make_float4(0.f, 0.f, 0.f, 0.f);
    if (live) {
        h = __builtin_nontemporal_load(a.qh + q);
        u = __builtin_nontemporal_load(a.qu + q);
        v = __builtin_nontemporal_load(a.qv + q);
        J = jac[q];
    }
    bool valid = live && (uint32_t)h < (uint32_t)a.H && isfinite(u) && isfinite(v) &&
                 isfinite(J.x) && isfinite(J.y) && isfinite(J.z) && isfinite(J.w);
    PrepRec rec = PrepRec{};
    if constexpr (PREP) {
        if (valid) {
            rec = static_cast<const PrepRec *>(a.prep)[h];
            valid = record_in_pool(rec, a.total_texels, a.has_mips != 0);
        }
    }
    if (live && !valid) {
        const float nan = __uint_as_float(0x7fc00000u);
        store_row<CH>(a.out, q, nan, nan, nan, nan);
        if (a.err) atomicAdd(a.err, 1);
        if (nprobe) nprobe[q] = 0;
    }
    int n = 0;
    if (valid) {
        AnisoQuery s;
        uint64_t w[3];
        int32_t e[3];
        if constexpr (PREP) {
#pragma unroll
            for (int f = 0; f < 3; ++f) {
                w[f] = rec.w[f];
                e[f] = rec.e[f];
            }
        } else {
            const int32_t g[3] = {h, a.next[h], a.prev[h]};
#pragma unroll
            for (int f = 0; f < 3; ++f) {
                e[f] = a.edge[g[f]];
                const bool flip = !(g[f] > a.twin[g[f]]);
                w[f] = (uint64_t)a.base[e[f]] | (uint64_t)a.log2res[e[f]] << 40 |
                       (uint64_t)(flip ? 1 : 0) << 45;
            }
        }
        const AnisoPlan A = aniso_plan(J, max_aniso);
        const Lod L = lod_of(A.f);
        n = A.n;
        s.u = u;
        s.v = v;
        s.au = A.au;
        s.av = A.av;
        s.phi = L.phi;
        s.om0 = L.om0;
        s.pack = A.n << 12 | (L.E + 256) << 2 | L.mode;
#pragma unroll
        for (int f = 0; f < 3; ++f) {
            s.w[2 * f] = (uint32_t)w[f];
            s.w[2 * f + 1] = (uint32_t)(w[f] >> 32);
        }
        s.e0 = e[0];
        s.e1 = e[1];
        s.e2 = e[2];
        sq[wv][lane] = s;
    }
    const int32_t end = wave_inclusive_sum(n), start = end - n;
    const int32_t T = __shfl(end, 63, 64);
    send[wv][lane] = end;
    wave_lds_sync();
    float4 C = make_float4(0.f, 0.f, 0.f, 0.f);
    float W = 0.0f;
    for (int32_t base = 0; base < T; base += 64) {
        const int32_t t = base + lane;
        const bool has = t < T;
        float4 Cp = make_float4(0.f, 0.f, 0.f, 0.f);
        float Wp = 0.0f;
        int o = 0;
        float ui = 0.0f, vi = 0.0f;
        bool need1 = false, need2 = false;
        if (has) {
            // the owner: the number of queries whose tasks all precede t
#pragma unroll
            for (int st = 32; st >= 1; st >>= 1)
                if (send[wv][o + st - 1] <= t) o += st;
            const AnisoQuery s = sq[wv][o];
            AnisoPlan A;
            A.n = s.pack >> 12;
            A.au = s.au;
            A.av = s.av;
            const Lod L = unpack_lod(s);
            const int i = t - (send[wv][o] - A.n) + 1;
            aniso_probe(A, i, s.u, s.v, ui, vi);
            // Alg. 3's own quad at (u, v), by this lane
            const FetchSpec f0 = {0, ui, vi, false, false};
            fetch<DT, CH, true, false>(a, L, f0, resolve_prepared<DT, CH>(a, word(s, 0), s.e0),
                                       Cp, Wp, nullptr, 0);
            // Next at (v, -u) and Prev at (-v, u), if they can reach a texel
            need1 = fetch_may_touch(L, word_k(word(s, 1)), vi, -ui);
            need2 = fetch_may_touch(L, word_k(word(s, 2)), -vi, ui);
        }
        // the Next and Prev fetches are dealt out to the wavefront (each
        // slot names the probe's lane; Next slots first)
        const uint64_t b1 = __ballot(need1), b2 = __ballot(need2);
        const int n1 = __popcll(b1), NT = n1 + __popcll(b2);
        const int s1 = mbcnt64(b1), s2 = n1 + mbcnt64(b2);
        if (need1) tl[wv][s1] = (uint8_t)lane;
        if (need2) tl[wv][s2] = (uint8_t)lane;
        wave_lds_sync();
        for (int tb = 0; tb < NT; tb += 64) {
            const int k = tb + lane;
            const bool nx = k < n1;   // a Next fetch, else a Prev fetch
            const int src = k < NT ? (int)tl[wv][k] << 2 : 0;
            const float uj = bperm(src, ui), vj = bperm(src, vi);
            const int oj = bperm(src, o);
            float4 Ct = make_float4(0.f, 0.f, 0.f, 0.f);
            float Wt = 0.0f;
            if (k < NT) {
                const AnisoQuery s = sq[wv][oj];
                const FetchSpec tf = {0, vj, uj, !nx, nx};
                fetch<DT, CH, true, false>(a, unpack_lod(s), tf,
                                           resolve_prepared<DT, CH>(a, word(s, nx ? 1 : 2),
                                                                    nx ? s.e1 : s.e2),
                                           Ct, Wt, nullptr, nx ? 1 : 2);
            }
            // each probe adds its fetches of this pass, Next before Prev
            const int r1 = s1 - tb, r2 = s2 - tb;
            const bool got1 = need1 && (uint32_t)r1 < 64u, got2 = need2 && (uint32_t)r2 < 64u;
            const int a1 = (r1 & 63) << 2, a2 = (r2 & 63) << 2;
            const float x1 = bperm(a1, Ct.x), x2 = bperm(a2, Ct.x);
            const float q1 = bperm(a1, Wt), q2 = bperm(a2, Wt);
            if constexpr (CH == 4) {
                const float y1 = bperm(a1, Ct.y), z1 = bperm(a1, Ct.z), w1 = bperm(a1, Ct.w);
                const float y2 = bperm(a2, Ct.y), z2 = bperm(a2, Ct.z), w2 = bperm(a2, Ct.w);
                if (got1) { Cp.x += x1; Cp.y += y1; Cp.z += z1; Cp.w += w1; Wp += q1; }
                if (got2) { Cp.x += x2; Cp.y += y2; Cp.z += z2; Cp.w += w2; Wp += q2; }
            } else {
                if (got1) { Cp.x += x1; Wp += q1; }
                if (got2) { Cp.x += x2; Wp += q2; }
            }
        }
        sc[wv][lane] = Cp;
        sw[wv][lane] = Wp;
        wave_lds_sync();
        // each query adds its probes of this round, in probe order
        const int32_t lo = max(start, base) - base, hi = min(end, base + 64) - base;
        for (int32_t j = lo; j < hi; ++j) {
            const float4 c = sc[wv][j];
            C.x += c.x;
            C.y += c.y;
            C.z += c.z;
            C.w += c.w;
            W += sw[wv][j];
        }
        wave_lds_sync();
    }
    if (valid) {
        const float r = __builtin_amdgcn_rcpf(W);
        store_row<CH>(a.out, q, C.x * r, C.y * r, C.z * r, C.w * r);
        if (nprobe) nprobe[q] = n;
    }
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
