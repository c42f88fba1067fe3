// htex_sample.hip -- batched Htex sampling (forward) and its transpose
// (backward scatter) for gfx950.
//
// One lane per query.  Per query: the halfedge operators Next/Prev/Twin/Edge
// (Section 2), Alg. 2's reflection for each of the three fetches of Alg. 3
// (own quad at (u, v), Next quad at (v, -u), Prev quad at (-v, u)), the
// OpenGL level pair for trilinear filtering, the bilinear taps of each level
// with a zero border, and the float32 blend normalized by the summed
// border-normalization channel (computed from the in-bounds tap weights, so
// it costs no memory).  This is a gather bound by HBM bandwidth: no MFMA.
//
// Integer tap bases are exact for every float32 input.  A quad coordinate
// is x = sigma * c + rho with c the query's u or v, sigma = +-1 and rho in
// {0, 1} (Alg. 2 and the neighbour maps).  With t = |c| n (exact: n is a
// power of two), q = floor(t) and r = t - q (exact), x n - 1/2 equals
// rho n + q + r - 1/2 when sigma c >= 0 and rho n - q - r - 1/2 otherwise, so
// floor and fraction follow from q, r and the comparison of r with 1/2,
// without ever forming 1 - c (which would round).
#include <hip/hip_runtime.h>

#include "htex_internal.h"

namespace htex {
namespace {

constexpr int kBlock = 256;

struct AxisTaps {
    int32_t i0;  // floor(x n - 1/2)
    float w0;    // weight of tap i0:     1 - a, a = x n - 1/2 - i0
    float w1;    // weight of tap i0 + 1: a
};

// x = (neg ? -1 : 1) * c + rho, sampled on a level of n = 2^m texels.  Both
// weights are formed from the exact fraction r without cancellation (each
// within an ulp of its exact value, however close to 0 it is).  Written with
// selects only, so lanes with different signs do not diverge.
__device__ __forceinline__ AxisTaps axis_taps(float c, bool neg, int rho, int m)
{
    const bool eneg = neg != ((__float_as_uint(c) >> 31) != 0u);
    const float t = ldexpf(fminf(fabsf(c), 4.0f), m);
    const float qf = floorf(t);
    const float r = t - qf;
    const int32_t q = (int32_t)qf;
    // x n - 1/2 = rn + q + r - 1/2 (eneg false) or rn - q - r - 1/2 (eneg true)
    const bool up = (r > 0.5f) | ((!eneg) & (r == 0.5f));
    const float fr = r + (up ? -0.5f : 0.5f);   // exact when up
    const float cf = (up ? 1.5f : 0.5f) - r;    // exact when up
    AxisTaps o;
    o.w1 = eneg ? cf : fr;
    o.w0 = eneg ? fr : cf;
    const int32_t G = q + (up ? 1 : 0);
    o.i0 = (rho << m) - 1 + (eneg ? -G : G);
    return o;
}

// One texel widened to float32: CH = 4 channels (RGBA) or 1 (a scalar map,
// returned in .x with the other lanes zero).
template <int DT, int CH>
__device__ __forceinline__ float4 load_texel(const char *p)
{
    if constexpr (CH == 4) {
        if constexpr (DT == HTEX_F32) {
            return *reinterpret_cast<const float4 *>(p);
        } else if constexpr (DT == HTEX_BF16) {
            const uint2 b = *reinterpret_cast<const uint2 *>(p);
            return make_float4(__uint_as_float(b.x << 16), __uint_as_float(b.x & 0xffff0000u),
                               __uint_as_float(b.y << 16), __uint_as_float(b.y & 0xffff0000u));
        } else {
            // OCP E4M3 -> float32 with gfx950's packed converter (exact for
            // all 256 codes, subnormals and NaN included)
            const int b = *reinterpret_cast<const int *>(p);
            const auto lo = __builtin_amdgcn_cvt_pk_f32_fp8(b, false);
            const auto hi = __builtin_amdgcn_cvt_pk_f32_fp8(b, true);
            return make_float4(lo[0], lo[1], hi[0], hi[1]);
        }
    } else {
        float x;
        if constexpr (DT == HTEX_F32) {
            x = *reinterpret_cast<const float *>(p);
        } else if constexpr (DT == HTEX_BF16) {
            x = __uint_as_float((uint32_t)*reinterpret_cast<const uint16_t *>(p) << 16);
        } else {
            x = __builtin_amdgcn_cvt_f32_fp8((int)*reinterpret_cast<const uint8_t *>(p), 0);
        }
        return make_float4(x, 0.0f, 0.0f, 0.0f);
    }
}

// log2(z) for z in [1/2, 2] through the series of atanh:
// log2(z) = (2 / ln 2) atanh(s), s = (z - 1) / (z + 1), here with
// |s| <= 1/3 so eight odd terms leave a relative truncation error below
// 2e-9.  The result keeps full relative precision when it is near zero, as
// long as z - 1 is passed exactly (numerator and denominator separately).
__device__ __forceinline__ float log2_atanh(float num, float den)
{
    const float s = num * __builtin_amdgcn_rcpf(den);
    const float s2 = s * s;
    float p = 1.923593388e-01f;
    p = fmaf(p, s2, 2.219530832e-01f);
    p = fmaf(p, s2, 2.623081893e-01f);
    p = fmaf(p, s2, 3.205988980e-01f);
    p = fmaf(p, s2, 4.121985831e-01f);
    p = fmaf(p, s2, 5.770780164e-01f);
    p = fmaf(p, s2, 9.617966939e-01f);
    p = fmaf(p, s2, 2.885390082e+00f);
    return s * p;
}

// Trilinear level selection from the footprint: f = m 2^E, m in [1, 2);
// floor(lambda) = E + k, frac(lambda) = log2(m).  `mode`: 0 = level 0 only,
// 1 = coarsest level only, 2 = level pair (E + k, E + k + 1) unless clamped
// per fetch.  The blend weights phi = log2(m) and 1 - phi = log2(2 / m) are
// each evaluated directly (m - 1 and 2 - m are exact), so each keeps full
// relative precision when it is close to zero.
struct Lod {
    int mode;
    int E;
    float phi;   // weight of the coarser level
    float om0;   // weight of the finer level, 1 - phi
};

__device__ __forceinline__ Lod lod_of(float f)
{
    Lod L{0, 0, 0.0f, 1.0f};
    const uint32_t b = __float_as_uint(f);
    const uint32_t ex = (b >> 23) & 0xffu;
    const bool finite_pos_normal = (f > 0.0f) & (ex != 0u) & (ex != 0xffu);
    L.mode = finite_pos_normal ? 2 : (b == 0x7f800000u ? 1 : 0);
    L.E = (int)ex - 127;
    const float m = __uint_as_float((b & 0x7fffffu) | 0x3f800000u);
    L.phi = finite_pos_normal ? log2_atanh(m - 1.0f, m + 1.0f) : 0.0f;
    L.om0 = finite_pos_normal ? log2_atanh(2.0f - m, 2.0f + m) : 1.0f;
    return L;
}

// Levels and weights of one fetch on a texture of log2 resolution k
// (selects only).  Returns the number of levels (1 or 2).
__device__ __forceinline__ int fetch_levels(const Lod &L, int k, int lv[2], float om[2])
{
    const int li = L.E + k;
    const bool pair = (L.mode == 2) && li >= 0 && li < k;
    const bool coarsest = (L.mode == 1) || (L.mode == 2 && li >= k);
    lv[0] = pair ? li : (coarsest ? k : 0);
    lv[1] = pair ? li + 1 : -1;
    om[0] = pair ? L.om0 : 1.0f;
    om[1] = pair ? L.phi : 0.0f;
    return pair ? 2 : 1;
}

// The three fetches of Alg. 3: halfedge and (raw coordinate, negated?) for x, y.
struct FetchSpec {
    int32_t g;
    float cx, cy;
    bool nx, ny;
};

__device__ __forceinline__ void fetch_specs(int32_t h, int32_t n1, int32_t p1, float u, float v,
                                            FetchSpec fs[3])
{
    fs[0] = {h, u, v, false, false};    // own quad at (u, v)
    fs[1] = {n1, v, u, false, true};    // Next quad at (v, -u)
    fs[2] = {p1, v, u, true, false};    // Prev quad at (-v, u)
}

// Texel offset of level l inside an edge of log2 resolution k, 32-bit:
// sum_{m<l} 4^(k-m) = 4^(k-l+1) (4^l - 1) / 3, and (4^l - 1) / 3 is the bit
// pattern 0101...01 with l ones (at most 1.43e9 texels for k = 15).
__device__ __forceinline__ uint32_t level_offset32(int k, int l)
{
    const uint32_t ones = l ? (0x55555555u >> (32 - 2 * l)) : 0u;
    return ones << (2 * (k - l) + 2);
}

template <int DT, int CH> struct TexelBytes {
    static constexpr int v = (DT == HTEX_F32 ? 4 : DT == HTEX_BF16 ? 2 : 1) * CH;
};

// One mip level of one fetch, planned before any texel is read: the
// bilinear taps (i0 + di, j0 + dj), their weights with the level weight `om`
// folded into the row weights and zeroed for out-of-bounds taps, and four
// clamped in-bounds texel offsets (so the loads of a partly covered level
// are harmless for the zero-weight taps).  `act` is false when no tap is in
// bounds; such a level is not read at all.  The level's normalization
// channel is om (wx0 + wx1)(wy0 + wy1).
struct LevelPlan {
    bool act;
    int32_t i0, j0;
    int mask;  // in-bounds taps, bit 2 dj + di
    float wx0, wx1, wy0, wy1;
    uint32_t o00, o01, o10, o11;
};

__device__ __forceinline__ LevelPlan plan_level(int k, int l, float om, const FetchSpec &fs, bool flip)
{
    const int m = k - l;
    const int32_t n = 1 << m;
    const AxisTaps X = axis_taps(fs.cx, fs.nx ^ flip, flip ? 1 : 0, m);
    const AxisTaps Y = axis_taps(fs.cy, fs.ny ^ flip, flip ? 1 : 0, m);
    const bool bx0 = (uint32_t)X.i0 < (uint32_t)n, bx1 = (uint32_t)(X.i0 + 1) < (uint32_t)n;
    const bool by0 = (uint32_t)Y.i0 < (uint32_t)n, by1 = (uint32_t)(Y.i0 + 1) < (uint32_t)n;
    LevelPlan p;
    p.act = (bx0 | bx1) & (by0 | by1);
    p.i0 = X.i0;
    p.j0 = Y.i0;
    p.mask = ((bx0 & by0) ? 1 : 0) | ((bx1 & by0) ? 2 : 0) | ((bx0 & by1) ? 4 : 0) | ((bx1 & by1) ? 8 : 0);
    p.wx0 = bx0 ? X.w0 : 0.0f;
    p.wx1 = bx1 ? X.w1 : 0.0f;
    p.wy0 = by0 ? om * Y.w0 : 0.0f;
    p.wy1 = by1 ? om * Y.w1 : 0.0f;
    const int32_t ic0 = min(max(X.i0, 0), n - 1), ic1 = min(max(X.i0 + 1, 0), n - 1);
    const int32_t jc0 = min(max(Y.i0, 0), n - 1), jc1 = min(max(Y.i0 + 1, 0), n - 1);
    const uint32_t lo = level_offset32(k, l);
    const uint32_t r0 = lo + (uint32_t)(jc0 << m), r1 = lo + (uint32_t)(jc1 << m);
    p.o00 = r0 + ic0;
    p.o01 = r0 + ic1;
    p.o10 = r1 + ic0;
    p.o11 = r1 + ic1;
    return p;
}

template <int CH>
__device__ __forceinline__ void accumulate(const LevelPlan &p, const float4 &t00, const float4 &t01,
                                           const float4 &t10, const float4 &t11, float4 &Cf,
                                           float &Wf)
{
    const float w00 = p.wx0 * p.wy0, w01 = p.wx1 * p.wy0, w10 = p.wx0 * p.wy1, w11 = p.wx1 * p.wy1;
    if constexpr (CH == 4) {
        Cf.x += w00 * t00.x; Cf.y += w00 * t00.y; Cf.z += w00 * t00.z; Cf.w += w00 * t00.w;
        Cf.x += w01 * t01.x; Cf.y += w01 * t01.y; Cf.z += w01 * t01.z; Cf.w += w01 * t01.w;
        Cf.x += w10 * t10.x; Cf.y += w10 * t10.y; Cf.z += w10 * t10.z; Cf.w += w10 * t10.w;
        Cf.x += w11 * t11.x; Cf.y += w11 * t11.y; Cf.z += w11 * t11.z; Cf.w += w11 * t11.w;
    } else {
        Cf.x += w00 * t00.x;
        Cf.x += w01 * t01.x;
        Cf.x += w10 * t10.x;
        Cf.x += w11 * t11.x;
    }
    Wf += (p.wx0 + p.wx1) * (p.wy0 + p.wy1);
}

// A fetch with its halfedge resolved: the quad's edge e, its log2
// resolution k, the reflection of Alg. 2 and the address of its level 0.
struct Resolved {
    int32_t e;
    int k;
    bool flip;
    const char *ep;
};

template <int DT, int CH>
__device__ __forceinline__ Resolved resolve_plain(const SampleArgs &a, int32_t g)
{
    Resolved r;
    r.flip = !(g > a.twin[g]);
    r.e = a.edge[g];
    r.k = a.log2res[r.e];
    r.ep = static_cast<const char *>(a.texels) + a.base[r.e] * TexelBytes<DT, CH>::v;
    return r;
}

// One of Alg. 3's fetches: Texture(Edge(g), TriangleToQuadUV(g, <x, y>)),
// colour and normalization channel.  Both mip levels are planned first and
// read under a single branch, so their eight loads are in flight together.
template <int DT, int CH, bool TRI, bool DBG>
__device__ __forceinline__ void fetch(const SampleArgs &a, const Lod &L, const FetchSpec &f,
                                      const Resolved &R, float4 &Cf, float &Wf,
                                      htex_debug_rec *d, int s)
{
    constexpr int TB = TexelBytes<DT, CH>::v;
    const int k = R.k;
    const bool flip = R.flip;
    const char *ep = R.ep;
    int lv[2];
    float om[2];
    const int nlev = fetch_levels(L, k, lv, om);
    const LevelPlan p0 = plan_level(k, lv[0], om[0], f, flip);
    LevelPlan p1;
    if constexpr (TRI) {
        p1 = plan_level(k, nlev == 2 ? lv[1] : lv[0], om[1], f, flip);
        p1.act = p1.act & (nlev == 2);
    }
    if (p0.act | (TRI && p1.act)) {
        const float4 t00 = load_texel<DT, CH>(ep + (uint64_t)p0.o00 * TB);
        const float4 t01 = load_texel<DT, CH>(ep + (uint64_t)p0.o01 * TB);
        const float4 t10 = load_texel<DT, CH>(ep + (uint64_t)p0.o10 * TB);
        const float4 t11 = load_texel<DT, CH>(ep + (uint64_t)p0.o11 * TB);
        if constexpr (TRI) {
            const float4 u00 = load_texel<DT, CH>(ep + (uint64_t)p1.o00 * TB);
            const float4 u01 = load_texel<DT, CH>(ep + (uint64_t)p1.o01 * TB);
            const float4 u10 = load_texel<DT, CH>(ep + (uint64_t)p1.o10 * TB);
            const float4 u11 = load_texel<DT, CH>(ep + (uint64_t)p1.o11 * TB);
            if (p0.act) accumulate<CH>(p0, t00, t01, t10, t11, Cf, Wf);
            if (p1.act) accumulate<CH>(p1, u00, u01, u10, u11, Cf, Wf);
        } else {
            accumulate<CH>(p0, t00, t01, t10, t11, Cf, Wf);
        }
        if constexpr (DT == HTEX_FP8_E4M3) {
            const float sc = a.scale[R.e];
            Cf.x *= sc;
            if constexpr (CH == 4) {
                Cf.y *= sc;
                Cf.z *= sc;
                Cf.w *= sc;
            }
        }
    }
    if constexpr (DBG) {
        d->edge[s] = R.e;
        d->flip[s] = flip ? 1 : 0;
        d->level[s][0] = lv[0];
        d->level[s][1] = lv[1];
        d->i0[s][0] = p0.i0;
        d->j0[s][0] = p0.j0;
        d->inb[s][0] = p0.mask;
        if (TRI && nlev == 2) {
            d->i0[s][1] = p1.i0;
            d->j0[s][1] = p1.j0;
            d->inb[s][1] = p1.mask;
        }
        d->wf[s] = Wf;
    }
}

// Prepared record of halfedge h: for its three fetches the packed word
// base | k << 40 | flip << 45 and the edge id, then Next(h) and Prev(h).
struct alignas(16) PrepRec {
    uint64_t w[3];
    int32_t e[3];
    int32_t next, prev, pad;
};
static_assert(sizeof(PrepRec) == HTEX_PREP_BYTES, "record size");

template <int DT, int CH>
__device__ __forceinline__ Resolved resolve_prepared(const SampleArgs &a, uint64_t w, int32_t e)
{
    Resolved r;
    r.e = e;
    r.k = (int)((w >> 40) & 31u);
    r.flip = ((w >> 45) & 1u) != 0;
    r.ep = static_cast<const char *>(a.texels) +
           (int64_t)(w & 0xffffffffffull) * TexelBytes<DT, CH>::v;
    return r;
}

typedef float f32x4 __attribute__((ext_vector_type(4)));

// Result row q (CH floats), streamed past the caches.
template <int CH>
__device__ __forceinline__ void store_row(float *out, int64_t q, float x, float y, float z, float w)
{
    if constexpr (CH == 4) {
        const f32x4 v = {x, y, z, w};
        __builtin_nontemporal_store(v, reinterpret_cast<f32x4 *>(out) + q);
    } else {
        __builtin_nontemporal_store(x, out + q);
    }
}

template <int CH>
__device__ __forceinline__ float4 load_row(const float *in, int64_t q)
{
    if constexpr (CH == 4) return reinterpret_cast<const float4 *>(in)[q];
    else return make_float4(in[q], 0.0f, 0.0f, 0.0f);
}

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
template <int DT, int CH, bool TRI>
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
        fetch<DT, CH, TRI, false>(a, L, fs[s], resolve_prepared<DT, CH>(a, rec.w[s], rec.e[s]),
                                  Cf, Wf, nullptr, s);
        C.x += Cf.x;
        C.y += Cf.y;
        C.z += Cf.z;
        C.w += Cf.w;
        W += Wf;
    }
    const float r = __builtin_amdgcn_rcpf(W);
    store_row<CH>(a.out, q, C.x * r, C.y * r, C.z * r, C.w * r);
}

template <int DT, int CH, bool TRI>
__global__ void __launch_bounds__(kBlock) k_sample_prep(SampleArgs a)
{
    const int64_t q = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (q >= a.Q) return;
    sample_one_prepared<DT, CH, TRI>(a, q);
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
            sample_one_prepared<DT, CH, TRI>(a, T.q0 + threadIdx.x);
        }
    }
}

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

// Backward: out_c = sum over taps (om w / W) T_c, so dL/dT_c at each tap
// receives (om w / W) dL/dout_c.  First the normalization W (weights only,
// no texel reads), then the scatter with float32 atomics.
template <int CH, bool TRI>
__global__ void __launch_bounds__(kBlock) k_backward(SampleArgs a)
{
    const int64_t q = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (q >= a.Q) return;
    const int32_t h = a.qh[q];
    const float u = a.qu[q], v = a.qv[q];
    if (!((uint32_t)h < (uint32_t)a.H) || !isfinite(u) || !isfinite(v)) return;
    const int32_t n1 = a.next[h], p1 = a.prev[h];
    Lod L{0, 0, 0.0f, 1.0f};
    if constexpr (TRI) L = lod_of(a.qf[q]);
    FetchSpec fs[3];
    fetch_specs(h, n1, p1, u, v, fs);
    int32_t es[3], ks[3];
    bool flips[3];
    float W = 0.0f;
#pragma unroll
    for (int s = 0; s < 3; ++s) {
        const int32_t g = fs[s].g;
        flips[s] = !(g > a.twin[g]);
        es[s] = a.edge[g];
        ks[s] = a.log2res[es[s]];
        int lv[2];
        float om[2];
        const int nlev = fetch_levels(L, ks[s], lv, om);
        for (int sl = 0; sl < nlev; ++sl) {
            const int m = ks[s] - lv[sl];
            const int32_t n = 1 << m;
            const AxisTaps X = axis_taps(fs[s].cx, fs[s].nx ^ flips[s], flips[s] ? 1 : 0, m);
            const AxisTaps Y = axis_taps(fs[s].cy, fs[s].ny ^ flips[s], flips[s] ? 1 : 0, m);
            for (int dj = 0; dj < 2; ++dj)
                for (int di = 0; di < 2; ++di) {
                    const int32_t i = X.i0 + di, j = Y.i0 + dj;
                    if ((uint32_t)i < (uint32_t)n && (uint32_t)j < (uint32_t)n)
                        W += om[sl] * ((di ? X.w1 : X.w0) * (dj ? Y.w1 : Y.w0));
                }
        }
    }
    const float4 g4 = load_row<CH>(a.dout, q);
    const float r = 1.0f / W;
#pragma unroll
    for (int s = 0; s < 3; ++s) {
        int lv[2];
        float om[2];
        const int nlev = fetch_levels(L, ks[s], lv, om);
        const int64_t eb = a.base[es[s]];
        for (int sl = 0; sl < nlev; ++sl) {
            const int m = ks[s] - lv[sl];
            const int32_t n = 1 << m;
            const AxisTaps X = axis_taps(fs[s].cx, fs[s].nx ^ flips[s], flips[s] ? 1 : 0, m);
            const AxisTaps Y = axis_taps(fs[s].cy, fs[s].ny ^ flips[s], flips[s] ? 1 : 0, m);
            const int64_t lvb = eb + level_offset(ks[s], lv[sl]);
            for (int dj = 0; dj < 2; ++dj)
                for (int di = 0; di < 2; ++di) {
                    const int32_t i = X.i0 + di, j = Y.i0 + dj;
                    if ((uint32_t)i < (uint32_t)n && (uint32_t)j < (uint32_t)n) {
                        const float w =
                            om[sl] * ((di ? X.w1 : X.w0) * (dj ? Y.w1 : Y.w0)) * r;
                        float *p = a.dtex + CH * (lvb + (int64_t)j * n + i);
                        unsafeAtomicAdd(p + 0, w * g4.x);
                        if constexpr (CH == 4) {
                            unsafeAtomicAdd(p + 1, w * g4.y);
                            unsafeAtomicAdd(p + 2, w * g4.z);
                            unsafeAtomicAdd(p + 3, w * g4.w);
                        }
                    }
                }
        }
    }
}

// Backward with a per-workgroup cache of gradient tiles in LDS.  A block
// takes kBwdChunk consecutive queries (sorted queries meet few textures
// there) and accumulates each tap into an on-chip tile holding one whole
// (edge, level) of the gradient.  Tiles live in an arena of kArenaFloats
// floats, found through an open-addressing table of kTiles 64-bit entries
// (key << 32 | arena offset) keyed by edge * 16 + level.  The first lane to
// meet a key claims a free entry with a compare-and-swap (marking it
// pending), reserves the level's texels with an atomic bump and publishes
// the offset; lanes that meet the key while it is pending, or whose level
// does not fit, or that find the table full, add their taps straight to
// the gradient pool with global atomics.  A key is never claimed twice.
// At the end every tile is added to the pool once, one float atomic per
// non-zero texel channel.  Trilinear batches touch about 3 edges x 6
// levels per block, which is why tiles are sized per level.
constexpr int kTiles = 32;
constexpr int kArenaFloats = 16384;   // 64 KB
constexpr int kBwdPerThread = 16;
constexpr int kBwdChunk = kBlock * kBwdPerThread;

template <int CH, bool TRI>
__global__ void __launch_bounds__(kBlock) k_backward_lds(SampleArgs a)
{
    __shared__ float arena[kArenaFloats];
    // entry = key << 32 | offset, read and written as one 64-bit word; the
    // low word is an arena offset, kPending while its owner reserves space,
    // or kNoRoom; kFree marks an unclaimed entry
    __shared__ uint64_t entry[kTiles];
    __shared__ int32_t used;
    constexpr uint64_t kFree = ~0ull;
    constexpr uint32_t kPending = 0xfffffffeu, kNoRoom = 0xfffffffdu;
    for (int i = threadIdx.x; i < kArenaFloats; i += kBlock) arena[i] = 0.0f;
    if (threadIdx.x < kTiles) entry[threadIdx.x] = kFree;
    if (threadIdx.x == 0) used = 0;
    __syncthreads();
    const int64_t q0 = (int64_t)blockIdx.x * kBwdChunk;
    // the last tile each of a lane's six (fetch, level) slots resolved: a
    // lane's consecutive queries are usually on the same halfedge
    int32_t memo_key[3][2], memo_base[3][2];
#pragma unroll
    for (int s = 0; s < 3; ++s)
        for (int sl = 0; sl < 2; ++sl) memo_key[s][sl] = -1;
    for (int r = 0; r < kBwdPerThread; ++r) {
        const int64_t q = q0 + (int64_t)r * kBlock + threadIdx.x;
        if (q >= a.Q) break;
        const int32_t h = a.qh[q];
        const float u = a.qu[q], v = a.qv[q];
        if (!((uint32_t)h < (uint32_t)a.H) || !isfinite(u) || !isfinite(v)) continue;
        const int32_t n1 = a.next[h], p1 = a.prev[h];
        Lod L{0, 0, 0.0f, 1.0f};
        if constexpr (TRI) L = lod_of(a.qf[q]);
        FetchSpec fs[3];
        fetch_specs(h, n1, p1, u, v, fs);
        int32_t es[3], ks[3];
        bool flips[3];
        float W = 0.0f;
#pragma unroll
        for (int s = 0; s < 3; ++s) {
            const int32_t g = fs[s].g;
            flips[s] = !(g > a.twin[g]);
            es[s] = a.edge[g];
            ks[s] = a.log2res[es[s]];
            int lv[2];
            float om[2];
            const int nlev = fetch_levels(L, ks[s], lv, om);
            for (int sl = 0; sl < nlev; ++sl) {
                const LevelPlan p = plan_level(ks[s], lv[sl], om[sl], fs[s], flips[s]);
                W += (p.wx0 + p.wx1) * (p.wy0 + p.wy1);
            }
        }
        const float4 g4 = load_row<CH>(a.dout, q);
        const float rW = 1.0f / W;
#pragma unroll
        for (int s = 0; s < 3; ++s) {
            int lv[2];
            float om[2];
            const int nlev = fetch_levels(L, ks[s], lv, om);
            const int64_t eb = a.base[es[s]];
#pragma unroll
            for (int sl = 0; sl < 2; ++sl) {
                if (sl >= nlev) break;
                const LevelPlan p = plan_level(ks[s], lv[sl], om[sl], fs[s], flips[s]);
                if (!p.act) continue;
                const int m = ks[s] - lv[sl];
                const uint32_t lo = level_offset32(ks[s], lv[sl]);
                // the tile of this (edge, level): remembered, found, or claimed
                const int32_t key = es[s] * 16 + lv[sl];
                // floats of this level's tile (computed in 64 bits: a level of
                // 2^15 x 2^15 RGBA texels needs 2^32 floats; it never fits)
                const int64_t need = (int64_t)CH << (2 * m);
                int32_t base_f = -1;
                const uint32_t h0 = ((uint32_t)key * 2654435761u) >> 27;   // 5 bits
                if (memo_key[s][sl] == key) base_f = memo_base[s][sl];
                else for (int pr = 0; pr < kTiles; ++pr) {
                    const int t = (int)((h0 + pr) & (kTiles - 1));
                    uint64_t en = __atomic_load_n(&entry[t], __ATOMIC_RELAXED);
                    if (en == kFree) {
                        const uint64_t mine = ((uint64_t)(uint32_t)key << 32) | kPending;
                        en = atomicCAS(&entry[t], kFree, mine);
                        if (en == kFree) {   // claimed: reserve the level's texels
                            const int32_t o = need <= kArenaFloats
                                                  ? atomicAdd(&used, (int32_t)need)
                                                  : kArenaFloats;
                            const bool fits = o + need <= kArenaFloats;
                            atomicExch(&entry[t], ((uint64_t)(uint32_t)key << 32) |
                                                      (fits ? (uint32_t)o : kNoRoom));
                            if (fits) base_f = o;
                            break;
                        }
                    }
                    if ((uint32_t)(en >> 32) == (uint32_t)key) {
                        const uint32_t lo32 = (uint32_t)(en & 0xffffffffu);
                        if (lo32 < (uint32_t)kArenaFloats) base_f = (int32_t)lo32;
                        break;   // pending or no room: global atomics
                    }
                }
                if (base_f >= 0) {
                    memo_key[s][sl] = key;
                    memo_base[s][sl] = base_f;
                }
                const float w[4] = {p.wx0 * p.wy0, p.wx1 * p.wy0, p.wx0 * p.wy1, p.wx1 * p.wy1};
                const uint32_t off[4] = {p.o00, p.o01, p.o10, p.o11};
#pragma unroll
                for (int t = 0; t < 4; ++t) {
                    if (!((p.mask >> t) & 1)) continue;
                    const float wt = w[t] * rW;
                    if (base_f >= 0) {
                        float *c = &arena[base_f + CH * (int32_t)(off[t] - lo)];
                        atomicAdd(c + 0, wt * g4.x);
                        if constexpr (CH == 4) {
                            atomicAdd(c + 1, wt * g4.y);
                            atomicAdd(c + 2, wt * g4.z);
                            atomicAdd(c + 3, wt * g4.w);
                        }
                    } else {
                        float *pg = a.dtex + CH * (eb + off[t]);
                        unsafeAtomicAdd(pg + 0, wt * g4.x);
                        if constexpr (CH == 4) {
                            unsafeAtomicAdd(pg + 1, wt * g4.y);
                            unsafeAtomicAdd(pg + 2, wt * g4.z);
                            unsafeAtomicAdd(pg + 3, wt * g4.w);
                        }
                    }
                }
            }
        }
    }
    __syncthreads();
    // flush the tiles
    for (int t = 0; t < kTiles; ++t) {
        const uint64_t en = entry[t];
        if (en == kFree || (uint32_t)(en & 0xffffffffu) >= (uint32_t)kArenaFloats) continue;
        const int32_t key = (int32_t)(en >> 32);
        const int32_t e = key >> 4, l = key & 15;
        const int k = a.log2res[e];
        const int cnt = CH << (2 * (k - l));
        float *dst = a.dtex + CH * (a.base[e] + level_offset32(k, l));
        const float *src = &arena[(int32_t)(en & 0xffffffffu)];
        for (int i = threadIdx.x; i < cnt; i += kBlock) {
            const float val = src[i];
            if (val != 0.0f) unsafeAtomicAdd(dst + i, val);
        }
    }
}

inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

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

template <int DT, int CH, bool TRI>
hipError_t launch_fwd_prep(const SampleArgs &a, hipStream_t s)
{
    const uint32_t G = (uint32_t)ceil_div(a.Q, kBlock);
    hipLaunchKernelGGL((k_sample_prep<DT, CH, TRI>), dim3(G), dim3(kBlock), 0, s, a);
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
        return launch_fwd_prep<DT, CH, TRI>(a, s);
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

hipError_t launch_sample_prepared(const SampleArgs &a, int dtype, int filter, hipStream_t s)
{
    if (a.Q == 0) return hipSuccess;
    return dispatch<FwdPrep>(a, dtype, filter, s);
}

hipError_t launch_sample(const SampleArgs &a, int dtype, int filter, hipStream_t s)
{
    if (a.Q == 0) return hipSuccess;
    return dispatch<Fwd>(a, dtype, filter, s);
}

template <int CH, bool TRI>
hipError_t launch_bwd(const SampleArgs &a, uint32_t flags, hipStream_t s)
{
    if (flags & HTEX_QUERIES_SORTED) {
        // sorted batches meet few textures per block: cache their gradients in LDS
        const uint32_t G = (uint32_t)ceil_div(a.Q, kBwdChunk);
        hipLaunchKernelGGL((k_backward_lds<CH, TRI>), dim3(G), dim3(kBlock), 0, s, a);
    } else {
        const uint32_t G = (uint32_t)ceil_div(a.Q, kBlock);
        hipLaunchKernelGGL((k_backward<CH, TRI>), dim3(G), dim3(kBlock), 0, s, a);
    }
    return hipGetLastError();
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

hipError_t launch_backward(const SampleArgs &a, int filter, uint32_t flags, hipStream_t s)
{
    if (a.Q == 0) return hipSuccess;
    const bool tri = filter == HTEX_TRILINEAR;
    if (a.channels == 1)
        return tri ? launch_bwd<1, true>(a, flags, s) : launch_bwd<1, false>(a, flags, s);
    return tri ? launch_bwd<4, true>(a, flags, s) : launch_bwd<4, false>(a, flags, s);
}

}  // namespace htex
