// htex_filter.h -- device building blocks of Htex sampling shared by the
// forward, anisotropic and backward kernels (htex_sample.hip,
// htex_aniso.hip, htex_backward.hip): exact tap bases, texel decoding,
// level selection, the three fetches of Alg. 3 and their level plans, the
// prepared per-halfedge records, result rows.  Private to libhtex.
//
// Integer tap bases are exact for every float32 input.  A quad coordinate
// is x = sigma * c + rho with c the query's u or v, sigma = +-1 and rho in
// {0, 1} (Alg. 2 and the neighbour maps).  With t = |c| n (exact: n is a
// power of two), q = floor(t) and r = t - q (exact), x n - 1/2 equals
// rho n + q + r - 1/2 when sigma c >= 0 and rho n - q - r - 1/2 otherwise, so
// floor and fraction follow from q, r and the comparison of r with 1/2,
// without ever forming 1 - c (which would round).
#pragma once

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

template <int CH>
__device__ __forceinline__ void accumulate_tap(float w, const float4 &t, float4 &Cf)
{
    Cf.x += w * t.x;
    if constexpr (CH == 4) {
        Cf.y += w * t.y;
        Cf.z += w * t.z;
        Cf.w += w * t.w;
    }
}

// The same fetch with one predicate per tap: only in-bounds taps are read
// and blended (bit-identical to `fetch`: a skipped tap's term is a zero
// weight times a finite texel).  For scattered batches, where every lane's
// taps lie in lines no other lane touches, each skipped tap saves a line
// fetch; in halfedge-sorted batches the neighbouring lanes read those lines
// anyway and the extra predicates cost more than the loads.
template <int DT, int CH, bool TRI>
__device__ __forceinline__ void fetch_in_bounds(const SampleArgs &a, const Lod &L,
                                                const FetchSpec &f, const Resolved &R,
                                                float4 &Cf, float &Wf)
{
    constexpr int TB = TexelBytes<DT, CH>::v;
    int lv[2];
    float om[2];
    const int nlev = fetch_levels(L, R.k, lv, om);
    const LevelPlan p0 = plan_level(R.k, lv[0], om[0], f, R.flip);
    LevelPlan p1;
    int m1 = 0;
    if constexpr (TRI) {
        p1 = plan_level(R.k, nlev == 2 ? lv[1] : lv[0], om[1], f, R.flip);
        m1 = (p1.act && nlev == 2) ? p1.mask : 0;
    }
    const int m0 = p0.act ? p0.mask : 0;
    if ((m0 | m1) == 0) return;
    const char *ep = R.ep;
    // every load is issued before the first blend term waits for one
    float4 t00, t01, t10, t11, u00, u01, u10, u11;
    if (m0 & 1) t00 = load_texel<DT, CH>(ep + (uint64_t)p0.o00 * TB);
    if (m0 & 2) t01 = load_texel<DT, CH>(ep + (uint64_t)p0.o01 * TB);
    if (m0 & 4) t10 = load_texel<DT, CH>(ep + (uint64_t)p0.o10 * TB);
    if (m0 & 8) t11 = load_texel<DT, CH>(ep + (uint64_t)p0.o11 * TB);
    if constexpr (TRI) {
        if (m1 & 1) u00 = load_texel<DT, CH>(ep + (uint64_t)p1.o00 * TB);
        if (m1 & 2) u01 = load_texel<DT, CH>(ep + (uint64_t)p1.o01 * TB);
        if (m1 & 4) u10 = load_texel<DT, CH>(ep + (uint64_t)p1.o10 * TB);
        if (m1 & 8) u11 = load_texel<DT, CH>(ep + (uint64_t)p1.o11 * TB);
    }
    if (m0) {
        if (m0 & 1) accumulate_tap<CH>(p0.wx0 * p0.wy0, t00, Cf);
        if (m0 & 2) accumulate_tap<CH>(p0.wx1 * p0.wy0, t01, Cf);
        if (m0 & 4) accumulate_tap<CH>(p0.wx0 * p0.wy1, t10, Cf);
        if (m0 & 8) accumulate_tap<CH>(p0.wx1 * p0.wy1, t11, Cf);
        Wf += (p0.wx0 + p0.wx1) * (p0.wy0 + p0.wy1);
    }
    if constexpr (TRI) {
        if (m1) {
            if (m1 & 1) accumulate_tap<CH>(p1.wx0 * p1.wy0, u00, Cf);
            if (m1 & 2) accumulate_tap<CH>(p1.wx1 * p1.wy0, u01, Cf);
            if (m1 & 4) accumulate_tap<CH>(p1.wx0 * p1.wy1, u10, Cf);
            if (m1 & 8) accumulate_tap<CH>(p1.wx1 * p1.wy1, u11, Cf);
            Wf += (p1.wx0 + p1.wx1) * (p1.wy0 + p1.wy1);
        }
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

// Prepared record of halfedge h: for its three fetches the packed word
// base | k << 40 | flip << 45 and the edge id, then Next(h) and Prev(h).
struct alignas(16) PrepRec {
    uint64_t w[3];
    int32_t e[3];
    int32_t next, prev, pad;
};
static_assert(sizeof(PrepRec) == HTEX_PREP_BYTES, "record size");

// Whether the three fetches of record r stay inside a pool of `total`
// texels laid out with (`mips`) or without mip levels: each fetch's edge,
// all of its levels, must end at or before `total`.  A record prepared for
// another pool layout then cannot make a kernel read outside the pool; its
// query is answered as invalid instead.
__device__ __forceinline__ bool record_in_pool(const PrepRec &r, int64_t total, bool mips)
{
    bool ok = true;
#pragma unroll
    for (int s = 0; s < 3; ++s) {
        const uint32_t k = (uint32_t)(r.w[s] >> 40) & 31u;
        const uint32_t kk = k > 15u ? 15u : k;
        // texels of an edge: (4^(k+1) - 1) / 3 with mips (bit pattern
        // 0101...01 of k + 1 pairs), 4^k without
        const uint32_t ext = mips ? (0x55555555u >> (30u - 2u * kk)) : (1u << (2u * kk));
        const int64_t end = (int64_t)(r.w[s] & 0xffffffffffull) + (int64_t)ext;
        ok = ok & (k <= 15u) & (end <= total);
    }
    return ok;
}

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

inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

}  // namespace
}  // namespace htex
