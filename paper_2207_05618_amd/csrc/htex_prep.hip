// htex_prep.hip -- per-pool and per-mesh preparation kernels: box-filtered
// mip chains, BF16 / FP8-E4M3 quantization, halfedge validation.  Pools hold
// 4 channels per texel (RGBA) or 1 (a scalar map such as displacement).
#include <hip/hip_runtime.h>

#include "htex_internal.h"

namespace htex {
namespace {

// Level l of every edge with k >= l, from level l-1: the mean of each 2x2
// block.  One workgroup per edge (grid-stride), threads over the level's
// texels.  T is float4 (RGBA texels) or float (one channel).
__device__ __forceinline__ float4 box4(const float4 &p, const float4 &q, const float4 &r,
                                       const float4 &s)
{
    return make_float4(0.25f * ((p.x + q.x) + (r.x + s.x)), 0.25f * ((p.y + q.y) + (r.y + s.y)),
                       0.25f * ((p.z + q.z) + (r.z + s.z)), 0.25f * ((p.w + q.w) + (r.w + s.w)));
}

__device__ __forceinline__ float box4(float p, float q, float r, float s)
{
    return 0.25f * ((p + q) + (r + s));
}

template <typename T>
__global__ void k_mip_level(T *tex, const uint8_t *log2res, const int64_t *base, int32_t E, int l)
{
    for (int64_t e = blockIdx.x; e < E; e += gridDim.x) {
        const int k = log2res[e];
        if (k < l) continue;
        const int m = k - l;
        const int32_t n = 1 << m;
        const int64_t src = base[e] + level_offset(k, l - 1);
        const int64_t dst = base[e] + level_offset(k, l);
        for (int32_t t = threadIdx.x; t < n * n; t += blockDim.x) {
            const int32_t i = t & (n - 1), j = t >> m;
            const int64_t r0 = src + (int64_t)(2 * j) * (2 * n) + 2 * i;
            const int64_t r1 = r0 + 2 * n;
            tex[dst + (int64_t)j * n + i] = box4(tex[r0], tex[r0 + 1], tex[r1], tex[r1 + 1]);
        }
    }
}

// Transpose of one mip step for gradients: every texel of level l hands a
// quarter of its gradient to each of the four level-(l-1) texels it is the
// mean of (one lane per level-l texel, so no two lanes write one texel),
// and is cleared afterwards when `clear` is set.
__device__ __forceinline__ void quarter_add(float4 &d, const float4 &g)
{
    d.x += g.x;
    d.y += g.y;
    d.z += g.z;
    d.w += g.w;
}

__device__ __forceinline__ void quarter_add(float &d, float g) { d += g; }

__device__ __forceinline__ float4 quarter(const float4 &g)
{
    return make_float4(0.25f * g.x, 0.25f * g.y, 0.25f * g.z, 0.25f * g.w);
}

__device__ __forceinline__ float quarter(float g) { return 0.25f * g; }

template <typename T>
__global__ void k_mip_backward_level(T *d, const uint8_t *log2res, const int64_t *base, int32_t E,
                                     int l, int clear)
{
    for (int64_t e = blockIdx.x; e < E; e += gridDim.x) {
        const int k = log2res[e];
        if (k < l) continue;
        const int m = k - l;
        const int32_t n = 1 << m;
        const int64_t src = base[e] + level_offset(k, l);
        const int64_t dst = base[e] + level_offset(k, l - 1);
        for (int32_t t = threadIdx.x; t < n * n; t += blockDim.x) {
            const int32_t i = t & (n - 1), j = t >> m;
            const T g = quarter(d[src + t]);
            const int64_t r0 = dst + (int64_t)(2 * j) * (2 * n) + 2 * i;
            const int64_t r1 = r0 + 2 * n;
            quarter_add(d[r0], g);
            quarter_add(d[r0 + 1], g);
            quarter_add(d[r1], g);
            quarter_add(d[r1 + 1], g);
            if (clear) d[src + t] = T{};
        }
    }
}

// float32 -> bfloat16, round to nearest even; NaN stays a quiet NaN.
__device__ __forceinline__ uint16_t to_bf16(float x)
{
    uint32_t b = __float_as_uint(x);
    if ((b & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((b >> 16) | 0x40u);
    b += 0x7fffu + ((b >> 16) & 1u);
    return (uint16_t)(b >> 16);
}

// With `vec` (both arrays 16-byte aligned), eight values per thread and
// step: two 16-byte loads, one 16-byte store; the last count % 8 values,
// or all of them without `vec`, one at a time.
__global__ void k_quant_bf16(const float *src, uint16_t *dst, int64_t count, bool vec)
{
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const int64_t n8 = vec ? count >> 3 : 0;
    const float4 *s4 = reinterpret_cast<const float4 *>(src);
    uint4 *d8 = reinterpret_cast<uint4 *>(dst);
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n8; i += stride) {
        const float4 a = s4[2 * i];
        const float4 b = s4[2 * i + 1];
        uint4 o;
        o.x = (uint32_t)to_bf16(a.x) | (uint32_t)to_bf16(a.y) << 16;
        o.y = (uint32_t)to_bf16(a.z) | (uint32_t)to_bf16(a.w) << 16;
        o.z = (uint32_t)to_bf16(b.x) | (uint32_t)to_bf16(b.y) << 16;
        o.w = (uint32_t)to_bf16(b.z) | (uint32_t)to_bf16(b.w) << 16;
        d8[i] = o;
    }
    for (int64_t i = (n8 << 3) + (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count;
         i += stride)
        dst[i] = to_bf16(src[i]);
}

// float32 -> OCP E4M3 (bias 7, no infinities, max 448), round to nearest
// even, saturating.  Magnitudes below 2^-6 are subnormal: code = nearest
// integer to |x| 2^9 (an exact scaling; 8 rolls over into the smallest
// normal).  Otherwise the 23-bit float mantissa is rounded to 3 bits.
__device__ __forceinline__ uint8_t to_e4m3(float x)
{
    const uint32_t b = __float_as_uint(x);
    const uint32_t sgn = (b >> 24) & 0x80u;
    const float ax = fabsf(x);
    if (ax != ax) return 0x7fu;
    uint32_t code;
    if (ax >= 448.0f) {
        code = 0x7eu;
    } else if (ax < 0x1p-6f) {
        code = (uint32_t)rintf(ax * 512.0f);
    } else {
        int32_t E = (int32_t)((b >> 23) & 0xffu) - 127;
        const uint32_t man = b & 0x7fffffu;
        uint32_t keep = man >> 20;
        const uint32_t rem = man & 0xfffffu;
        if (rem > 0x80000u || (rem == 0x80000u && (keep & 1u))) ++keep;
        if (keep == 8u) { keep = 0; ++E; }
        code = ((uint32_t)(E + 7) << 3) | keep;
        if (code > 0x7eu) code = 0x7eu;
    }
    return (uint8_t)(sgn | code);
}

// One workgroup per edge: max |T| over all of the edge's texel channels,
// scale = max / 448 (float32), then the codes of T / scale.
__global__ void __launch_bounds__(256) k_quant_fp8(const float *src, uint8_t *dst, float *scale,
                                                   const uint8_t *log2res, const int64_t *base,
                                                   int32_t E, int has_mips, int channels)
{
    __shared__ float red[256];
    for (int64_t e = blockIdx.x; e < E; e += gridDim.x) {
        const int k = log2res[e];
        const int64_t cnt =
            channels * (has_mips ? ((int64_t(4) << (2 * k)) - 1) / 3 : (int64_t(1) << (2 * k)));
        const float *t = src + channels * base[e];
        float mx = 0.0f;
        if (channels == 4) {
            // RGBA texels: one 16-byte load per texel
            const float4 *t4 = reinterpret_cast<const float4 *>(t);
            for (int64_t i = threadIdx.x; i < (cnt >> 2); i += blockDim.x) {
                const float4 x = t4[i];
                mx = fmaxf(mx, fmaxf(fmaxf(fabsf(x.x), fabsf(x.y)), fmaxf(fabsf(x.z), fabsf(x.w))));
            }
        } else {
            for (int64_t i = threadIdx.x; i < cnt; i += blockDim.x) mx = fmaxf(mx, fabsf(t[i]));
        }
        red[threadIdx.x] = mx;
        __syncthreads();
        for (int w = 128; w > 0; w >>= 1) {
            if ((int)threadIdx.x < w) red[threadIdx.x] = fmaxf(red[threadIdx.x], red[threadIdx.x + w]);
            __syncthreads();
        }
        const float s = red[0] / 448.0f;
        __syncthreads();
        if (threadIdx.x == 0) scale[e] = s;
        uint8_t *o = dst + channels * base[e];
        if (channels == 4) {
            // last texels first: the lines the max pass read most recently
            // are the likeliest still in the L2
            const float4 *t4 = reinterpret_cast<const float4 *>(t);
            uint32_t *o4 = reinterpret_cast<uint32_t *>(o);
            const int64_t n4 = cnt >> 2;
            for (int64_t i = n4 - 1 - threadIdx.x; i >= 0; i -= blockDim.x) {
                uint32_t c = 0;
                if (s != 0.0f) {
                    const float4 x = t4[i];
                    c = (uint32_t)to_e4m3(x.x / s) | (uint32_t)to_e4m3(x.y / s) << 8 |
                        (uint32_t)to_e4m3(x.z / s) << 16 | (uint32_t)to_e4m3(x.w / s) << 24;
                }
                o4[i] = c;
            }
        } else {
            for (int64_t i = threadIdx.x; i < cnt; i += blockDim.x)
                o[i] = (s == 0.0f) ? (uint8_t)0 : to_e4m3(t[i] / s);
        }
    }
}

// Halfedge invariants, pass 1: ranges, Next/Prev inverse, Twin involution,
// shared edge, face size >= 3; counts the uses of every edge id.
__global__ void k_validate1(htex_mesh m, int32_t *use, int32_t *bad)
{
    const int32_t h = blockIdx.x * blockDim.x + threadIdx.x;
    if (h >= m.H) return;
    const int32_t t = m.twin[h], n = m.next[h], p = m.prev[h], e = m.edge[h];
    bool ok = t >= -1 && t < m.H && t != h && n >= 0 && n < m.H && p >= 0 && p < m.H &&
              e >= 0 && e < m.E;
    if (ok) ok = m.prev[n] == h && m.next[p] == h;
    if (ok && t >= 0) ok = m.twin[t] == h && m.edge[t] == e;
    if (ok) ok = n != h && m.next[n] != h;
    if (!ok) {
        atomicMin(bad, h);
        return;
    }
    atomicAdd(use + e, 1);
}

// Pass 2: each edge id used by exactly one pair or one boundary halfedge.
__global__ void k_validate2(htex_mesh m, const int32_t *use, int32_t *bad, int32_t *unused)
{
    const int32_t h = blockIdx.x * blockDim.x + threadIdx.x;
    if (h < m.H) {
        const int32_t e = m.edge[h];
        // halfedges with an out-of-range edge id were flagged by pass 1
        if (e >= 0 && e < m.E && use[e] != (m.twin[h] >= 0 ? 2 : 1)) atomicMin(bad, h);
    }
    if (h < m.E && use[h] == 0) atomicAdd(unused, 1);
}

}  // namespace

hipError_t launch_build_mips(float *texels, const uint8_t *log2res, const int64_t *base,
                             int32_t E, int max_k, int channels, hipStream_t s)
{
    if (E == 0) return hipSuccess;
    for (int l = 1; l <= max_k; ++l) {
        const int threads = (max_k - l) >= 4 ? 256 : 64;
        const uint32_t grid = (uint32_t)(E < (1 << 20) ? E : (1 << 20));
        if (channels == 4)
            hipLaunchKernelGGL(k_mip_level<float4>, dim3(grid), dim3(threads), 0, s,
                               reinterpret_cast<float4 *>(texels), log2res, base, E, l);
        else
            hipLaunchKernelGGL(k_mip_level<float>, dim3(grid), dim3(threads), 0, s, texels,
                               log2res, base, E, l);
        hipError_t err = hipGetLastError();
        if (err != hipSuccess) return err;
    }
    return hipSuccess;
}

hipError_t launch_mip_backward(float *dtex, const uint8_t *log2res, const int64_t *base, int32_t E,
                               int max_k, int channels, int clear, hipStream_t s)
{
    if (E == 0) return hipSuccess;
    for (int l = max_k; l >= 1; --l) {
        const int threads = (max_k - l) >= 4 ? 256 : 64;
        const uint32_t grid = (uint32_t)(E < (1 << 20) ? E : (1 << 20));
        if (channels == 4)
            hipLaunchKernelGGL(k_mip_backward_level<float4>, dim3(grid), dim3(threads), 0, s,
                               reinterpret_cast<float4 *>(dtex), log2res, base, E, l, clear);
        else
            hipLaunchKernelGGL(k_mip_backward_level<float>, dim3(grid), dim3(threads), 0, s, dtex,
                               log2res, base, E, l, clear);
        hipError_t err = hipGetLastError();
        if (err != hipSuccess) return err;
    }
    return hipSuccess;
}

hipError_t launch_quantize_bf16(const float *src, uint16_t *dst, int64_t count, hipStream_t s)
{
    if (count == 0) return hipSuccess;
    const int64_t want = (count + 255) / 256;
    const uint32_t grid = (uint32_t)(want < 65536 ? want : 65536);
    const bool vec = reinterpret_cast<uintptr_t>(src) % 16 == 0 &&
                     reinterpret_cast<uintptr_t>(dst) % 16 == 0;
    hipLaunchKernelGGL(k_quant_bf16, dim3(grid), dim3(256), 0, s, src, dst, count, vec);
    return hipGetLastError();
}

hipError_t launch_quantize_fp8(const float *src, uint8_t *dst, float *scale, const uint8_t *log2res,
                               const int64_t *base, int32_t E, int has_mips, int channels,
                               int64_t total_texels, hipStream_t s)
{
    hipError_t err = hipMemsetAsync(dst, 0, (size_t)total_texels * channels, s);
    if (err != hipSuccess || E == 0) return err;
    const uint32_t grid = (uint32_t)(E < (1 << 20) ? E : (1 << 20));
    hipLaunchKernelGGL(k_quant_fp8, dim3(grid), dim3(256), 0, s, src, dst, scale, log2res, base, E,
                       has_mips, channels);
    return hipGetLastError();
}

hipError_t launch_validate(const htex_mesh &m, int32_t *ws_use, int32_t *ws_bad, hipStream_t s)
{
    // ws_bad[0] = smallest bad halfedge (init INT32_MAX), ws_bad[1] = unused edge ids
    const int32_t n = m.H > m.E ? m.H : m.E;
    if (n == 0) return hipSuccess;
    const uint32_t grid = (uint32_t)((n + 255) / 256);
    hipLaunchKernelGGL(k_validate1, dim3((uint32_t)((m.H + 255) / 256 > 0 ? (m.H + 255) / 256 : 1)),
                       dim3(256), 0, s, m, ws_use, ws_bad);
    hipError_t err = hipGetLastError();
    if (err != hipSuccess) return err;
    hipLaunchKernelGGL(k_validate2, dim3(grid), dim3(256), 0, s, m, ws_use, ws_bad, ws_bad + 1);
    return hipGetLastError();
}

}  // namespace htex
