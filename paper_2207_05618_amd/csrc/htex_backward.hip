// htex_backward.hip -- the transpose of Htex sampling with respect to the
// texels (the output of Alg. 3 is linear in them): for every in-bounds tap
// of every query, the tap's normalized weight times dL/dout is added to the
// texel's gradient.  Float atomics to the gradient pool, or for sorted
// batches per-level gradient tiles cached in LDS and flushed once.
#include <hip/hip_runtime.h>

#include "htex_filter.h"

namespace htex {
namespace {

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

}  // namespace

hipError_t launch_backward(const SampleArgs &a, int filter, uint32_t flags, hipStream_t s)
{
    if (a.Q == 0) return hipSuccess;
    const bool tri = filter == HTEX_TRILINEAR;
    if (a.channels == 1)
        return tri ? launch_bwd<1, true>(a, flags, s) : launch_bwd<1, false>(a, flags, s);
    return tri ? launch_bwd<4, true>(a, flags, s) : launch_bwd<4, false>(a, flags, s);
}

}  // namespace htex
