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
//
// Dense segments.  LDS float atomics cost about as much as the rest of the
// kernel, while LDS integer atomics are cheap.  The halfedges of a block's
// first and last queries are its segments when their textures have at most
// 32 x 32 texels and each holds an eighth of the block (many samples per
// texel, as when fitting a texture; in a sorted batch a block straddles at
// most two such halfedges).  A segment bins its queries by the level and
// tap cell (i0, j0) of their own fetch's finer level, counting with integer
// atomics, and each thread then walks a run of binned queries: consecutive
// queries of one cell share their four target texels, so their
// contributions are summed in registers and added to the tile once per run
// (the coarser level of a trilinear fetch keeps a run of its own; the walk
// reads each query's inputs two queries ahead).  Next and Prev textures of
// the own size ride on these runs and collect their taps in two small
// strips, one line of texels along the shared edge per level, so a segment
// needs only its own texture in the arena.  Queries on other halfedges, or
// whose taps fall outside the cell range, take the per-query path.
constexpr int kTiles = 32;
constexpr int kArenaFloats = 16384;   // 64 KB
constexpr int kBwdPerThread = 16;
constexpr int kBwdChunk = kBlock * kBwdPerThread;
constexpr int kDenseMaxLog2 = 5;
// tap cells: bases -1 .. n - 1 per axis on every level of a texture of up to
// 2^kDenseMaxLog2 texels a side, level after level
__host__ __device__ constexpr int dense_cells_before(int k, int l)
{
    int c = 0;
    for (int m = 0; m < l; ++m) c += ((1 << (k - m)) + 1) * ((1 << (k - m)) + 1);
    return c;
}
constexpr int kDenseCells = dense_cells_before(kDenseMaxLog2, kDenseMaxLog2 + 1);
// a neighbour strip: one line of texels per level, n = 2^(k - l) on level l
constexpr int kStripTexels = (2 << kDenseMaxLog2) - 1;
// Batches whose textures have at most 32 x 32 texels: the arena holds one
// segment's RGBA texture (16 KB, 21.8 KB with mips) and the strips, a block
// that straddles two halfedges adds its first segment's tiles to the pool
// before the second, and four blocks fit per compute unit (config 4: 286
// and 586 us bilinear / trilinear, against 295 and 604 us with room for a
// second texture and three blocks, and 706 us trilinear with two blocks and
// the 64 KB arena).  A block with three or more large runs of halfedges
// then adds its middle ones' taps to the pool directly.
template <bool TRI>
constexpr int arena_small()
{
    return 4 * (TRI ? ((4 << (2 * kDenseMaxLog2)) - 1) / 3 : 1 << (2 * kDenseMaxLog2)) +
           2 * 4 * kStripTexels;
}
// texels of levels 0 .. l - 1 (l <= k + 1): 2^(k+1) - 2^(k+1-l)
__host__ __device__ constexpr int strip_before(int k, int l) { return (2 << k) - ((2 << k) >> l); }
static_assert(strip_before(0, 1) == 1 && strip_before(5, 6) == kStripTexels &&
                  strip_before(5, 1) == 32 && strip_before(3, 2) == 12,
              "strip offsets");
constexpr int kCellsPerThread = (kDenseCells + kBlock - 1) / kBlock;

// Cell key of a level plan on level l of a texture of log2 size k, or -1
// when its tap bases fall outside -1 .. n - 1.
__device__ __forceinline__ int32_t dense_cell(int k, int l, const LevelPlan &p)
{
    const int32_t n = 1 << (k - l);
    if (p.i0 < -1 || p.i0 > n - 1 || p.j0 < -1 || p.j0 > n - 1) return -1;
    return dense_cells_before(k, l) + (p.j0 + 1) * (n + 1) + (p.i0 + 1);
}
static_assert(kBwdChunk <= 65536, "binned query indices are 16-bit");
static_assert(kDenseCells < 0x7fff, "a query's cell and segment share 16 bits");

constexpr uint64_t kFree = ~0ull;
constexpr uint32_t kPending = 0xfffffffeu, kNoRoom = 0xfffffffdu;

struct TileTable {
    float *arena;
    uint64_t *entry;   // key << 32 | offset (kPending, kNoRoom) or kFree
    int32_t *used;
    int32_t cap;       // arena floats
};

// Arena offset (floats) of the tile `key` of `need` floats: found, or
// claimed for this block; -1 when it is pending, does not fit, or the
// table is full.
__device__ __forceinline__ int32_t find_tile(const TileTable &T, int32_t key, int64_t need)
{
    const uint32_t h0 = ((uint32_t)key * 2654435761u) >> 27;   // 5 bits
    for (int pr = 0; pr < kTiles; ++pr) {
        const int t = (int)((h0 + pr) & (kTiles - 1));
        uint64_t en = __atomic_load_n(&T.entry[t], __ATOMIC_RELAXED);
        if (en == kFree) {
            const uint64_t mine = ((uint64_t)(uint32_t)key << 32) | kPending;
            en = atomicCAS(&T.entry[t], kFree, mine);
            if (en == kFree) {   // claimed: reserve the level's texels
                const int32_t o = need <= T.cap ? atomicAdd(T.used, (int32_t)need) : T.cap;
                const bool fits = o + need <= T.cap;
                atomicExch(&T.entry[t], ((uint64_t)(uint32_t)key << 32) |
                                            (fits ? (uint32_t)o : kNoRoom));
                return fits ? o : -1;
            }
        }
        if ((uint32_t)(en >> 32) == (uint32_t)key) {
            const uint32_t lo32 = (uint32_t)(en & 0xffffffffu);
            return lo32 < (uint32_t)T.cap ? (int32_t)lo32 : -1;
        }
    }
    return -1;
}

// Adds w * g to texel `off` of a level: into its tile when it has one,
// else into the gradient pool.
template <int CH>
__device__ __forceinline__ void add_tap(float *arena, int32_t base_f, uint32_t rel, float *pool_c,
                                        float4 x)
{
    if (base_f >= 0) {
        float *c = &arena[base_f + CH * (int32_t)rel];
        atomicAdd(c + 0, x.x);
        if constexpr (CH == 4) {
            atomicAdd(c + 1, x.y);
            atomicAdd(c + 2, x.z);
            atomicAdd(c + 3, x.w);
        }
    } else {
        unsafeAtomicAdd(pool_c + 0, x.x);
        if constexpr (CH == 4) {
            unsafeAtomicAdd(pool_c + 1, x.y);
            unsafeAtomicAdd(pool_c + 2, x.z);
            unsafeAtomicAdd(pool_c + 3, x.w);
        }
    }
}

// A query's inputs, read ahead of its scatter.
struct QIn {
    float u, v, f;
    float4 g;
};

template <int CH, bool TRI>
__device__ __forceinline__ QIn load_qin(const SampleArgs &a, int64_t q)
{
    QIn x;
    x.u = a.qu[q];
    x.v = a.qv[q];
    x.f = TRI ? a.qf[q] : 0.0f;
    x.g = load_row<CH>(a.dout, q);
    return x;
}

// The navigation of one halfedge's three fetches: their edges, log2
// resolutions, reflections and texel bases.
struct Topo {
    int32_t n1, p1;
    int32_t es[3], ks[3];
    bool flips[3];
    int64_t ebs[3];
};

__device__ __forceinline__ Topo topo_of(const SampleArgs &a, int32_t h)
{
    Topo t;
    t.n1 = a.next[h];
    t.p1 = a.prev[h];
    const int32_t g[3] = {h, t.n1, t.p1};
#pragma unroll
    for (int s = 0; s < 3; ++s) {
        t.flips[s] = !(g[s] > a.twin[g[s]]);
        t.es[s] = a.edge[g[s]];
        t.ks[s] = a.log2res[t.es[s]];
        t.ebs[s] = a.base[t.es[s]];
    }
    return t;
}

// The transpose of Alg. 3 for query q: every in-bounds tap of every fetch
// and level receives (om w / W) dL/dout.  Returns false for an invalid
// query.
template <int CH, bool TRI>
__device__ __forceinline__ bool scatter_query(const SampleArgs &a, int64_t q, const TileTable &T,
                                              int32_t (&memo_key)[3][2], int32_t (&memo_base)[3][2])
{
    const int32_t h = a.qh[q];
    const float u = a.qu[q], v = a.qv[q];
    if (!((uint32_t)h < (uint32_t)a.H) || !isfinite(u) || !isfinite(v)) return false;
    const Topo tp = topo_of(a, h);
    Lod L{0, 0, 0.0f, 1.0f};
    if constexpr (TRI) L = lod_of(a.qf[q]);
    FetchSpec fs[3];
    fetch_specs(h, tp.n1, tp.p1, u, v, fs);
    const int32_t *es = tp.es, *ks = tp.ks;
    const bool *flips = tp.flips;
    // every fetch's level plans, planned once: for the normalization W
    // first, then for the scatter
    float W = 0.0f;
    int nl[3], lvs[3][2];
    LevelPlan pl[3][2];
#pragma unroll
    for (int s = 0; s < 3; ++s) {
        float om[2];
        nl[s] = fetch_levels(L, ks[s], lvs[s], om);
#pragma unroll
        for (int sl = 0; sl < (TRI ? 2 : 1); ++sl) {
            pl[s][sl] = plan_level(ks[s], sl < nl[s] ? lvs[s][sl] : lvs[s][0], om[sl], fs[s],
                                   flips[s]);
            if (sl < nl[s]) W += (pl[s][sl].wx0 + pl[s][sl].wx1) * (pl[s][sl].wy0 + pl[s][sl].wy1);
        }
    }
    const float4 g4 = load_row<CH>(a.dout, q);
    const float rW = 1.0f / W;
#pragma unroll
    for (int s = 0; s < 3; ++s) {
        const int nlev = nl[s];
        const int *lv = lvs[s];
        const int64_t eb = tp.ebs[s];
#pragma unroll
        for (int sl = 0; sl < (TRI ? 2 : 1); ++sl) {
            if (sl >= nlev) break;
            const LevelPlan &p = pl[s][sl];
            if (!p.act) continue;
            const int m = ks[s] - lv[sl];
            const uint32_t lo = level_offset32(ks[s], lv[sl]);
            // the tile of this (edge, level): remembered, found, or claimed
            const int32_t key = es[s] * 16 + lv[sl];
            // floats of this level's tile (computed in 64 bits: a level of
            // 2^15 x 2^15 RGBA texels needs 2^32 floats; it never fits)
            const int64_t need = (int64_t)CH << (2 * m);
            int32_t base_f = memo_key[s][sl] == key ? memo_base[s][sl] : find_tile(T, key, need);
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
                add_tap<CH>(T.arena, base_f, off[t] - lo, a.dtex + CH * (eb + off[t]),
                            make_float4(wt * g4.x, wt * g4.y, wt * g4.z, wt * g4.w));
            }
        }
    }
    return true;
}

// One axis of a neighbour fetch as a map of texel indices: x' = sg x + an n
// + ac on a level of n texels a side, from the own fetch's index x on the
// axis that reads the same query coordinate.  The neighbour axis reads
// (neg ? -c : c) under its reflection `flip`, the own axis c under `flip0`
// (Alg. 2: x -> 1 - x per axis); the map sends texel centres to texel
// centres and keeps distances.
struct AxisMap {
    int32_t sg, an, ac;
};

__device__ __forceinline__ AxisMap mirror_axis(bool neg, bool flip, bool flip0)
{
    const int32_t rho0 = flip0 ? 1 : 0, rs = flip ? 1 : 0;
    AxisMap m;
    m.sg = ((neg != flip) != flip0) ? -1 : 1;
    m.an = m.sg == 1 ? rs - rho0 : rho0 + rs;
    m.ac = m.sg == 1 ? 0 : -1;
    return m;
}

// (the small arena's launches hold four blocks per compute unit, 128 VGPRs)
template <int CH, bool TRI, int CAP>
__global__ void __launch_bounds__(kBlock, (CAP < kArenaFloats ? 4 : 1)) k_backward_lds(SampleArgs a)
{
    __shared__ float arena[CAP];
    __shared__ uint64_t entry[kTiles];
    __shared__ int32_t used;
    // dense segments: per-cell counts, then offsets; the binned query order;
    // the tile of each level of the segment's own texture
    __shared__ int32_t cell_ofs[kDenseCells];
    __shared__ int32_t part[kBlock];
    __shared__ uint16_t order[kBwdChunk];
    __shared__ int32_t own_base[kDenseMaxLog2 + 1];
    __shared__ int32_t seg_h[2], nbinned;
    for (int i = threadIdx.x; i < CAP; i += kBlock) arena[i] = 0.0f;
    if (threadIdx.x < kTiles) entry[threadIdx.x] = kFree;
    const int64_t q0 = (int64_t)blockIdx.x * kBwdChunk;
    if (threadIdx.x == 0) {
        // dense segments: the halfedges of the block's first and last
        // queries, each binned by tap cell when its texture is small and
        // it holds an eighth of the block at least (in a sorted batch: the
        // query an eighth in from that end has it too)
        const int64_t n = (q0 + kBwdChunk < a.Q ? q0 + kBwdChunk : a.Q) - q0, ql = q0 + n - 1;
        const int32_t hf = a.qh[q0], hl = a.qh[ql];
        auto small = [&](int32_t h) {
            return (uint32_t)h < (uint32_t)a.H && a.log2res[a.edge[h]] <= kDenseMaxLog2;
        };
        seg_h[0] = (small(hf) && a.qh[q0 + n / 8] == hf) ? hf : -1;
        seg_h[1] = (hl != hf && small(hl) && a.qh[ql - n / 8] == hl) ? hl : -1;
        // a dense segment's Next and Prev strips (below) open the arena
        used = (seg_h[0] >= 0 || seg_h[1] >= 0) ? 2 * CH * kStripTexels : 0;
    }
    __syncthreads();
    const TileTable T{arena, entry, &used, CAP};
    // the last tile each of a lane's six (fetch, level) slots resolved: a
    // lane's consecutive queries are usually on the same halfedge
    int32_t memo_key[3][2], memo_base[3][2];
#pragma unroll
    for (int s = 0; s < 3; ++s)
        for (int sl = 0; sl < 2; ++sl) memo_key[s][sl] = -1;
    // every tile to the pool, one float atomic per non-zero texel channel
    auto flush_tiles = [&]() {
        for (int t = 0; t < kTiles; ++t) {
            const uint64_t en = entry[t];
            if (en == kFree || (uint32_t)(en & 0xffffffffu) >= (uint32_t)CAP) continue;
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
    };
    // a second segment's texture fits beside the first's in this arena
    // (a texture of 2^kDenseMaxLog2 texels a side: 4^k texels, (4^(k+1) - 1)
    // / 3 with its mips)
    constexpr int kChain = TRI ? ((4 << (2 * kDenseMaxLog2)) - 1) / 3 : 1 << (2 * kDenseMaxLog2);
    constexpr bool kTwoChains = CAP >= 2 * CH * kStripTexels + 2 * CH * kChain;
    // the segments' halfedges, edges, log2 sizes and reflections
    // (block-uniform: read with scalar loads)
    int32_t sh[2], se[2], sk[2];
    bool sflip[2];
#pragma unroll
    for (int sg = 0; sg < 2; ++sg) {
        sh[sg] = __builtin_amdgcn_readfirstlane(seg_h[sg]);
        se[sg] = sh[sg] >= 0 ? a.edge[sh[sg]] : 0;
        sk[sg] = sh[sg] >= 0 ? a.log2res[se[sg]] : 0;
        sflip[sg] = sh[sg] >= 0 && !(sh[sg] > a.twin[sh[sg]]);
    }
    // 1. the tap cell of each query's own fetch on its finer level, for
    // the segment that holds the query: 16 bits per query, cell | segment
    // << 15, or 0xffff (computed once: recomputed per segment, the query
    // loads would be hoisted and held through both walks)
    uint32_t cells[kBwdPerThread / 2];
    uint32_t binned = 0;   // bit r: query r of this thread is in a segment
#pragma unroll
    for (int r = 0; r < kBwdPerThread; ++r) {
        const int64_t q = q0 + (int64_t)r * kBlock + threadIdx.x;
        uint32_t c16 = 0xffffu;
        if (q < a.Q && (sh[0] >= 0 || sh[1] >= 0)) {
            const int32_t h = a.qh[q];
            const float u = a.qu[q], v = a.qv[q];
            const int sg = (sh[0] >= 0 && h == sh[0]) ? 0 : (sh[1] >= 0 && h == sh[1]) ? 1 : -1;
            if (sg >= 0 && isfinite(u) && isfinite(v)) {
                const int k = sg ? sk[1] : sk[0];
                Lod L{0, 0, 0.0f, 1.0f};
                if constexpr (TRI) L = lod_of(a.qf[q]);
                int lv[2];
                float om[2];
                fetch_levels(L, k, lv, om);
                const FetchSpec f0 = {h, u, v, false, false};
                const int32_t c =
                    dense_cell(k, lv[0], plan_level(k, lv[0], om[0], f0, sg ? sflip[1] : sflip[0]));
                if (c >= 0) {
                    c16 = (uint32_t)c | (uint32_t)sg << 15;
                    binned |= 1u << r;
                }
            }
        }
        if (r & 1)
            cells[r >> 1] |= c16 << 16;
        else
            cells[r >> 1] = c16;
    }
    // the cell of query r in segment sg, or -1
    auto cell_of = [&](int r, int sg) -> int32_t {
        const uint32_t c16 = (cells[r >> 1] >> (16 * (r & 1))) & 0xffffu;
        return (c16 != 0xffffu && (int)(c16 >> 15) == sg) ? (int32_t)(c16 & 0x7fffu) : -1;
    };
    // one dense segment (called for each: a loop over the two would keep
    // values live across its iterations)
    auto segment = [&](const int sg) {
        const int32_t hb = sg ? sh[1] : sh[0];
        if (!kTwoChains && sg == 1 && sh[0] >= 0) {
            // the first segment's tiles to the pool, the arena cleared
            flush_tiles();
            __syncthreads();
            if (threadIdx.x < kTiles) entry[threadIdx.x] = kFree;
            if (threadIdx.x == 0) used = 2 * CH * kStripTexels;
            for (int i = threadIdx.x; i < CAP; i += kBlock) arena[i] = 0.0f;
#pragma unroll
            for (int f = 0; f < 3; ++f)
                for (int sl = 0; sl < 2; ++sl) memo_key[f][sl] = -1;
            __syncthreads();
        }
        const int32_t e0 = sg ? se[1] : se[0];
        const int k0 = sg ? sk[1] : sk[0];
        const bool flip0 = sg ? sflip[1] : sflip[0];
        for (int i = threadIdx.x; i < kDenseCells; i += kBlock) cell_ofs[i] = 0;
        for (int i = threadIdx.x; i < 2 * CH * kStripTexels; i += kBlock) arena[i] = 0.0f;
        if (threadIdx.x <= (TRI ? k0 : 0))
            own_base[threadIdx.x] = find_tile(T, e0 * 16 + (int)threadIdx.x,
                                              (int64_t)CH << (2 * (k0 - (int)threadIdx.x)));
        __syncthreads();
#pragma unroll
        for (int r = 0; r < kBwdPerThread; ++r) {
            const int32_t c = cell_of(r, sg);
            if (c >= 0) atomicAdd(&cell_ofs[c], 1);
        }
        __syncthreads();
        // 2. exclusive offsets: per-thread sums, one wavefront scans them
        int32_t sum = 0;
#pragma unroll
        for (int j = 0; j < kCellsPerThread; ++j) {
            const int c = threadIdx.x * kCellsPerThread + j;
            if (c < kDenseCells) sum += cell_ofs[c];
        }
        part[threadIdx.x] = sum;
        __syncthreads();
        if (threadIdx.x < 64) {
            const int l = threadIdx.x;
            const int32_t v0 = part[4 * l], v1 = part[4 * l + 1], v2 = part[4 * l + 2],
                          v3 = part[4 * l + 3];
            const int32_t tot = v0 + v1 + v2 + v3;
            int32_t inc = tot;
            for (int d = 1; d < 64; d <<= 1) {
                const int32_t y = __shfl_up(inc, d);
                if (l >= d) inc += y;
            }
            const int32_t ex = inc - tot;
            part[4 * l] = ex;
            part[4 * l + 1] = ex + v0;
            part[4 * l + 2] = ex + v0 + v1;
            part[4 * l + 3] = ex + v0 + v1 + v2;
            if (l == 63) nbinned = inc;
        }
        __syncthreads();
        int32_t run = part[threadIdx.x];
#pragma unroll
        for (int j = 0; j < kCellsPerThread; ++j) {
            const int c = threadIdx.x * kCellsPerThread + j;
            if (c < kDenseCells) {
                const int32_t cnt = cell_ofs[c];
                cell_ofs[c] = run;
                run += cnt;
            }
        }
        __syncthreads();
        // 3. the binned order
#pragma unroll
        for (int r = 0; r < kBwdPerThread; ++r) {
            const int32_t c = cell_of(r, sg);
            if (c >= 0) order[atomicAdd(&cell_ofs[c], 1)] = (uint16_t)(r * kBlock + threadIdx.x);
        }
        __syncthreads();
        // 4. runs of binned queries, kBwdPerThread consecutive entries per
        // thread.  Queries of one cell share the four taps of their own
        // fetch's finer level, so their contributions are summed in
        // registers over the run and added to the tiles when the cell
        // changes; the coarser level's cell changes less often than the
        // query does and gets a run of its own.
        //
        // The Next and Prev fetches ride on these runs where their texture
        // has the own texture's size.  Alg. 3 reads them at (v, -u) and
        // (-v, u), each under its own Alg. 2 reflection: per axis an index
        // map (AxisMap) that sends texel centres to texel centres and keeps
        // distances, on the same level (same size, same footprint).  Each
        // tap of such a fetch is then the image of a tap of the own fetch,
        // with the same bilinear weight (axis_taps forms the weights of both
        // from the same exact fraction of the coordinate), so a run's four
        // sums go to every fetch whose texture holds their images, and W
        // counts each own tap once per fetch that holds it.  A neighbour
        // texture of another size is planned and added per query.
        constexpr int NL = TRI ? 2 : 1;
        const int i0 = threadIdx.x * kBwdPerThread;
        const int i1 = i0 + kBwdPerThread < nbinned ? i0 + kBwdPerThread : nbinned;
        const Topo tb = topo_of(a, hb);
        const int rho0 = flip0 ? 1 : 0;
        const bool eq1 = tb.ks[1] == k0, eq2 = tb.ks[2] == k0;
        // Own taps (i, j) on a level of n texels a side lie in 0 .. n - 1 on
        // both axes.  Those of Next are (edge, 0 .. n - 1) and those of Prev
        // (0 .. n - 1, edge), with edge = -1, or n under the own fetch's
        // reflection: one line along each shared edge, the index along it
        // a strip index.  `image` maps a strip texel into its texture.
        auto holder = [&](int32_t i, int32_t j, int32_t n, int32_t edge) -> int {
            const bool in_i = (uint32_t)i < (uint32_t)n, in_j = (uint32_t)j < (uint32_t)n;
            return (in_i && in_j) ? 0 : (eq1 && i == edge && in_j) ? 1
                                      : (eq2 && j == edge && in_i) ? 2 : -1;
        };
        const AxisMap nx = mirror_axis(false, tb.flips[1], flip0);   // Next: x' = v
        const AxisMap ny = mirror_axis(true, tb.flips[1], flip0);    //       y' = -u
        const AxisMap px = mirror_axis(true, tb.flips[2], flip0);    // Prev: x' = -v
        const AxisMap py = mirror_axis(false, tb.flips[2], flip0);   //       y' = u
        auto image = [&](int s, int32_t i, int32_t j, int32_t n, int32_t &x, int32_t &y) -> bool {
            const AxisMap mx = s == 1 ? nx : px, my = s == 1 ? ny : py;
            x = mx.sg * j + mx.an * n + mx.ac;
            y = my.sg * i + my.an * n + my.ac;
            return (uint32_t)x < (uint32_t)n && (uint32_t)y < (uint32_t)n;
        };
        // adds x[t] to the holders of the taps of cell (ti, tj) on level l:
        // the own tile, or the Next or Prev strip at the arena's start
        auto spread = [&](int l, int32_t ti, int32_t tj, const float4 (&x)[4]) {
            const int m = k0 - l;
            const int32_t n = 1 << m, edge = flip0 ? n : -1;
            float *lev = a.dtex + CH * (tb.ebs[0] + level_offset32(k0, l));
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                const int32_t i = ti + (t & 1), j = tj + (t >> 1);
                const int s = holder(i, j, n, edge);
                if (s < 0) continue;
                if (s == 0) {
                    const uint32_t rel = ((uint32_t)j << m) + (uint32_t)i;
                    add_tap<CH>(arena, own_base[l], rel, lev + CH * rel, x[t]);
                } else {
                    float *c = &arena[CH * ((s - 1) * kStripTexels + strip_before(k0, l) +
                                            (s == 1 ? j : i))];
                    atomicAdd(c + 0, x[t].x);
                    if constexpr (CH == 4) {
                        atomicAdd(c + 1, x[t].y);
                        atomicAdd(c + 2, x[t].z);
                        atomicAdd(c + 3, x[t].w);
                    }
                }
            }
        };
        // a neighbour fetch of another size, planned per query: its part of
        // W, or (add) its taps.  (Its fields are selected, not indexed, so
        // that a call site in a rolled loop keeps them in registers.)
        auto other = [&](int s, const QIn &x, const Lod &L, bool add, float rW) -> float {
            FetchSpec fs[3];
            fetch_specs(hb, tb.n1, tb.p1, x.u, x.v, fs);
            const FetchSpec f = s == 1 ? fs[1] : fs[2];
            const int k = s == 1 ? tb.ks[1] : tb.ks[2];
            const bool flip = s == 1 ? tb.flips[1] : tb.flips[2];
            const int32_t es = s == 1 ? tb.es[1] : tb.es[2];
            const int64_t eb = s == 1 ? tb.ebs[1] : tb.ebs[2];
            int lv[2];
            float om[2];
            const int nl = fetch_levels(L, k, lv, om);
            float Wn = 0.0f;
#pragma unroll
            for (int sl = 0; sl < NL; ++sl) {
                if (sl >= nl) break;
                const LevelPlan p = plan_level(k, lv[sl], om[sl], f, flip);
                if (!add) {
                    Wn += (p.wx0 + p.wx1) * (p.wy0 + p.wy1);
                    continue;
                }
                if (!p.act) continue;
                const float w[4] = {p.wx0 * p.wy0, p.wx1 * p.wy0, p.wx0 * p.wy1, p.wx1 * p.wy1};
                const uint32_t off[4] = {p.o00, p.o01, p.o10, p.o11};
                const uint32_t lo = level_offset32(k, lv[sl]);
                const int32_t bf =
                    find_tile(T, es * 16 + lv[sl], (int64_t)CH << (2 * (k - lv[sl])));
#pragma unroll
                for (int t = 0; t < 4; ++t) {
                    if (!((p.mask >> t) & 1)) continue;
                    const float wt = w[t] * rW;
                    add_tap<CH>(arena, bf, off[t] - lo, a.dtex + CH * (eb + off[t]),
                                make_float4(wt * x.g.x, wt * x.g.y, wt * x.g.z, wt * x.g.w));
                }
            }
            return Wn;
        };
        int32_t rkey[NL];
        float cov[NL][4];
        float4 acc[NL][4];
#pragma unroll
        for (int sl = 0; sl < NL; ++sl) rkey[sl] = -1;
        // each query's inputs are read two queries ahead
        QIn nxt{}, nxt2{};
        if (i0 < i1) nxt = load_qin<CH, TRI>(a, q0 + order[i0]);
        if (i0 + 1 < i1) nxt2 = load_qin<CH, TRI>(a, q0 + order[i0 + 1]);
        // one pass past the last query flushes the open runs
#pragma nounroll
        for (int i = i0; i <= i1; ++i) {
            const bool last = i == i1;
            QIn cur{};
            if (!last) {
                cur = nxt;
                nxt = nxt2;
                if (i + 2 < i1) nxt2 = load_qin<CH, TRI>(a, q0 + order[i + 2]);
            }
            Lod L{0, 0, 0.0f, 1.0f};
            if constexpr (TRI) L = lod_of(cur.f);
            int lv[2] = {0, 0};
            float om[2] = {0.0f, 0.0f};
            const int nl = last ? 0 : fetch_levels(L, k0, lv, om);
            float w[NL][4];
            float W = 0.0f;
#pragma unroll
            for (int sl = 0; sl < NL; ++sl) {
                // the own fetch's taps on this level, weights not masked:
                // their bases lie in -1 .. n - 1 (binned on the finer level;
                // the coarser level's follow from it)
                const bool on = sl < nl;
                const int m = k0 - (on ? lv[sl] : 0);
                const AxisTaps X = axis_taps(cur.u, flip0, rho0, m);
                const AxisTaps Y = axis_taps(cur.v, flip0, rho0, m);
                const float wy0 = om[sl] * Y.w0, wy1 = om[sl] * Y.w1;
                w[sl][0] = X.w0 * wy0;
                w[sl][1] = X.w1 * wy0;
                w[sl][2] = X.w0 * wy1;
                w[sl][3] = X.w1 * wy1;
                const int32_t key = on ? (lv[sl] << 20 | (Y.i0 + 1) << 10 | (X.i0 + 1)) : -1;
                if (key != rkey[sl] && (on || last)) {
                    if (rkey[sl] >= 0)
                        spread(rkey[sl] >> 20, (rkey[sl] & 1023) - 1, ((rkey[sl] >> 10) & 1023) - 1,
                               acc[sl]);
                    rkey[sl] = key;
                    const int32_t n = 1 << m, edge = flip0 ? n : -1;
#pragma unroll
                    for (int t = 0; t < 4; ++t) {
                        acc[sl][t] = make_float4(0.f, 0.f, 0.f, 0.f);
                        cov[sl][t] = holder(X.i0 + (t & 1), Y.i0 + (t >> 1), n, edge) >= 0 ? 1.0f
                                                                                          : 0.0f;
                    }
                }
                if (on)
#pragma unroll
                    for (int t = 0; t < 4; ++t) W = fmaf(w[sl][t], cov[sl][t], W);
            }
            if (last) break;
            // (one call site per pass: inlined twice more, the rarely taken
            // plans would hold registers that cost occupancy)
#pragma nounroll
            for (int s = 1; s < 3; ++s)
                if (!(s == 1 ? eq1 : eq2)) W += other(s, cur, L, false, 0.0f);
            const float rW = 1.0f / W;
#pragma unroll
            for (int sl = 0; sl < NL; ++sl) {
                if (sl >= nl) break;
#pragma unroll
                for (int t = 0; t < 4; ++t) {
                    const float wt = w[sl][t] * rW;
                    acc[sl][t].x += wt * cur.g.x;
                    acc[sl][t].y += wt * cur.g.y;
                    acc[sl][t].z += wt * cur.g.z;
                    acc[sl][t].w += wt * cur.g.w;
                }
            }
#pragma nounroll
            for (int s = 1; s < 3; ++s)
                if (!(s == 1 ? eq1 : eq2)) other(s, cur, L, true, rW);
        }
        // the strips to the pool: strip texel idx of level l is own tap
        // (edge, idx) (Next) or (idx, edge) (Prev), edge = -1, or n under the
        // own fetch's reflection
        __syncthreads();
        const int nstrip = strip_before(k0, TRI ? k0 + 1 : 1);
        for (int e = threadIdx.x; e < 2 * nstrip; e += kBlock) {
            const int s = e < nstrip ? 1 : 2;
            if (!(s == 1 ? eq1 : eq2)) continue;
            const int r = e - (s - 1) * nstrip;
            int l = 0;
            while (strip_before(k0, l + 1) <= r) ++l;
            const int m = k0 - l;
            const int32_t n = 1 << m, idx = r - strip_before(k0, l), edge = flip0 ? n : -1;
            int32_t xs, ys;
            if (!image(s, s == 1 ? edge : idx, s == 1 ? idx : edge, n, xs, ys)) continue;
            float *dst = a.dtex + CH * (tb.ebs[s] + level_offset32(k0, l) +
                                        (((uint32_t)ys << m) + (uint32_t)xs));
            const float *src = &arena[CH * ((s - 1) * kStripTexels + r)];
#pragma unroll
            for (int c = 0; c < CH; ++c)
                if (src[c] != 0.0f) unsafeAtomicAdd(dst + c, src[c]);
        }
        // strips and cell counts free for the next segment
        __syncthreads();
    };
    if (sh[0] >= 0) segment(0);
    if (sh[1] >= 0) segment(1);
    // the queries left to the per-query path
    for (int r = 0; r < kBwdPerThread; ++r) {
        const int64_t q = q0 + (int64_t)r * kBlock + threadIdx.x;
        if (q >= a.Q) break;
        if (!((binned >> r) & 1)) scatter_query<CH, TRI>(a, q, T, memo_key, memo_base);
    }
    __syncthreads();
    flush_tiles();
}

template <int CH, bool TRI>
hipError_t launch_bwd(const SampleArgs &a, uint32_t flags, int max_log2res, hipStream_t s)
{
    if (flags & HTEX_QUERIES_SORTED) {
        // sorted batches meet few textures per block: cache their gradients in LDS
        const uint32_t G = (uint32_t)ceil_div(a.Q, kBwdChunk);
        if (max_log2res <= kDenseMaxLog2)
            hipLaunchKernelGGL((k_backward_lds<CH, TRI, arena_small<TRI>()>), dim3(G),
                               dim3(kBlock), 0, s, a);
        else
            hipLaunchKernelGGL((k_backward_lds<CH, TRI, kArenaFloats>), dim3(G), dim3(kBlock), 0,
                               s, a);
    } else {
        const uint32_t G = (uint32_t)ceil_div(a.Q, kBlock);
        hipLaunchKernelGGL((k_backward<CH, TRI>), dim3(G), dim3(kBlock), 0, s, a);
    }
    return hipGetLastError();
}

}  // namespace

hipError_t launch_backward(const SampleArgs &a, int filter, uint32_t flags, int max_log2res,
                           hipStream_t s)
{
    if (a.Q == 0) return hipSuccess;
    const bool tri = filter == HTEX_TRILINEAR;
    const int k = max_log2res;
    if (a.channels == 1)
        return tri ? launch_bwd<1, true>(a, flags, k, s) : launch_bwd<1, false>(a, flags, k, s);
    return tri ? launch_bwd<4, true>(a, flags, k, s) : launch_bwd<4, false>(a, flags, k, s);
}

}  // namespace htex
