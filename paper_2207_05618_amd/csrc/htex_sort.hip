// htex_sort.hip -- ordering a query batch by halfedge (optional step before
// sampling) and moving queries and results between the two orders.
//
// Stable LSD radix sort of (key, input index) pairs; the key of a query is h
// (or a caller's key of h, such as its edge), and queries with an invalid h
// sort last.  Digits are as wide as needed to cover the keys in the fewest
// passes of at most 8 bits (three passes for a million halfedges).  The
// passes follow the one-sweep scheme of Adinets and Merrill (2022): one read
// of the keys counts every pass's digits up front, so a pass knows where
// each digit's run begins in the output, and each pass is then a single
// launch over tiles of kTile keys.  Tile t finds how many keys of each digit
// the tiles before it hold by decoupled look-back over the counts those
// tiles publish, instead of from a separate histogram and scan.
//
// Inside a tile the keys are ranked stably: each wavefront ranks its quarter
// on its own (ballots within a round of 64 keys and the wavefront's running
// digit counts in LDS), one scan per digit across the four wavefronts places
// the quarters, and the tile is written from LDS in sorted order, so
// consecutive lanes store consecutive addresses of a digit's run.  The
// counting read can also copy the queries into 16-byte records (h, u, v,
// footprint): for a sorted batch the last pass then gathers each output
// row's record -- one 16-byte read per query instead of one per array --
// and for sampling through the permutation the records stay in input order.
#include <hip/hip_runtime.h>

#include <mutex>

#include "htex_internal.h"

namespace htex {
namespace {

constexpr int kThreads = 256;
constexpr int kPerThread = 16;
constexpr int kTile = kThreads * kPerThread;   // 4096 keys per tile
constexpr int kWaves = kThreads / 64;
constexpr int kMaxDigitBits = 8;
constexpr int kMaxBins = 1 << kMaxDigitBits;
constexpr int kDigitsPerThread = kMaxBins / kThreads;   // consecutive digits of one thread
constexpr int kMaxPasses = 4;                  // keys below 2^32
constexpr int kCountBlocks = 1024;             // blocks of the counting read (at most)
constexpr int kLookWindow = 4;                 // predecessors read at once in the look-back
static_assert(kMaxBins % kThreads == 0, "whole digits per thread");

// Published per-tile digit counts: the top two bits say what the low 32 hold.
constexpr uint64_t kAggregate = uint64_t(1) << 62;   // this tile's count alone
constexpr uint64_t kPrefix = uint64_t(2) << 62;      // this tile's and all before it
// Polls of a predecessor's count before a tile gives up waiting.  Every tile
// publishes its own count before it waits, and tile numbers are handed out
// in the order blocks start, so a wait only ever depends on blocks already
// running; the limit only keeps the kernel finite.
constexpr int kSpinLimit = 1 << 22;

// The keys of a pass: computed from h (first pass) or read back (later
// passes).  The key of a query is its halfedge h, or key_of_h[h] when a key
// map is given; a query whose h lies outside [0, H), or whose mapped key
// lies outside [0, K), takes the key K and sorts last.
struct KeySrc {
    const int32_t *h;      // first pass, else NULL
    const uint32_t *k;     // later passes
    const int32_t *map;    // key of each halfedge, or NULL for h itself
    int32_t H, K;          // halfedges; keys 0 .. K - 1 (K = H without a map)

    __device__ __forceinline__ uint32_t first(int32_t hv) const
    {
        if ((uint32_t)hv >= (uint32_t)H) return (uint32_t)K;
        if (!map) return (uint32_t)hv;
        const uint32_t m = (uint32_t)map[hv];
        return m < (uint32_t)K ? m : (uint32_t)K;
    }
    __device__ __forceinline__ uint32_t operator()(int64_t i) const
    {
        return h ? first(h[i]) : k[i];
    }
};

// Zeroes n 16-byte words (the digit counts, tile tickets and published
// counts of every pass).
__global__ void __launch_bounds__(kThreads) k_clear(uint4 *p, int64_t n)
{
    const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (i < n) p[i] = make_uint4(0u, 0u, 0u, 0u);
}

// count[pass * kMaxBins + d] += the keys whose digit of that pass is d,
// over the tiles blockIdx.x, blockIdx.x + gridDim.x, ...  With `rec`, also
// rec[i] = (h, u, v, f); with `keys`, keys[i] = the key of query i (so that
// a key map is read once, here, not again by the first pass).
__global__ void __launch_bounds__(kThreads) k_count(KeySrc ks, int64_t Q, int passes, int bits,
                                                    uint32_t *count, const float *u,
                                                    const float *v, const float *f, float4 *rec,
                                                    uint32_t *keys)
{
    __shared__ uint32_t cnt[kMaxPasses][kMaxBins];
    for (int p = 0; p < kMaxPasses; ++p)
        for (int d = threadIdx.x; d < kMaxBins; d += kThreads) cnt[p][d] = 0u;
    const uint32_t mask = (1u << bits) - 1u;
    __syncthreads();
    for (int64_t tile = blockIdx.x; tile * kTile < Q; tile += gridDim.x) {
        const int64_t t0 = tile * kTile + threadIdx.x;
        int32_t hv[kPerThread];
#pragma unroll
        for (int r = 0; r < kPerThread; ++r) {
            const int64_t i = t0 + (int64_t)r * kThreads;
            hv[r] = i < Q ? ks.h[i] : 0;
        }
        if (rec) {
#pragma unroll 4
            for (int r = 0; r < kPerThread; ++r) {
                const int64_t i = t0 + (int64_t)r * kThreads;
                if (i < Q)
                    rec[i] = make_float4(__int_as_float(hv[r]), u[i], v[i], f ? f[i] : 0.0f);
            }
        }
        uint32_t key[kPerThread];   // every key of this thread (and its map lookup) in flight at once
#pragma unroll
        for (int r = 0; r < kPerThread; ++r) key[r] = ks.first(hv[r]);
#pragma unroll
        for (int r = 0; r < kPerThread; ++r) {
            if (t0 + (int64_t)r * kThreads >= Q) break;
            if (keys) keys[t0 + (int64_t)r * kThreads] = key[r];
            for (int p = 0; p < passes; ++p) atomicAdd(&cnt[p][(key[r] >> (p * bits)) & mask], 1u);
        }
    }
    __syncthreads();
    const int nb = 1 << bits;
    for (int p = 0; p < passes; ++p)
        for (int d = threadIdx.x; d < nb; d += kThreads)
            if (cnt[p][d]) atomicAdd(&count[p * kMaxBins + d], cnt[p][d]);
}

// Exclusive scans of a and b over the block's threads (one value each).
__device__ __forceinline__ void block_scan2(int32_t &a, int32_t &b, int32_t (*wsum)[kWaves])
{
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    int32_t ia = a, ib = b;
    for (int d = 1; d < 64; d <<= 1) {
        const int32_t ya = __shfl_up(ia, d), yb = __shfl_up(ib, d);
        if (lane >= d) ia += ya, ib += yb;
    }
    if (lane == 63) wsum[0][w] = ia, wsum[1][w] = ib;
    __syncthreads();
    int32_t ba = 0, bb = 0;
    for (int v = 0; v < w; ++v) ba += wsum[0][v], bb += wsum[1][v];
    a = ba + ia - a;
    b = bb + ib - b;
}

struct PassArgs {
    KeySrc ks;
    const int32_t *idx_in;    // input index of each key; NULL: the identity
    uint32_t *kout;           // sorted keys; NULL on the last pass
    int32_t *iout;            // their input indices (perm on the last pass)
    const float4 *rec;        // last pass of a sorted batch: the query records
    int32_t *ho;
    float *uo, *vo, *fo;      // ... gathered into the sorted arrays
    int64_t Q;
    int shift, bits;
    const uint32_t *count;    // this pass's digit counts over the batch
    uint64_t *status;         // this pass's published counts [tile][kMaxBins]
    uint32_t *ticket;         // this pass's tile counter
};

// One pass: a block takes the next tile, ranks it, publishes its digit
// counts, looks back for the counts of the tiles before it and writes the
// tile to its places.
__global__ void __launch_bounds__(kThreads) k_pass(PassArgs a)
{
    // per-wave digit counts, then each wavefront's first slot for the digit
    __shared__ int32_t wcnt[kWaves][kMaxBins];
    __shared__ int32_t delta[kMaxBins];          // a digit's output start minus its tile start
    __shared__ int32_t wsum[2][kWaves];
    __shared__ uint32_t s_tile;
    __shared__ uint32_t lkey[kTile];             // the tile in sorted order
    __shared__ int32_t lidx[kTile];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int d0 = threadIdx.x * kDigitsPerThread;   // this thread's digits: d0 + k
    const int nb = 1 << a.bits;
    const uint32_t mask = (uint32_t)nb - 1u;
    if (threadIdx.x == 0) s_tile = atomicAdd(a.ticket, 1u);
    for (int v = 0; v < kWaves; ++v)
        for (int k = 0; k < kDigitsPerThread; ++k) wcnt[v][d0 + k] = 0;
    __syncthreads();
    const uint32_t tile = s_tile;
    const int64_t t0 = (int64_t)tile * kTile;
    const int tcount = (int)(a.Q - t0 < kTile ? a.Q - t0 : kTile);
    int32_t gcount[kDigitsPerThread];   // this pass's batch-wide count of each of this thread's digits
#pragma unroll
    for (int k = 0; k < kDigitsPerThread; ++k)
        gcount[k] = d0 + k < nb ? (int32_t)a.count[d0 + k] : 0;
    // 1. each wavefront ranks its quarter of the tile, 64 keys a round, in
    // input order: a key's rank is the wavefront's count of its digit before
    // the round plus the equal digits on lower lanes (one wavefront's LDS
    // accesses are done in program order, so every lane of a group reads the
    // count before the group's first lane writes the new one)
    const uint64_t below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    int32_t *const cnt = wcnt[w];
    uint32_t key[kPerThread];
    int32_t rank_in_wave[kPerThread], src[kPerThread];
    // every key and input index of this thread in flight at once
    if (a.ks.h) {
        int32_t hv[kPerThread];
#pragma unroll
        for (int r = 0; r < kPerThread; ++r) {
            const int p = w * (kTile / kWaves) + r * 64 + lane;
            hv[r] = p < tcount ? a.ks.h[t0 + p] : -1;
        }
#pragma unroll
        for (int r = 0; r < kPerThread; ++r) key[r] = a.ks.first(hv[r]);
    } else {
#pragma unroll
        for (int r = 0; r < kPerThread; ++r) {
            const int p = w * (kTile / kWaves) + r * 64 + lane;
            key[r] = p < tcount ? a.ks.k[t0 + p] : 0u;
        }
    }
#pragma unroll
    for (int r = 0; r < kPerThread; ++r) {
        const int p = w * (kTile / kWaves) + r * 64 + lane;
        src[r] = a.idx_in && p < tcount ? a.idx_in[t0 + p] : (int32_t)(t0 + p);
    }
#pragma unroll
    for (int r = 0; r < kPerThread; ++r) {
        const int p = w * (kTile / kWaves) + r * 64 + lane;
        const bool valid = p < tcount;
        const uint32_t dig = (key[r] >> a.shift) & mask;
        uint64_t same = __ballot(valid);
        for (int b = 0; b < a.bits; ++b) {
            const uint64_t ones = __ballot(((dig >> b) & 1u) != 0u);
            same &= ((dig >> b) & 1u) ? ones : ~ones;
        }
        const int rank = __popcll(same & below);
        const int32_t before = valid ? cnt[dig] : 0;
        if (valid && rank == 0) cnt[dig] = before + __popcll(same);
        rank_in_wave[r] = before + rank;
    }
    __syncthreads();
    // 2. this thread's digits: the tile's counts, published at once; the
    // wavefronts' offsets; each digit's start in the tile and in the batch
    int32_t c[kDigitsPerThread];
    int32_t csum = 0, gsum = 0;
    uint64_t *const st = a.status + (size_t)tile * kMaxBins + d0;
#pragma unroll
    for (int k = 0; k < kDigitsPerThread; ++k) {
        c[k] = 0;
        if (d0 + k < nb) {
            for (int v = 0; v < kWaves; ++v) c[k] += wcnt[v][d0 + k];
            __hip_atomic_store(st + k, (tile == 0 ? kPrefix : kAggregate) | (uint32_t)c[k],
                               __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            gsum += gcount[k];
        }
        csum += c[k];
    }
    // the keys and their ranks wait in LDS (in input order) during the
    // look-back, which then has the registers for its window
#pragma unroll
    for (int r = 0; r < kPerThread; ++r) {
        const int p = w * (kTile / kWaves) + r * 64 + lane;
        lkey[p] = key[r];
        lidx[p] = rank_in_wave[r];
    }
    int32_t lbase = csum, gbase = gsum;
    block_scan2(lbase, gbase, wsum);
    // 3. look-back: the keys of each digit in the tiles before this one,
    // kLookWindow predecessors at a time, nearest first; the counts are
    // added up to the first inclusive one, and the walk resumes at the first
    // tile not yet published, polling it
    uint32_t before[kDigitsPerThread];
    bool done[kDigitsPerThread];
    int64_t j[kDigitsPerThread];
#pragma unroll
    for (int k = 0; k < kDigitsPerThread; ++k) {
        before[k] = 0;
        done[k] = tile == 0 || d0 + k >= nb;
        j[k] = (int64_t)tile - 1;
    }
    for (int polls = 0;;) {
        uint64_t x[kDigitsPerThread][kLookWindow];
#pragma unroll
        for (int k = 0; k < kDigitsPerThread; ++k)
#pragma unroll
            for (int i = 0; i < kLookWindow; ++i)
                x[k][i] = !done[k] && j[k] - i >= 0
                              ? __hip_atomic_load(a.status + (size_t)(j[k] - i) * kMaxBins + d0 + k,
                                                  __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)
                              : kPrefix;
        bool all = true, progress = false;
#pragma unroll
        for (int k = 0; k < kDigitsPerThread; ++k) {
            if (done[k]) continue;
            int taken = 0;
#pragma unroll
            for (int i = 0; i < kLookWindow; ++i) {
                if (done[k] || taken < i || !(x[k][i] >> 62)) continue;
                before[k] += (uint32_t)x[k][i];
                taken = i + 1;
                done[k] = (x[k][i] & kPrefix) != 0;
            }
            j[k] -= taken;
            progress |= taken > 0;
            all &= done[k];
        }
        if (all) break;
        if (!progress) {
            if (++polls >= kSpinLimit) break;   // never expected; keeps the kernel finite
            __builtin_amdgcn_s_sleep(1);
        }
    }
    int32_t lrun = lbase, grun = gbase;
#pragma unroll
    for (int k = 0; k < kDigitsPerThread; ++k) {
        const int d = d0 + k;
        if (d < nb) {
            if (tile > 0)
                __hip_atomic_store(st + k, kPrefix | (uint32_t)(before[k] + c[k]),
                                   __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            for (int v = 0, o = lrun; v < kWaves; ++v) {
                const int32_t x = wcnt[v][d];
                wcnt[v][d] = o;
                o += x;
            }
            delta[d] = grun + (int32_t)before[k] - lrun;
            lrun += c[k];
            grun += gcount[k];
        }
    }
    __syncthreads();
    // 4. the tile's sorted order in LDS
#pragma unroll
    for (int r = 0; r < kPerThread; ++r) {
        const int p = w * (kTile / kWaves) + r * 64 + lane;
        key[r] = lkey[p];
        rank_in_wave[r] = lidx[p];
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < kPerThread; ++r) {
        const int p = w * (kTile / kWaves) + r * 64 + lane;
        if (p < tcount) {
            const uint32_t dig = (key[r] >> a.shift) & mask;
            const int slot = cnt[dig] + rank_in_wave[r];
            lkey[slot] = key[r];
            lidx[slot] = src[r];
        }
    }
    __syncthreads();
    // 5. the tile written out in sorted order: consecutive lanes, consecutive
    // addresses within each digit's run
    for (int o = threadIdx.x; o < tcount; o += kThreads) {
        const uint32_t k = lkey[o];
        const uint32_t dg = (k >> a.shift) & mask;
        const int32_t to = delta[dg] + o;
        const int32_t from = lidx[o];
        if (a.kout) a.kout[to] = k;
        a.iout[to] = from;
        if (a.rec) {
            const float4 r = a.rec[from];
            a.ho[to] = __float_as_int(r.x);
            a.uo[to] = r.y;
            a.vo[to] = r.z;
            if (a.fo) a.fo[to] = r.w;
        }
    }
}

__global__ void __launch_bounds__(kThreads) k_gather(const int32_t *perm, int64_t Q,
                                                     const int32_t *h, const float *u,
                                                     const float *v, const float *f, int32_t *ho,
                                                     float *uo, float *vo, float *fo)
{
    const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (i >= Q) return;
    const int32_t p = perm[i];
    ho[i] = h[p];
    uo[i] = u[p];
    vo[i] = v[p];
    if (f) fo[i] = f[p];
}

// Row is float or a 4-float vector type (the nontemporal builtins take
// native vectors, not HIP's float4 struct).  The sorted rows and the
// permutation stream through once, so they are loaded nontemporally; the
// scattered stores stay ordinary: nontemporal ones miss the L2's combining
// of the 16-byte pieces of a line and took three times as long.
typedef float row4 __attribute__((ext_vector_type(4)));

template <typename Row>
__global__ void __launch_bounds__(kThreads) k_unpermute(const int32_t *perm, int64_t Q,
                                                        const Row *in, Row *out)
{
    const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (i >= Q) return;
    out[__builtin_nontemporal_load(perm + i)] = __builtin_nontemporal_load(in + i);
}

constexpr int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }

constexpr size_t align256(size_t x) { return (x + 255) / 256 * 256; }

// Passes and digit width for keys 0..H: the fewest passes of at most
// kMaxDigitBits bits, digits split evenly.
struct SortPlan {
    int passes, bits;
};

constexpr SortPlan sort_plan(int32_t H)
{
    int kb = 0;
    for (uint32_t top = (uint32_t)(H > 0 ? H : 0); top > 0; top >>= 1) ++kb;
    if (kb == 0) kb = 1;
    const int passes = (kb + kMaxDigitBits - 1) / kMaxDigitBits;
    return {passes, (kb + passes - 1) / passes};
}

// Workspace layout: the 16-byte query records; the keys of a mapped sort;
// the (key, index) sets the passes between the first and the last write
// (one set for two passes, two for more); then the region cleared before
// every sort -- the digit counts and tile tickets of every pass, and the
// published counts of every tile of every pass.
constexpr size_t kControlBytes = align256(sizeof(uint32_t) * kMaxPasses * (kMaxBins + 1));

constexpr size_t sort_status_bytes(int passes, int64_t ntiles)
{
    return align256(sizeof(uint64_t) * (size_t)passes * (size_t)ntiles * kMaxBins);
}

constexpr size_t sort_ws_bytes(int32_t H, int64_t Q)
{
    const SortPlan p = sort_plan(H);
    const int64_t q = Q > 0 ? Q : 1;
    const int sets = p.passes >= 3 ? 2 : p.passes - 1;
    return align256(16 * (size_t)q) + align256(sizeof(int32_t) * (size_t)q) +
           (size_t)sets * 2 * align256(sizeof(int32_t) * (size_t)q) + kControlBytes +
           sort_status_bytes(p.passes, cdiv(q, kTile));
}

// Device scratch of the allocation-free sort: the workspace of the largest
// batch it takes (kStaticSortMaxQ queries, any H < 2^31), per GPU.
constexpr size_t kStaticSortBytes = sort_ws_bytes(INT32_MAX, kStaticSortMaxQ);
static_assert(kStaticSortBytes <= (size_t)HTEX_SORT_NOALLOC_SCRATCH_MIB << 20,
              "the scratch size stated in htex.h");
static __device__ __align__(256) char scratch[kStaticSortBytes];

}  // namespace

size_t sort_workspace_bytes(int32_t H, int64_t Q) { return sort_ws_bytes(H, Q); }

size_t static_sort_scratch_bytes() { return kStaticSortBytes; }

// The device address of this GPU's `scratch`, looked up once per device with
// that device current (each GPU holds its own copy of the array; in host code
// the array's name is not a device address).
hipError_t static_sort_scratch(void **ptr)
{
    static std::mutex mu;
    static void *addr[kMaxDevices] = {};
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return e;
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(mu);
    if (!addr[dev]) {
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        addr[dev] = p;
    }
    *ptr = addr[dev];
    return hipSuccess;
}

hipError_t launch_sort(int32_t H, const int32_t *key_of_h, int32_t nkeys, int64_t Q,
                       const int32_t *h, const float *u, const float *v, const float *f,
                       int32_t *perm, int32_t *h_out, float *u_out, float *v_out, float *f_out,
                       void *records, void *ws, hipStream_t s)
{
    if (Q == 0) return hipSuccess;
    const int32_t K = key_of_h ? nkeys : H;
    const SortPlan plan = sort_plan(K);
    const bool batch = u_out != nullptr;            // the sorted arrays, gathered by the last pass
    const bool copy = batch || records != nullptr;  // the queries as records
    const int64_t ntiles = cdiv(Q, kTile);
    char *p = static_cast<char *>(ws);
    float4 *rec = records ? static_cast<float4 *>(records) : reinterpret_cast<float4 *>(p);
    p += align256(16 * (size_t)Q);
    const size_t arr = align256(sizeof(int32_t) * (size_t)Q);
    uint32_t *mapped = key_of_h ? reinterpret_cast<uint32_t *>(p) : nullptr;
    p += arr;
    uint32_t *keys[2] = {};
    int32_t *idx[2] = {};
    const int nsets = plan.passes >= 3 ? 2 : plan.passes - 1;
    for (int k = 0; k < nsets; ++k) {
        keys[k] = reinterpret_cast<uint32_t *>(p);
        idx[k] = reinterpret_cast<int32_t *>(p + arr);
        p += 2 * arr;
    }
    uint32_t *count = reinterpret_cast<uint32_t *>(p);   // [kMaxPasses][kMaxBins]
    uint32_t *ticket = count + kMaxPasses * kMaxBins;    // [kMaxPasses]
    uint64_t *status = reinterpret_cast<uint64_t *>(p + kControlBytes);
    const int64_t nclear = (int64_t)(kControlBytes + sort_status_bytes(plan.passes, ntiles)) / 16;
    const dim3 block(kThreads);
    hipLaunchKernelGGL(k_clear, dim3((uint32_t)cdiv(nclear, kThreads)), block, 0, s,
                       reinterpret_cast<uint4 *>(p), nclear);
    hipError_t e = hipGetLastError();
    if (!e) {
        hipLaunchKernelGGL(k_count, dim3((uint32_t)(ntiles < kCountBlocks ? ntiles : kCountBlocks)),
                           block, 0, s, KeySrc{h, nullptr, key_of_h, H, K}, Q, plan.passes,
                           plan.bits, count, copy ? u : nullptr, copy ? v : nullptr,
                           copy ? f : nullptr, copy ? rec : nullptr, mapped);
        e = hipGetLastError();
    }
    // the first pass reads the keys the counting read wrote, or h itself
    KeySrc ks = mapped ? KeySrc{nullptr, mapped, nullptr, H, K} : KeySrc{h, nullptr, nullptr, H, K};
    const int32_t *idx_in = nullptr;
    for (int pass = 0; pass < plan.passes && !e; ++pass) {
        const bool last = pass == plan.passes - 1;
        PassArgs a{};
        a.ks = ks;
        a.idx_in = idx_in;
        a.kout = last ? nullptr : keys[pass & 1];
        a.iout = last ? perm : idx[pass & 1];
        if (last && batch) {
            a.rec = rec;
            a.ho = h_out, a.uo = u_out, a.vo = v_out, a.fo = f_out;
        }
        a.Q = Q;
        a.shift = plan.bits * pass;
        a.bits = plan.bits;
        a.count = count + pass * kMaxBins;
        a.status = status + (size_t)pass * (size_t)ntiles * kMaxBins;
        a.ticket = ticket + pass;
        hipLaunchKernelGGL(k_pass, dim3((uint32_t)ntiles), block, 0, s, a);
        e = hipGetLastError();
        ks = KeySrc{nullptr, a.kout, nullptr, H, K};
        idx_in = a.iout;
    }
    return e;
}

hipError_t launch_gather_queries(const int32_t *perm, int64_t Q, const int32_t *h, const float *u,
                                 const float *v, const float *f, int32_t *ho, float *uo, float *vo,
                                 float *fo, hipStream_t s)
{
    if (Q == 0) return hipSuccess;
    hipLaunchKernelGGL(k_gather, dim3((uint32_t)cdiv(Q, kThreads)), dim3(kThreads), 0, s, perm, Q,
                       h, u, v, f, ho, uo, vo, fo);
    return hipGetLastError();
}

hipError_t launch_unpermute(const int32_t *perm, int64_t Q, int channels, const float *in,
                            float *out, hipStream_t s)
{
    if (Q == 0) return hipSuccess;
    const dim3 grid((uint32_t)cdiv(Q, kThreads));
    if (channels == 4)
        hipLaunchKernelGGL((k_unpermute<row4>), grid, dim3(kThreads), 0, s, perm, Q,
                           reinterpret_cast<const row4 *>(in), reinterpret_cast<row4 *>(out));
    else
        hipLaunchKernelGGL((k_unpermute<float>), grid, dim3(kThreads), 0, s, perm, Q, in, out);
    return hipGetLastError();
}

}  // namespace htex
