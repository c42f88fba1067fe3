// htex_sort.hip -- ordering a query batch by halfedge (optional step before
// sampling) and moving queries and results between the two orders.
//
// Stable LSD radix sort of the keys h (8-bit digits, as many passes as the
// key range needs); invalid h (outside [0, H)) get the key H and sort last.
// Each pass: a 256-bin digit histogram per tile of kTile keys, an exclusive
// scan of the histograms in digit-major order (so tile t's digit d starts
// after every smaller digit and after digit d of tiles < t), then a stable
// scatter in which every key's rank among equal digits of its tile comes
// from wave ballots (within a wave) and per-wave counts (across waves).
#include <hip/hip_runtime.h>

#include "htex_internal.h"

namespace htex {
namespace {

constexpr int kThreads = 256;
constexpr int kPerThread = 16;
constexpr int kTile = kThreads * kPerThread;   // 4096 keys per tile
constexpr int kWaves = kThreads / 64;

__device__ __forceinline__ uint32_t sort_key(int32_t h, int32_t H)
{
    return ((uint32_t)h < (uint32_t)H) ? (uint32_t)h : (uint32_t)H;
}

__global__ void __launch_bounds__(kThreads) k_init(const int32_t *h, int32_t H, int64_t Q,
                                                   uint32_t *keys, int32_t *idx)
{
    const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (i < Q) {
        keys[i] = sort_key(h[i], H);
        idx[i] = (int32_t)i;
    }
}

// hist[d * ntiles + t] = number of keys of tile t whose digit is d
__global__ void __launch_bounds__(kThreads) k_hist(const uint32_t *keys, int64_t Q, int shift,
                                                   int32_t ntiles, int32_t *hist)
{
    __shared__ int32_t cnt[256];
    cnt[threadIdx.x] = 0;
    __syncthreads();
    const int64_t t0 = (int64_t)blockIdx.x * kTile;
    for (int r = 0; r < kPerThread; ++r) {
        const int64_t i = t0 + (int64_t)r * kThreads + threadIdx.x;
        if (i < Q) atomicAdd(&cnt[(keys[i] >> shift) & 255u], 1);
    }
    __syncthreads();
    hist[(int64_t)threadIdx.x * ntiles + blockIdx.x] = cnt[threadIdx.x];
}

// Exclusive scan of int32 data in place, one level: each block scans 1024
// values and writes its total to sums[block].
__global__ void __launch_bounds__(kThreads) k_scan_block(int32_t *data, int64_t n, int32_t *sums)
{
    __shared__ int32_t s[kThreads];
    const int64_t b0 = (int64_t)blockIdx.x * kThreads * 4;
    int32_t v[4];
    int32_t local = 0;
    for (int j = 0; j < 4; ++j) {
        const int64_t i = b0 + (int64_t)threadIdx.x * 4 + j;
        v[j] = i < n ? data[i] : 0;
        local += v[j];
    }
    s[threadIdx.x] = local;
    __syncthreads();
    for (int off = 1; off < kThreads; off <<= 1) {
        const int32_t add = threadIdx.x >= (unsigned)off ? s[threadIdx.x - off] : 0;
        __syncthreads();
        s[threadIdx.x] += add;
        __syncthreads();
    }
    int32_t run = s[threadIdx.x] - local;   // exclusive prefix of this thread
    for (int j = 0; j < 4; ++j) {
        const int64_t i = b0 + (int64_t)threadIdx.x * 4 + j;
        if (i < n) data[i] = run;
        run += v[j];
    }
    if (threadIdx.x == kThreads - 1 && sums) sums[blockIdx.x] = s[kThreads - 1];
}

__global__ void __launch_bounds__(kThreads) k_scan_add(int32_t *data, int64_t n, const int32_t *sums)
{
    const int64_t b0 = (int64_t)blockIdx.x * kThreads * 4;
    const int32_t add = sums[blockIdx.x];
    for (int j = 0; j < 4; ++j) {
        const int64_t i = b0 + (int64_t)threadIdx.x * 4 + j;
        if (i < n) data[i] += add;
    }
}

// Stable scatter of one tile: keys are taken in input order, kThreads at a
// time; a key's destination is the global start of its digit for this tile
// plus the number of equal digits before it in the tile.
__global__ void __launch_bounds__(kThreads) k_scatter(const uint32_t *kin, const int32_t *vin,
                                                      uint32_t *kout, int32_t *vout, int64_t Q,
                                                      int shift, int32_t ntiles,
                                                      const int32_t *offs)
{
    __shared__ int32_t base[256];          // running start of each digit
    __shared__ int32_t wcnt[kWaves][256];  // per-wave digit counts of a round
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    base[threadIdx.x] = offs[(int64_t)threadIdx.x * ntiles + blockIdx.x];
    const int64_t t0 = (int64_t)blockIdx.x * kTile;
    for (int r = 0; r < kPerThread; ++r) {
        for (int d = threadIdx.x; d < kWaves * 256; d += kThreads) (&wcnt[0][0])[d] = 0;
        __syncthreads();
        const int64_t i = t0 + (int64_t)r * kThreads + threadIdx.x;
        const bool valid = i < Q;
        const uint32_t key = valid ? kin[i] : 0u;
        const uint32_t dig = (key >> shift) & 255u;
        // lanes of this wave holding the same digit
        uint64_t same = __ballot(valid);
        for (int b = 0; b < 8; ++b) {
            const uint64_t ones = __ballot(((dig >> b) & 1u) != 0u);
            same &= ((dig >> b) & 1u) ? ones : ~ones;
        }
        const uint64_t below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
        const int rank = __popcll(same & below);
        if (valid && rank == 0) wcnt[w][dig] = __popcll(same);
        __syncthreads();
        if (valid) {
            int before = 0;
            for (int v = 0; v < w; ++v) before += wcnt[v][dig];
            const int32_t dst = base[dig] + before + rank;
            kout[dst] = key;
            vout[dst] = vin[i];
        }
        __syncthreads();
        // advance the digit starts past this round
        {
            int tot = 0;
            for (int v = 0; v < kWaves; ++v) tot += wcnt[v][threadIdx.x];
            base[threadIdx.x] += tot;
        }
        __syncthreads();
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

__global__ void __launch_bounds__(kThreads) k_unpermute(const int32_t *perm, int64_t Q,
                                                        const float4 *in, float4 *out)
{
    const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (i >= Q) return;
    out[perm[i]] = in[i];
}

inline int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }

size_t align256(size_t x) { return (x + 255) / 256 * 256; }

// Scan workspace: one partial-sum array per level.
size_t scan_ws_bytes(int64_t n)
{
    size_t b = 0;
    while (n > 1) {
        n = cdiv(n, kThreads * 4);
        b += align256(sizeof(int32_t) * (size_t)n);
    }
    return b;
}

hipError_t scan_exclusive(int32_t *data, int64_t n, int32_t *ws, hipStream_t s)
{
    const int64_t nb = cdiv(n, kThreads * 4);
    int32_t *sums = ws;
    hipLaunchKernelGGL(k_scan_block, dim3((uint32_t)nb), dim3(kThreads), 0, s, data, n,
                       nb > 1 ? sums : nullptr);
    hipError_t e = hipGetLastError();
    if (e || nb == 1) return e;
    int32_t *next_ws = ws + align256(sizeof(int32_t) * nb) / sizeof(int32_t);
    e = scan_exclusive(sums, nb, next_ws, s);
    if (e) return e;
    hipLaunchKernelGGL(k_scan_add, dim3((uint32_t)nb), dim3(kThreads), 0, s, data, n, sums);
    return hipGetLastError();
}

}  // namespace

size_t sort_workspace_bytes(int64_t Q)
{
    const int64_t ntiles = cdiv(Q > 0 ? Q : 1, kTile);
    return 2 * align256(sizeof(uint32_t) * Q) + align256(sizeof(int32_t) * Q) +
           align256(sizeof(int32_t) * 256 * ntiles) + scan_ws_bytes(256 * ntiles);
}

hipError_t launch_sort(const int32_t *h, int32_t H, int64_t Q, int32_t *perm, void *ws,
                       hipStream_t s)
{
    if (Q == 0) return hipSuccess;
    char *p = static_cast<char *>(ws);
    uint32_t *ka = reinterpret_cast<uint32_t *>(p);
    p += align256(sizeof(uint32_t) * Q);
    uint32_t *kb = reinterpret_cast<uint32_t *>(p);
    p += align256(sizeof(uint32_t) * Q);
    int32_t *vb = reinterpret_cast<int32_t *>(p);
    p += align256(sizeof(int32_t) * Q);
    const int64_t ntiles = cdiv(Q, kTile);
    int32_t *hist = reinterpret_cast<int32_t *>(p);
    p += align256(sizeof(int32_t) * 256 * ntiles);
    int32_t *scan_ws = reinterpret_cast<int32_t *>(p);
    // passes: enough 8-bit digits to cover keys 0..H
    int passes = 0;
    for (uint64_t top = (uint64_t)H; top > 0; top >>= 8) ++passes;
    if (passes == 0) passes = 1;
    // the last pass must land in perm: start in perm when the count is odd
    int32_t *va = (passes & 1) ? vb : perm;
    int32_t *vc = (passes & 1) ? perm : vb;
    hipLaunchKernelGGL(k_init, dim3((uint32_t)cdiv(Q, kThreads)), dim3(kThreads), 0, s, h, H, Q, ka,
                       va);
    hipError_t e = hipGetLastError();
    for (int pass = 0; pass < passes && !e; ++pass) {
        const int shift = 8 * pass;
        hipLaunchKernelGGL(k_hist, dim3((uint32_t)ntiles), dim3(kThreads), 0, s, ka, Q, shift,
                           (int32_t)ntiles, hist);
        e = hipGetLastError();
        if (!e) e = scan_exclusive(hist, 256 * ntiles, scan_ws, s);
        if (!e) {
            hipLaunchKernelGGL(k_scatter, dim3((uint32_t)ntiles), dim3(kThreads), 0, s, ka, va, kb,
                               vc, Q, shift, (int32_t)ntiles, hist);
            e = hipGetLastError();
        }
        uint32_t *kt = ka;
        ka = kb;
        kb = kt;
        int32_t *vt = va;
        va = vc;
        vc = vt;
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

hipError_t launch_unpermute(const int32_t *perm, int64_t Q, const float *in, float *out,
                            hipStream_t s)
{
    if (Q == 0) return hipSuccess;
    hipLaunchKernelGGL(k_unpermute, dim3((uint32_t)cdiv(Q, kThreads)), dim3(kThreads), 0, s, perm,
                       Q, reinterpret_cast<const float4 *>(in), reinterpret_cast<float4 *>(out));
    return hipGetLastError();
}

}  // namespace htex
