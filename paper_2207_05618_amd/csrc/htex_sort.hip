// htex_sort.hip -- ordering a query batch by halfedge (optional step before
// sampling) and moving queries and results between the two orders.
//
// Stable LSD radix sort of (key, input index) pairs; the key of a query is h,
// or H for an invalid h (outside [0, H)), which sorts last.  Digits are as
// wide as needed to cover keys 0..H in the fewest passes of at most 10 bits
// (two passes for a million halfedges).  Each pass: a digit histogram per
// tile of kTile keys, an exclusive scan of the histograms in digit-major
// order (so tile t's digit d starts after every smaller digit and after
// digit d of tiles < t), then the scatter.  The scatter first sorts its tile
// in LDS, stably (a key's rank among equal digits comes from wave ballots
// within a wave and per-wave counts across the waves of a round), and then
// writes the tile out in that order, so consecutive lanes store consecutive
// addresses of a digit's run instead of one scattered word each.
// A sorted batch: the first histogram pass also copies the queries into
// 16-byte records (h, u, v, footprint), which are gathered through the
// final permutation -- one 16-byte read per query instead of one read per
// array.
#include <hip/hip_runtime.h>

#include <mutex>

#include "htex_internal.h"

namespace htex {
namespace {

constexpr int kThreads = 256;
constexpr int kPerThread = 16;
constexpr int kTile = kThreads * kPerThread;   // 4096 keys per tile
constexpr int kWaves = kThreads / 64;
constexpr int kMaxDigitBits = 10;
constexpr int kMaxBins = 1 << kMaxDigitBits;

__device__ __forceinline__ uint32_t sort_key(int32_t h, int32_t H)
{
    return ((uint32_t)h < (uint32_t)H) ? (uint32_t)h : (uint32_t)H;
}

// The keys of a pass: computed from h (first pass) or read back (later
// passes).
struct KeySrc {
    const int32_t *h;     // first pass, else NULL
    const uint32_t *k;    // later passes
    int32_t H;

    __device__ __forceinline__ uint32_t operator()(int64_t i) const
    {
        return h ? sort_key(h[i], H) : k[i];
    }
};

// hist[d * ntiles + t] = number of keys of tile t whose digit is d;
// hist[nb * ntiles] = 0, so that the exclusive scan leaves Q there.  With
// `rec`, the first pass also writes every query as one 16-byte record.
__global__ void __launch_bounds__(kThreads) k_hist(KeySrc ks, int64_t Q, int shift, int bits,
                                                   int32_t ntiles, int32_t *hist,
                                                   const float *u, const float *v,
                                                   const float *f, float4 *rec)
{
    __shared__ int32_t cnt[kMaxBins];
    const int nb = 1 << bits;
    for (int d = threadIdx.x; d < nb; d += kThreads) cnt[d] = 0;
    __syncthreads();
    const int64_t t0 = (int64_t)blockIdx.x * kTile;
    const uint32_t mask = (uint32_t)nb - 1u;
    for (int r = 0; r < kPerThread; ++r) {
        const int64_t i = t0 + (int64_t)r * kThreads + threadIdx.x;
        if (i < Q) {
            atomicAdd(&cnt[(ks(i) >> shift) & mask], 1);
            if (rec)
                rec[i] = make_float4(__int_as_float(ks.h[i]), u[i], v[i], f ? f[i] : 0.0f);
        }
    }
    __syncthreads();
    for (int d = threadIdx.x; d < nb; d += kThreads)
        hist[(int64_t)d * ntiles + blockIdx.x] = cnt[d];
    if (blockIdx.x == 0 && threadIdx.x == 0) hist[(int64_t)nb * ntiles] = 0;
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

// One pass of the scatter.  offs: the scanned histograms (nb * ntiles + 1
// entries).  idx_in NULL stands for the identity; kout NULL on the last pass
// (the keys are no longer needed).
__global__ void __launch_bounds__(kThreads) k_scatter(KeySrc ks, const int32_t *idx_in,
                                                      uint32_t *kout, int32_t *iout, int64_t Q,
                                                      int shift, int bits, int32_t ntiles,
                                                      const int32_t *offs)
{
    __shared__ int32_t gstart[kMaxBins];        // global start of each digit's run of this tile
    __shared__ int32_t lstart[kMaxBins];        // its start inside the tile
    __shared__ int32_t lrun[kMaxBins];          // next free local slot of each digit
    __shared__ int32_t wcnt[kWaves][kMaxBins];  // per-wave digit counts of a round
    __shared__ int32_t part[kThreads];
    __shared__ uint32_t lkey[kTile];
    __shared__ int32_t lidx[kTile];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int nb = 1 << bits;
    const uint32_t mask = (uint32_t)nb - 1u;
    const int64_t t0 = (int64_t)blockIdx.x * kTile;
    const int tcount = (int)(Q - t0 < kTile ? Q - t0 : kTile);
    // digit runs of this tile: global starts, counts, and a local exclusive
    // scan of the counts (each thread scans a chunk of nb / 256 digits)
    const int per = (nb + kThreads - 1) / kThreads;
    int32_t csum = 0;
    for (int j = 0; j < per; ++j) {
        const int d = threadIdx.x * per + j;
        if (d < nb) {
            const int64_t at = (int64_t)d * ntiles + blockIdx.x;
            const int32_t g = offs[at];
            gstart[d] = g;
            lstart[d] = offs[at + 1] - g;   // the count, for now
            csum += offs[at + 1] - g;
            for (int v = 0; v < kWaves; ++v) wcnt[v][d] = 0;
        }
    }
    part[threadIdx.x] = csum;
    __syncthreads();
    if (threadIdx.x < 64) {
        const int l = threadIdx.x;
        const int32_t v0 = part[4 * l], v1 = part[4 * l + 1], v2 = part[4 * l + 2],
                      v3 = part[4 * l + 3];
        const int32_t tot = v0 + v1 + v2 + v3;
        int32_t inc = tot;
        for (int dd = 1; dd < 64; dd <<= 1) {
            const int32_t y = __shfl_up(inc, dd);
            if (l >= dd) inc += y;
        }
        const int32_t ex = inc - tot;
        part[4 * l] = ex;
        part[4 * l + 1] = ex + v0;
        part[4 * l + 2] = ex + v0 + v1;
        part[4 * l + 3] = ex + v0 + v1 + v2;
    }
    __syncthreads();
    {
        int32_t run = part[threadIdx.x];
        for (int j = 0; j < per; ++j) {
            const int d = threadIdx.x * per + j;
            if (d < nb) {
                const int32_t c = lstart[d];
                lstart[d] = run;
                lrun[d] = run;
                run += c;
            }
        }
    }
    __syncthreads();
    // the tile sorted into LDS, kThreads keys per round
    const uint64_t below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    for (int r = 0; r < kPerThread; ++r) {
        const int li = r * kThreads + (int)threadIdx.x;
        const int64_t i = t0 + li;
        const bool valid = li < tcount;
        const uint32_t key = valid ? ks(i) : 0u;
        const int32_t id = valid ? (idx_in ? idx_in[i] : (int32_t)i) : 0;
        const uint32_t dig = (key >> shift) & mask;
        // lanes of this wave holding the same digit
        uint64_t same = __ballot(valid);
        for (int b = 0; b < bits; ++b) {
            const uint64_t ones = __ballot(((dig >> b) & 1u) != 0u);
            same &= ((dig >> b) & 1u) ? ones : ~ones;
        }
        const int rank = __popcll(same & below);
        const int cnt = __popcll(same);
        const bool leader = valid && rank == 0;
        if (leader) wcnt[w][dig] = cnt;
        __syncthreads();
        int before = 0, after = 0;
        if (valid) {
            for (int v = 0; v < kWaves; ++v) {
                const int c = wcnt[v][dig];
                before += v < w ? c : 0;
                after += v > w ? c : 0;
            }
            const int p = lrun[dig] + before + rank;
            lkey[p] = key;
            lidx[p] = id;
        }
        __syncthreads();
        if (leader) {
            if (after == 0) lrun[dig] += before + cnt;
            wcnt[w][dig] = 0;
        }
        __syncthreads();
    }
    // the tile written out in sorted order: consecutive lanes, consecutive
    // addresses within each digit's run
    for (int o = threadIdx.x; o < tcount; o += kThreads) {
        const uint32_t key = lkey[o];
        const uint32_t d = (key >> shift) & mask;
        const int32_t dst = gstart[d] + (o - lstart[d]);
        if (kout) kout[dst] = key;
        iout[dst] = lidx[o];
    }
}

// The sorted batch: query perm[i] of the 16-byte records into row i of the
// sorted arrays.
__global__ void __launch_bounds__(kThreads) k_gather_records(const int32_t *perm, int64_t Q,
                                                             const float4 *rec, int32_t *ho,
                                                             float *uo, float *vo, float *fo)
{
    const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (i >= Q) return;
    const float4 r = rec[perm[i]];
    ho[i] = __float_as_int(r.x);
    uo[i] = r.y;
    vo[i] = r.z;
    if (fo) fo[i] = r.w;
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

template <typename Row>
__global__ void __launch_bounds__(kThreads) k_unpermute(const int32_t *perm, int64_t Q,
                                                        const Row *in, Row *out)
{
    const int64_t i = (int64_t)blockIdx.x * kThreads + threadIdx.x;
    if (i >= Q) return;
    out[perm[i]] = in[i];
}

constexpr int64_t cdiv(int64_t a, int64_t b) { return (a + b - 1) / b; }

constexpr size_t align256(size_t x) { return (x + 255) / 256 * 256; }

// Scan workspace: one partial-sum array per level.
constexpr size_t scan_ws_bytes(int64_t n)
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

// Workspace layout: the 16-byte query records, the (key, index) sets the
// passes between the first and the last write (one set for two passes, two
// for more), the histograms and the scan partials.
constexpr size_t sort_ws_bytes(int32_t H, int64_t Q)
{
    const SortPlan p = sort_plan(H);
    const int64_t q = Q > 0 ? Q : 1;
    const int64_t ntiles = cdiv(q, kTile);
    const int64_t nhist = ((int64_t)1 << p.bits) * ntiles + 1;
    const int sets = p.passes >= 3 ? 2 : p.passes - 1;
    return align256(16 * (size_t)q) + (size_t)sets * 2 * align256(sizeof(int32_t) * (size_t)q) +
           align256(sizeof(int32_t) * (size_t)nhist) + scan_ws_bytes(nhist);
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

hipError_t launch_sort(int32_t H, int64_t Q, const int32_t *h, const float *u, const float *v,
                       const float *f, int32_t *perm, int32_t *h_out, float *u_out, float *v_out,
                       float *f_out, void *ws, hipStream_t s)
{
    if (Q == 0) return hipSuccess;
    const SortPlan plan = sort_plan(H);
    const bool batch = u_out != nullptr;
    char *p = static_cast<char *>(ws);
    float4 *rec = reinterpret_cast<float4 *>(p);
    p += align256(16 * (size_t)Q);
    const size_t arr = align256(sizeof(int32_t) * (size_t)Q);
    uint32_t *keys[2];
    int32_t *idx[2];
    const int nsets = plan.passes >= 3 ? 2 : plan.passes - 1;
    for (int k = 0; k < nsets; ++k) {
        keys[k] = reinterpret_cast<uint32_t *>(p);
        idx[k] = reinterpret_cast<int32_t *>(p + arr);
        p += 2 * arr;
    }
    const int64_t ntiles = cdiv(Q, kTile);
    const int64_t nhist = ((int64_t)1 << plan.bits) * ntiles + 1;
    int32_t *hist = reinterpret_cast<int32_t *>(p);
    p += align256(sizeof(int32_t) * (size_t)nhist);
    int32_t *scan_ws = reinterpret_cast<int32_t *>(p);
    KeySrc ks{h, nullptr, H};
    const int32_t *idx_in = nullptr;
    hipError_t e = hipSuccess;
    const dim3 grid((uint32_t)ntiles), block(kThreads);
    for (int pass = 0; pass < plan.passes && !e; ++pass) {
        const int shift = plan.bits * pass;
        const bool last = pass == plan.passes - 1;
        uint32_t *kout = last ? nullptr : keys[pass & 1];
        int32_t *iout = last ? perm : idx[pass & 1];
        const bool copy = batch && pass == 0;
        hipLaunchKernelGGL(k_hist, grid, block, 0, s, ks, Q, shift, plan.bits, (int32_t)ntiles,
                           hist, copy ? u : nullptr, copy ? v : nullptr, copy ? f : nullptr,
                           copy ? rec : nullptr);
        e = hipGetLastError();
        if (!e) e = scan_exclusive(hist, nhist, scan_ws, s);
        if (!e) {
            hipLaunchKernelGGL(k_scatter, grid, block, 0, s, ks, idx_in, kout, iout, Q, shift,
                               plan.bits, (int32_t)ntiles, hist);
            e = hipGetLastError();
        }
        ks = KeySrc{nullptr, kout, H};
        idx_in = iout;
    }
    if (!e && batch) {
        hipLaunchKernelGGL(k_gather_records, dim3((uint32_t)cdiv(Q, kThreads)), block, 0, s, perm,
                           Q, rec, h_out, u_out, v_out, f_out);
        e = hipGetLastError();
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
        hipLaunchKernelGGL((k_unpermute<float4>), grid, dim3(kThreads), 0, s, perm, Q,
                           reinterpret_cast<const float4 *>(in), reinterpret_cast<float4 *>(out));
    else
        hipLaunchKernelGGL((k_unpermute<float>), grid, dim3(kThreads), 0, s, perm, Q, in, out);
    return hipGetLastError();
}

}  // namespace htex
