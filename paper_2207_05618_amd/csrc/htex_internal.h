// htex_internal.h -- declarations shared by the HIP kernel sources and the
// C-ABI host layer of libhtex.  Not part of the public interface.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "htex.h"

namespace htex {

// Thread-local last-error message shared by every entry point of libhtex.
htex_status set_error(htex_status st, const char *fmt, ...);
void clear_error();

// Everything one sampling or backward launch needs, by value.
struct SampleArgs {
    int32_t H;
    const int32_t *twin, *next, *prev, *edge;
    const uint8_t *log2res;
    const int64_t *base;
    const void *texels;
    const float *scale;
    int64_t Q;
    const int32_t *qh;
    const float *qu, *qv, *qf;
    float *out;                 // forward: [Q][channels]
    htex_debug_rec *dbg;        // forward, nullable
    int32_t *err;               // forward, nullable
    const float *dout;          // backward: [Q][channels]
    float *dtex;                // backward: pool-shaped float32
    const void *prep;           // prepared descriptors (fast path), nullable
    int32_t channels;           // values per texel and per output row: 4 or 1
    int32_t has_mips;           // prepared path: the pool's layout has mip levels
    int64_t total_texels;       // prepared path: size of the pool in texels
    const int32_t *order;       // prepared forward, nullable: query q is record order[q] ...
    const void *qrec;           // ... of these 16-byte records (h bits, u, v, footprint)
};

// Offset of mip level l inside an edge of log2 resolution k, in texels:
// levels are stored from the finest to the coarsest, so level l follows
// sum_{m<l} 4^(k-m) = (4^(k+1) - 4^(k+1-l)) / 3 texels.
__host__ __device__ inline int64_t level_offset(int k, int l)
{
    return ((int64_t(1) << (2 * k + 2)) - (int64_t(1) << (2 * (k - l) + 2))) / 3;
}

// A sum of float32 values kept as an unevaluated pair hi + lo: each
// addition's rounding error is recovered exactly (Knuth's TwoSum) and
// collected in lo, so a mean of a few values comes out correctly rounded
// without leaving float32 arithmetic.
struct PairSum {
    float hi = 0.0f, lo = 0.0f;

    __device__ __forceinline__ void add(float x)
    {
        const float s = hi + x;
        const float bb = s - hi;
        const float e = (hi - (s - bb)) + (x - bb);
        hi = s;
        lo += e;
    }

    // (hi + lo) / n: the remainder of the first quotient, hi - q0 n, is exact
    // in one fused multiply-add, and is folded back with lo.
    __device__ __forceinline__ float mean(int n) const
    {
        const float fn = (float)n;
        const float q0 = hi / fn;
        const float r = __builtin_fmaf(-q0, fn, hi) + lo;
        return q0 + r / fn;
    }
};

// Serving: a resident mesh (prepared records + pool) and a tile of one
// request's queries.
struct ServeMesh {
    const void *prep;
    const void *texels;
    const float *scale;
    int64_t total_texels;
    int32_t H;
    int32_t has_mips;
};

struct ServeTile {
    const int32_t *h;
    const float *u, *v, *f;
    float *out;
    int64_t q0;        // first query of the tile inside the request's arrays
    int32_t mesh;
    int32_t count;     // 1..kTileQueries
};
constexpr int kTileQueries = 256;

// Largest batch of the allocation-free sort, and the most devices whose
// scratch addresses are kept.
constexpr int64_t kStaticSortMaxQ = HTEX_SORT_NOALLOC_MAX_Q;
constexpr int kMaxDevices = 64;

hipError_t launch_sample(const SampleArgs &a, int dtype, int filter, hipStream_t s);
size_t sort_workspace_bytes(int32_t H, int64_t Q);
size_t static_sort_scratch_bytes();
hipError_t static_sort_scratch(void **ptr);
// Sorts by halfedge (or by key_of_h[h], keys 0 .. nkeys - 1, when key_of_h
// is non-NULL): perm, and (when u_out is non-NULL) the sorted h, u, v and
// (when f_out is non-NULL) footprint.  The workspace is sized for the key
// range: sort_workspace_bytes(key_of_h ? nkeys : H, Q).
// With `records` (16 bytes per query), the queries are also copied there
// in input order as (h bits, u, v, footprint), and no sorted arrays are
// written (u_out must then be NULL).
hipError_t launch_sort(int32_t H, const int32_t *key_of_h, int32_t nkeys, int64_t Q,
                       const int32_t *h, const float *u, const float *v, const float *f,
                       int32_t *perm, int32_t *h_out, float *u_out, float *v_out, float *f_out,
                       void *records, void *ws, hipStream_t s);
hipError_t launch_gather_queries(const int32_t *perm, int64_t Q, const int32_t *h, const float *u,
                                 const float *v, const float *f, int32_t *ho, float *uo, float *vo,
                                 float *fo, hipStream_t s);
hipError_t launch_unpermute(const int32_t *perm, int64_t Q, int channels, const float *in,
                            float *out, hipStream_t s);
hipError_t launch_serve(const ServeMesh *meshes, const ServeTile *tiles, int32_t ntiles,
                        int32_t grid, int dtype, int channels, int filter, int32_t *err,
                        hipStream_t s);
hipError_t launch_backward(const SampleArgs &a, int filter, uint32_t flags, int max_log2res,
                           hipStream_t s);
hipError_t launch_prepare(const SampleArgs &a, void *prep, hipStream_t s);
hipError_t launch_sample_prepared(const SampleArgs &a, int dtype, int filter, bool scattered,
                                  bool cache_resident, hipStream_t s);
hipError_t launch_sample_aniso(const SampleArgs &a, int dtype, const float *jac, int max_aniso,
                               int32_t *nprobe, hipStream_t s);
hipError_t launch_build_mips(float *texels, const uint8_t *log2res, const int64_t *base,
                             int32_t E, int max_k, int channels, hipStream_t s);
hipError_t launch_mip_backward(float *dtex, const uint8_t *log2res, const int64_t *base, int32_t E,
                               int max_k, int channels, int clear, hipStream_t s);
hipError_t launch_quantize_bf16(const float *src, uint16_t *dst, int64_t count,
                                hipStream_t s);
hipError_t launch_quantize_fp8(const float *src, uint8_t *dst, float *scale,
                               const uint8_t *log2res, const int64_t *base, int32_t E,
                               int has_mips, int channels, int64_t total_texels, hipStream_t s);
hipError_t launch_corner_average(const htex_mesh &m, float *texels, const uint8_t *log2res,
                                 const int64_t *base, int channels, int has_mips, int kmax,
                                 int32_t *err, hipStream_t s);
hipError_t launch_triangle_vertices(const htex_mesh &m, const int32_t *vert, int32_t V,
                                    const float *pos, float *out, int32_t *err, hipStream_t s);
hipError_t launch_validate(const htex_mesh &m, int32_t *ws_use, int32_t *ws_bad,
                           hipStream_t s);

}  // namespace htex
