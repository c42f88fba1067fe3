// htex_api.cpp -- the C ABI of libhtex: synchronous argument checks, pool
// layout, dispatch of the HIP kernels, status codes and messages.
#include <hip/hip_runtime.h>

#include <climits>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>

#include "htex.h"
#include "htex_internal.h"

namespace {
thread_local std::string g_last_error;
}  // namespace

namespace htex {

htex_status set_error(htex_status st, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return st;
}

void clear_error() { g_last_error.clear(); }

}  // namespace htex

namespace {

#define fail htex::set_error

htex_status ok()
{
    htex::clear_error();
    return HTEX_OK;
}

htex_status from_hip(hipError_t e, const char *what)
{
    if (e == hipSuccess) return ok();
    return fail(HTEX_E_DEVICE, "%s: %s", what, hipGetErrorString(e));
}

bool aligned(const void *p, size_t a) { return (reinterpret_cast<uintptr_t>(p) % a) == 0; }

// Bytes of one stored texel (all channels), 0 for an unknown dtype.
size_t texel_bytes(int32_t dtype, int32_t channels)
{
    switch (dtype) {
    case HTEX_F32: return 4 * (size_t)channels;
    case HTEX_BF16: return 2 * (size_t)channels;
    case HTEX_FP8_E4M3: return (size_t)channels;
    default: return 0;
    }
}

htex_status check_flags(uint32_t flags)
{
    if (flags & ~(HTEX_QUERIES_SORTED | HTEX_QUERIES_SCATTERED))
        return fail(HTEX_E_ARG, "unknown flags 0x%x", flags);
    if ((flags & HTEX_QUERIES_SORTED) && (flags & HTEX_QUERIES_SCATTERED))
        return fail(HTEX_E_ARG, "HTEX_QUERIES_SORTED and HTEX_QUERIES_SCATTERED contradict");
    return HTEX_OK;
}

htex_status check_mesh(const htex_mesh *m)
{
    if (!m) return fail(HTEX_E_ARG, "mesh is NULL");
    if (m->H < 0 || m->E < 0) return fail(HTEX_E_ARG, "negative H or E");
    if (m->H > 0 && (!m->twin || !m->next || !m->prev || !m->edge))
        return fail(HTEX_E_ARG, "a halfedge array is NULL");
    if (m->E > m->H) return fail(HTEX_E_ARG, "E (%d) exceeds H (%d)", m->E, m->H);
    return HTEX_OK;
}

htex_status check_pool(const htex_pool *p, const htex_mesh *m)
{
    if (!p) return fail(HTEX_E_ARG, "pool is NULL");
    if (m && p->E != m->E) return fail(HTEX_E_ARG, "pool has %d edges, mesh has %d", p->E, m->E);
    if (p->E < 0 || p->total_texels < 0) return fail(HTEX_E_ARG, "negative pool size");
    if (p->channels != 1 && p->channels != 4)
        return fail(HTEX_E_ARG, "channels must be 1 or 4, got %d", p->channels);
    if (p->reserved != 0) return fail(HTEX_E_ARG, "pool->reserved must be 0");
    const size_t tb = texel_bytes(p->dtype, p->channels);
    if (!tb) return fail(HTEX_E_ARG, "unknown texel dtype %d", p->dtype);
    if (p->has_mips != 0 && p->has_mips != 1) return fail(HTEX_E_ARG, "has_mips must be 0 or 1");
    if (p->max_log2res < 0 || p->max_log2res > 15)
        return fail(HTEX_E_RANGE, "max_log2res %d outside [0, 15]", p->max_log2res);
    if (p->E > 0 && (!p->log2res || !p->base || !p->texels))
        return fail(HTEX_E_ARG, "a pool array is NULL");
    if (p->texels && !aligned(p->texels, tb))
        return fail(HTEX_E_ARG, "texels must be %zu-byte aligned", tb);
    if (p->dtype == HTEX_FP8_E4M3 && p->E > 0 && !p->scale)
        return fail(HTEX_E_ARG, "FP8 pool needs per-edge scales");
    return HTEX_OK;
}

htex_status check_queries(const htex_queries *q, int32_t filter)
{
    if (!q) return fail(HTEX_E_ARG, "queries is NULL");
    if (q->Q < 0) return fail(HTEX_E_ARG, "negative query count");
    if (q->Q > (int64_t)INT32_MAX * 128) return fail(HTEX_E_RANGE, "too many queries in one call");
    if (q->Q > 0 && (!q->h || !q->u || !q->v)) return fail(HTEX_E_ARG, "a query array is NULL");
    if (filter != HTEX_BILINEAR && filter != HTEX_TRILINEAR)
        return fail(HTEX_E_ARG, "unknown filter %d", filter);
    if (filter == HTEX_TRILINEAR && q->Q > 0 && !q->footprint)
        return fail(HTEX_E_ARG, "trilinear filtering needs footprints");
    return HTEX_OK;
}

htex::SampleArgs make_args(const htex_mesh *m, const htex_pool *p, const htex_queries *q)
{
    htex::SampleArgs a{};
    a.H = m->H;
    a.twin = m->twin;
    a.next = m->next;
    a.prev = m->prev;
    a.edge = m->edge;
    a.log2res = p->log2res;
    a.base = p->base;
    a.texels = p->texels;
    a.scale = p->scale;
    a.Q = q->Q;
    a.qh = q->h;
    a.qu = q->u;
    a.qv = q->v;
    a.qf = q->footprint;
    a.channels = p->channels;
    return a;
}

}  // namespace

extern "C" {

const char *htex_last_error(void) { return g_last_error.c_str(); }

const char *htex_status_string(htex_status s)
{
    switch (s) {
    case HTEX_OK: return "ok";
    case HTEX_E_ARG: return "invalid argument";
    case HTEX_E_TOPOLOGY: return "invalid halfedge topology";
    case HTEX_E_RANGE: return "size out of supported range";
    case HTEX_E_DEVICE: return "device error";
    case HTEX_E_UNSUPPORTED: return "unsupported";
    case HTEX_E_BUSY: return "busy";
    case HTEX_E_NOMEM: return "out of memory budget";
    default: return "unknown status";
    }
}

htex_status htex_pool_layout(int32_t E, const uint8_t *log2res_host, int32_t has_mips,
                             int64_t *base_host_out, int64_t *total_texels_out)
{
    if (E < 0) return fail(HTEX_E_ARG, "negative E");
    if ((E > 0 && (!log2res_host || !base_host_out)) || !total_texels_out)
        return fail(HTEX_E_ARG, "NULL argument");
    if (has_mips != 0 && has_mips != 1) return fail(HTEX_E_ARG, "has_mips must be 0 or 1");
    int64_t off = 0;
    for (int32_t e = 0; e < E; ++e) {
        const int k = log2res_host[e];
        if (k > 15) return fail(HTEX_E_RANGE, "log2res[%d] = %d exceeds 15", e, k);
        int64_t cnt = has_mips ? ((int64_t(4) << (2 * k)) - 1) / 3 : (int64_t(1) << (2 * k));
        cnt = (cnt + 15) / 16 * 16;
        base_host_out[e] = off;
        off += cnt;
    }
    *total_texels_out = off;
    return ok();
}

htex_status htex_mesh_validate(const htex_mesh *mesh, int32_t *first_bad_host, void *stream)
{
    htex_status st = check_mesh(mesh);
    if (st) return st;
    if (!first_bad_host) return fail(HTEX_E_ARG, "first_bad_host is NULL");
    *first_bad_host = -1;
    if (mesh->H == 0) return ok();
    hipStream_t s = static_cast<hipStream_t>(stream);
    int32_t *ws = nullptr;
    const size_t words = (size_t)mesh->E + 2;
    hipError_t e = hipMalloc(&ws, words * sizeof(int32_t));
    if (e != hipSuccess) return from_hip(e, "hipMalloc");
    int32_t init[2] = {INT32_MAX, 0};
    e = hipMemsetAsync(ws, 0, (size_t)mesh->E * sizeof(int32_t), s);
    if (e == hipSuccess) e = hipMemcpyAsync(ws + mesh->E, init, sizeof init, hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = htex::launch_validate(*mesh, ws, ws + mesh->E, s);
    int32_t res[2] = {0, 0};
    if (e == hipSuccess) e = hipMemcpyAsync(res, ws + mesh->E, sizeof res, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    (void)hipFree(ws);
    if (e != hipSuccess) return from_hip(e, "mesh validation");
    if (res[0] != INT32_MAX) {
        *first_bad_host = res[0];
        return fail(HTEX_E_TOPOLOGY, "halfedge %d violates an invariant", res[0]);
    }
    if (res[1] != 0) return fail(HTEX_E_TOPOLOGY, "%d edge ids are unused", res[1]);
    return ok();
}

htex_status htex_build_mips(const htex_pool *pool, void *texels_rw, void *stream)
{
    htex_status st = check_pool(pool, nullptr);
    if (st) return st;
    if (pool->dtype != HTEX_F32) return fail(HTEX_E_UNSUPPORTED, "mips are built on float32 pools");
    if (!pool->has_mips) return fail(HTEX_E_ARG, "pool has no mip levels");
    if (texels_rw != pool->texels) return fail(HTEX_E_ARG, "texels_rw must be pool->texels");
    return from_hip(htex::launch_build_mips(static_cast<float *>(texels_rw), pool->log2res,
                                            pool->base, pool->E, pool->max_log2res,
                                            pool->channels, static_cast<hipStream_t>(stream)),
                    "mip build");
}

htex_status htex_triangle_vertices(const htex_mesh *mesh, const int32_t *vert, int32_t V,
                                   const float *positions, float *out, int32_t *err_count,
                                   void *stream)
{
    htex_status st = check_mesh(mesh);
    if (st) return st;
    if (V < 0) return fail(HTEX_E_ARG, "negative V");
    if (mesh->H > 0 && (!vert || !positions || !out))
        return fail(HTEX_E_ARG, "vert, positions and out must be non-NULL");
    if (mesh->H > 0 && V == 0) return fail(HTEX_E_ARG, "a mesh with halfedges needs vertices");
    if (!aligned(vert, 4) || !aligned(positions, 4) || !aligned(out, 4))
        return fail(HTEX_E_ARG, "arrays must be 4-byte aligned");
    return from_hip(htex::launch_triangle_vertices(*mesh, vert, V, positions, out, err_count,
                                                   static_cast<hipStream_t>(stream)),
                    "triangle vertices");
}

htex_status htex_mip_backward(const htex_pool *pool, float *dtexels, int32_t clear_coarse,
                              void *stream)
{
    htex_status st = check_pool(pool, nullptr);
    if (st) return st;
    if (!pool->has_mips) return fail(HTEX_E_ARG, "pool has no mip levels");
    if (clear_coarse != 0 && clear_coarse != 1) return fail(HTEX_E_ARG, "clear_coarse must be 0 or 1");
    if (pool->total_texels > 0 && (!dtexels || !aligned(dtexels, 4 * (size_t)pool->channels)))
        return fail(HTEX_E_ARG, "dtexels must be non-NULL and %d-byte aligned",
                    4 * pool->channels);
    return from_hip(htex::launch_mip_backward(dtexels, pool->log2res, pool->base, pool->E,
                                              pool->max_log2res, pool->channels, clear_coarse,
                                              static_cast<hipStream_t>(stream)),
                    "mip backward");
}

htex_status htex_corner_average(const htex_mesh *mesh, const htex_pool *pool, void *texels_rw,
                                int32_t *err_count, void *stream)
{
    htex_status st = check_mesh(mesh);
    if (!st) st = check_pool(pool, mesh);
    if (st) return st;
    if (pool->dtype != HTEX_F32)
        return fail(HTEX_E_UNSUPPORTED, "corners are averaged on float32 pools");
    if (texels_rw != pool->texels) return fail(HTEX_E_ARG, "texels_rw must be pool->texels");
    return from_hip(htex::launch_corner_average(*mesh, static_cast<float *>(texels_rw),
                                                pool->log2res, pool->base, pool->channels,
                                                pool->has_mips,
                                                pool->max_log2res, err_count,
                                                static_cast<hipStream_t>(stream)),
                    "corner average");
}

htex_status htex_quantize(const htex_pool *src, int32_t dtype, void *dst, float *scale_out,
                          void *stream)
{
    htex_status st = check_pool(src, nullptr);
    if (st) return st;
    if (src->dtype != HTEX_F32) return fail(HTEX_E_ARG, "quantize reads a float32 pool");
    if (!dst && src->total_texels > 0) return fail(HTEX_E_ARG, "dst is NULL");
    hipStream_t s = static_cast<hipStream_t>(stream);
    const int C = src->channels;
    if (dtype == HTEX_BF16) {
        if (!aligned(dst, texel_bytes(HTEX_BF16, C)))
            return fail(HTEX_E_ARG, "dst must be %zu-byte aligned", texel_bytes(HTEX_BF16, C));
        return from_hip(htex::launch_quantize_bf16(static_cast<const float *>(src->texels),
                                                   static_cast<uint16_t *>(dst),
                                                   src->total_texels * C, s),
                        "bf16 quantize");
    }
    if (dtype == HTEX_FP8_E4M3) {
        if (!aligned(dst, texel_bytes(HTEX_FP8_E4M3, C)))
            return fail(HTEX_E_ARG, "dst must be %zu-byte aligned", texel_bytes(HTEX_FP8_E4M3, C));
        if (!scale_out && src->E > 0) return fail(HTEX_E_ARG, "scale_out is NULL");
        return from_hip(htex::launch_quantize_fp8(static_cast<const float *>(src->texels),
                                                  static_cast<uint8_t *>(dst), scale_out,
                                                  src->log2res, src->base, src->E,
                                                  src->has_mips, C, src->total_texels, s),
                        "fp8 quantize");
    }
    return fail(HTEX_E_ARG, "quantize target must be HTEX_BF16 or HTEX_FP8_E4M3");
}

htex_status htex_sample(const htex_mesh *mesh, const htex_pool *pool, const htex_queries *queries,
                        int32_t filter, uint32_t flags, float *out, htex_debug_rec *debug,
                        int32_t *err_count, void *stream)
{
    htex_status st = check_mesh(mesh);
    if (!st) st = check_pool(pool, mesh);
    if (!st) st = check_queries(queries, filter);
    if (st) return st;
    if (const htex_status fs = check_flags(flags)) return fs;
    if (filter == HTEX_TRILINEAR && !pool->has_mips)
        return fail(HTEX_E_ARG, "trilinear filtering needs a pool with mips");
    const size_t row = 4 * (size_t)pool->channels;   // bytes of one result row
    if (queries->Q > 0 && (!out || !aligned(out, row)))
        return fail(HTEX_E_ARG, "out must be non-NULL and %zu-byte aligned", row);
    if (debug && !aligned(debug, 4)) return fail(HTEX_E_ARG, "debug must be 4-byte aligned");
    if (queries->Q > 0 && mesh->H == 0) return fail(HTEX_E_ARG, "queries on an empty mesh");
    htex::SampleArgs a = make_args(mesh, pool, queries);
    a.out = out;
    a.dbg = debug;
    a.err = err_count;
    return from_hip(htex::launch_sample(a, pool->dtype, filter, static_cast<hipStream_t>(stream)),
                    "sample launch");
}

htex_status htex_sample_backward(const htex_mesh *mesh, const htex_pool *pool,
                                 const htex_queries *queries, int32_t filter, uint32_t flags,
                                 const float *dout, float *dtexels, void *stream)
{
    htex_status st = check_mesh(mesh);
    if (!st) st = check_pool(pool, mesh);
    if (!st) st = check_queries(queries, filter);
    if (st) return st;
    if (const htex_status fs = check_flags(flags)) return fs;
    if (pool->dtype != HTEX_F32) return fail(HTEX_E_UNSUPPORTED, "gradients need a float32 pool");
    if (filter == HTEX_TRILINEAR && !pool->has_mips)
        return fail(HTEX_E_ARG, "trilinear filtering needs a pool with mips");
    const size_t row = 4 * (size_t)pool->channels;
    if (queries->Q > 0) {
        if (!dout || !aligned(dout, row))
            return fail(HTEX_E_ARG, "dout must be %zu-byte aligned", row);
        if (!dtexels || !aligned(dtexels, row))
            return fail(HTEX_E_ARG, "dtexels must be %zu-byte aligned", row);
        if (mesh->H == 0) return fail(HTEX_E_ARG, "queries on an empty mesh");
    }
    htex::SampleArgs a = make_args(mesh, pool, queries);
    a.dout = dout;
    a.dtex = dtexels;
    // the LDS tile cache keys (edge, level) as edge * 16 + level in an int32
    if (mesh->E >= (1 << 27)) flags &= ~HTEX_QUERIES_SORTED;
    return from_hip(htex::launch_backward(a, filter, flags, pool->max_log2res,
                                          static_cast<hipStream_t>(stream)),
                    "backward launch");
}

size_t htex_sort_workspace_bytes(int32_t H, int64_t Q)
{
    return htex::sort_workspace_bytes(H < 0 ? 0 : H, Q < 0 ? 0 : Q);
}

namespace {

// Whether [a, a + an) and [b, b + bn) (bytes) overlap; NULL ranges never do.
bool overlap(const void *a, size_t an, const void *b, size_t bn)
{
    if (!a || !b) return false;
    const uintptr_t x = reinterpret_cast<uintptr_t>(a), y = reinterpret_cast<uintptr_t>(b);
    return x < y + bn && y < x + an;
}

htex_status check_sort(int32_t H, int64_t Q, const void *ws, size_t ws_bytes)
{
    if (H < 0 || Q < 0) return fail(HTEX_E_ARG, "negative size");
    if (Q >= (int64_t(1) << 31)) return fail(HTEX_E_RANGE, "sorting needs Q < 2^31");
    if (Q > 0) {
        if (!ws) return fail(HTEX_E_ARG, "workspace is NULL");
        if (!aligned(ws, 256)) return fail(HTEX_E_ARG, "workspace must be 256-byte aligned");
        const size_t need = htex::sort_workspace_bytes(H, Q);
        if (ws_bytes < need)
            return fail(HTEX_E_ARG, "workspace of %zu bytes is smaller than the %zu needed",
                        ws_bytes, need);
    }
    return HTEX_OK;
}

// The sorted batch must not overlap the batch it comes from or the
// workspace (the radix passes scatter; they cannot run in place).
htex_status check_sort_batch(const htex_queries *in, const int32_t *perm, const int32_t *h_out,
                             const float *u_out, const float *v_out, const float *f_out,
                             const void *ws, size_t ws_bytes)
{
    if (!in) return fail(HTEX_E_ARG, "queries is NULL");
    if (in->Q == 0) return HTEX_OK;
    if (!in->h || !in->u || !in->v || !perm || !h_out || !u_out || !v_out)
        return fail(HTEX_E_ARG, "NULL argument");
    if (in->footprint && !f_out) return fail(HTEX_E_ARG, "f_out is NULL");
    const size_t n = 4 * (size_t)in->Q;
    const void *outs[5] = {perm, h_out, u_out, v_out, in->footprint ? f_out : nullptr};
    const void *ins[4] = {in->h, in->u, in->v, in->footprint};
    for (int i = 0; i < 5; ++i) {
        if (outs[i] && !aligned(outs[i], 4)) return fail(HTEX_E_ARG, "outputs must be 4-byte aligned");
        for (int j = 0; j < 4; ++j)
            if (overlap(outs[i], n, ins[j], n))
                return fail(HTEX_E_ARG, "sorted outputs must not overlap the input batch");
        for (int j = i + 1; j < 5; ++j)
            if (overlap(outs[i], n, outs[j], n))
                return fail(HTEX_E_ARG, "sorted outputs must not overlap each other");
        if (overlap(outs[i], n, ws, ws_bytes))
            return fail(HTEX_E_ARG, "sorted outputs must not overlap the workspace");
    }
    return HTEX_OK;
}

}  // namespace

htex_status htex_sort_queries(int32_t H, int64_t Q, const int32_t *h, int32_t *perm, void *ws,
                              size_t ws_bytes, void *stream)
{
    if (htex_status st = check_sort(H, Q, ws, ws_bytes)) return st;
    if (Q == 0) return ok();
    if (!h || !perm) return fail(HTEX_E_ARG, "NULL argument");
    if (overlap(perm, 4 * (size_t)Q, ws, ws_bytes))
        return fail(HTEX_E_ARG, "perm must not overlap the workspace");
    return from_hip(htex::launch_sort(H, nullptr, 0, Q, h, nullptr, nullptr, nullptr, perm, nullptr,
                                      nullptr, nullptr, nullptr, nullptr, ws,
                                      static_cast<hipStream_t>(stream)),
                    "sort launch");
}

htex_status htex_sort_batch(int32_t H, const htex_queries *in, int32_t *perm, int32_t *h_out,
                            float *u_out, float *v_out, float *f_out, void *ws, size_t ws_bytes,
                            void *stream)
{
    if (!in) return fail(HTEX_E_ARG, "queries is NULL");
    if (htex_status st = check_sort(H, in->Q, ws, ws_bytes)) return st;
    if (htex_status st = check_sort_batch(in, perm, h_out, u_out, v_out, f_out, ws, ws_bytes))
        return st;
    if (in->Q == 0) return ok();
    return from_hip(htex::launch_sort(H, nullptr, 0, in->Q, in->h, in->u, in->v, in->footprint, perm, h_out,
                                      u_out, v_out, in->footprint ? f_out : nullptr, nullptr, ws,
                                      static_cast<hipStream_t>(stream)),
                    "sort launch");
}

htex_status htex_sort_batch_by_key(int32_t H, int32_t nkeys, const int32_t *key_of_h,
                                   const htex_queries *in, int32_t *perm, int32_t *h_out,
                                   float *u_out, float *v_out, float *f_out, void *ws,
                                   size_t ws_bytes, void *stream)
{
    if (!in) return fail(HTEX_E_ARG, "queries is NULL");
    if (H < 0) return fail(HTEX_E_ARG, "negative size");
    if (nkeys < 1) return fail(HTEX_E_ARG, "nkeys must be positive, got %d", nkeys);
    if (htex_status st = check_sort(nkeys, in->Q, ws, ws_bytes)) return st;
    if (htex_status st = check_sort_batch(in, perm, h_out, u_out, v_out, f_out, ws, ws_bytes))
        return st;
    if (in->Q == 0) return ok();
    if (H > 0) {
        if (!key_of_h || !aligned(key_of_h, 4))
            return fail(HTEX_E_ARG, "key_of_h must be non-NULL and 4-byte aligned");
        const size_t n = 4 * (size_t)in->Q, nk = 4 * (size_t)H;
        const void *outs[5] = {perm, h_out, u_out, v_out, in->footprint ? f_out : nullptr};
        for (const void *o : outs)
            if (overlap(o, n, key_of_h, nk))
                return fail(HTEX_E_ARG, "sorted outputs must not overlap key_of_h");
    }
    return from_hip(htex::launch_sort(H, key_of_h, nkeys, in->Q, in->h, in->u, in->v,
                                      in->footprint, perm, h_out, u_out, v_out,
                                      in->footprint ? f_out : nullptr, nullptr, ws,
                                      static_cast<hipStream_t>(stream)),
                    "sort launch");
}

htex_status htex_sort_batch_noalloc(int32_t H, const htex_queries *in, int32_t *perm,
                                    int32_t *h_out, float *u_out, float *v_out, float *f_out,
                                    void *stream)
{
    if (!in) return fail(HTEX_E_ARG, "queries is NULL");
    if (H < 0 || in->Q < 0) return fail(HTEX_E_ARG, "negative size");
    if (in->Q > htex::kStaticSortMaxQ)
        return fail(HTEX_E_RANGE, "the allocation-free sort takes at most %lld queries, got %lld",
                    (long long)htex::kStaticSortMaxQ, (long long)in->Q);
    if (htex_status st = check_sort_batch(in, perm, h_out, u_out, v_out, f_out, nullptr, 0))
        return st;
    if (in->Q == 0) return ok();
    void *ws = nullptr;
    hipError_t e = htex::static_sort_scratch(&ws);
    if (e != hipSuccess) return from_hip(e, "sort scratch lookup");
    const size_t need = htex::sort_workspace_bytes(H, in->Q);
    if (need > htex::static_sort_scratch_bytes())
        return fail(HTEX_E_RANGE, "sort scratch of %zu bytes is smaller than the %zu needed",
                    htex::static_sort_scratch_bytes(), need);
    if (htex_status st = check_sort_batch(in, perm, h_out, u_out, v_out, f_out, ws, need))
        return st;
    return from_hip(htex::launch_sort(H, nullptr, 0, in->Q, in->h, in->u, in->v, in->footprint, perm, h_out,
                                      u_out, v_out, in->footprint ? f_out : nullptr, nullptr, ws,
                                      static_cast<hipStream_t>(stream)),
                    "sort launch");
}

htex_status htex_permute_queries(const htex_queries *in, const int32_t *perm, int32_t *h_out,
                                 float *u_out, float *v_out, float *f_out, void *stream)
{
    if (!in || in->Q < 0) return fail(HTEX_E_ARG, "bad queries");
    if (in->Q == 0) return ok();
    if (!in->h || !in->u || !in->v || !perm || !h_out || !u_out || !v_out)
        return fail(HTEX_E_ARG, "NULL argument");
    if (in->footprint && !f_out) return fail(HTEX_E_ARG, "f_out is NULL");
    return from_hip(htex::launch_gather_queries(perm, in->Q, in->h, in->u, in->v, in->footprint,
                                                h_out, u_out, v_out,
                                                in->footprint ? f_out : nullptr,
                                                static_cast<hipStream_t>(stream)),
                    "permute launch");
}

htex_status htex_unpermute_results(int64_t Q, int32_t channels, const int32_t *perm,
                                   const float *in, float *out, void *stream)
{
    if (Q < 0) return fail(HTEX_E_ARG, "negative Q");
    if (channels != 1 && channels != 4) return fail(HTEX_E_ARG, "channels must be 1 or 4");
    if (Q == 0) return ok();
    const size_t row = 4 * (size_t)channels;
    if (!perm || !in || !out || !aligned(in, row) || !aligned(out, row))
        return fail(HTEX_E_ARG, "in/out must be non-NULL and %zu-byte aligned", row);
    if (overlap(in, row * (size_t)Q, out, row * (size_t)Q))
        return fail(HTEX_E_ARG, "in and out must not overlap");
    return from_hip(htex::launch_unpermute(perm, Q, channels, in, out,
                                           static_cast<hipStream_t>(stream)),
                    "unpermute launch");
}

htex_status htex_prepare(const htex_mesh *mesh, const htex_pool *pool, void *prep, void *stream)
{
    htex_status st = check_mesh(mesh);
    if (!st) st = check_pool(pool, mesh);
    if (st) return st;
    if (pool->total_texels >= (int64_t(1) << 40))
        return fail(HTEX_E_RANGE, "prepared records address pools below 2^40 texels");
    if (mesh->H > 0 && (!prep || !aligned(prep, 16)))
        return fail(HTEX_E_ARG, "prep must be non-NULL and 16-byte aligned");
    htex_queries none{};
    htex::SampleArgs a = make_args(mesh, pool, &none);
    return from_hip(htex::launch_prepare(a, prep, static_cast<hipStream_t>(stream)), "prepare launch");
}

namespace {

// Checks and launch arguments shared by the prepared sampling entry points.
htex_status prepared_args(int32_t H, const void *prep, const htex_pool *pool,
                          const htex_queries *queries, int32_t filter, uint32_t flags,
                          float *out, int32_t *err_count, htex::SampleArgs *a)
{
    htex_status st = check_pool(pool, nullptr);
    if (!st) st = check_queries(queries, filter);
    if (st) return st;
    if (H < 0) return fail(HTEX_E_ARG, "negative H");
    if (const htex_status fs = check_flags(flags)) return fs;
    if (filter == HTEX_TRILINEAR && !pool->has_mips)
        return fail(HTEX_E_ARG, "trilinear filtering needs a pool with mips");
    if (queries->Q > 0) {
        if (H == 0) return fail(HTEX_E_ARG, "queries on an empty mesh");
        if (!prep || !aligned(prep, 16)) return fail(HTEX_E_ARG, "prep must be 16-byte aligned");
        if (!out || !aligned(out, 4 * (size_t)pool->channels))
            return fail(HTEX_E_ARG, "out must be %d-byte aligned", 4 * pool->channels);
    }
    *a = htex::SampleArgs{};
    a->H = H;
    a->channels = pool->channels;
    a->texels = pool->texels;
    a->scale = pool->scale;
    a->has_mips = pool->has_mips;
    a->total_texels = pool->total_texels;
    a->Q = queries->Q;
    a->qh = queries->h;
    a->qu = queries->u;
    a->qv = queries->v;
    a->qf = queries->footprint;
    a->out = out;
    a->err = err_count;
    a->prep = prep;
    return HTEX_OK;
}

htex_status launch_prepared(const htex::SampleArgs &a, const htex_pool *pool, int32_t filter,
                            uint32_t flags, void *stream)
{
    // a pool that fits the 256 MB fabric-side cache leaves the sampler
    // bound by the VALU rather than by memory
    const bool resident = pool->total_texels * (int64_t)texel_bytes(pool->dtype, pool->channels) <=
                          (int64_t(256) << 20);
    return from_hip(htex::launch_sample_prepared(a, pool->dtype, filter,
                                                 (flags & HTEX_QUERIES_SCATTERED) != 0, resident,
                                                 static_cast<hipStream_t>(stream)),
                    "prepared sample launch");
}

}  // namespace

htex_status htex_sample_prepared(int32_t H, const void *prep, const htex_pool *pool,
                                 const htex_queries *queries, int32_t filter, uint32_t flags,
                                 float *out, int32_t *err_count, void *stream)
{
    htex::SampleArgs a;
    if (htex_status st = prepared_args(H, prep, pool, queries, filter, flags, out, err_count, &a))
        return st;
    return launch_prepared(a, pool, filter, flags, stream);
}

namespace {

size_t round256(size_t x) { return (x + 255) / 256 * 256; }

// Workspace of htex_sample_prepared_reordered: the permutation, the query
// records in input order, the results in sorted order, then the sort's own.
size_t reordered_ws_bytes(int32_t H, int64_t Q, int32_t channels)
{
    const size_t q = (size_t)(Q > 0 ? Q : 1);
    return round256(4 * q) + round256(16 * q) + round256(4 * (size_t)channels * q) +
           htex::sort_workspace_bytes(H, Q);
}

}  // namespace

size_t htex_sample_reordered_workspace_bytes(int32_t H, int64_t Q, int32_t channels)
{
    if (H < 0 || Q < 0 || (channels != 1 && channels != 4)) return 0;
    return reordered_ws_bytes(H, Q, channels);
}

htex_status htex_sample_prepared_reordered(int32_t H, const void *prep, const htex_pool *pool,
                                           const htex_queries *queries, int32_t filter,
                                           float *out, void *ws, size_t ws_bytes,
                                           int32_t *err_count, void *stream)
{
    htex::SampleArgs a;
    if (htex_status st = prepared_args(H, prep, pool, queries, filter, 0, out, err_count, &a))
        return st;
    const int64_t Q = queries->Q;
    if (Q == 0) return ok();
    if (Q >= (int64_t(1) << 31)) return fail(HTEX_E_RANGE, "reordering needs Q < 2^31");
    const size_t need = reordered_ws_bytes(H, Q, pool->channels);
    if (!ws || !aligned(ws, 256)) return fail(HTEX_E_ARG, "workspace must be 256-byte aligned");
    if (ws_bytes < need)
        return fail(HTEX_E_ARG, "workspace of %zu bytes is smaller than the %zu needed", ws_bytes,
                    need);
    const size_t n = 4 * (size_t)Q, rows = 4 * (size_t)pool->channels * (size_t)Q;
    if (overlap(out, rows, ws, ws_bytes)) return fail(HTEX_E_ARG, "out must not overlap the workspace");
    const void *ins[4] = {queries->h, queries->u, queries->v, queries->footprint};
    for (const void *in : ins)
        if (overlap(in, n, ws, ws_bytes))
            return fail(HTEX_E_ARG, "the queries must not overlap the workspace");
    char *p = static_cast<char *>(ws);
    int32_t *perm = reinterpret_cast<int32_t *>(p);
    p += round256(n);
    void *records = p;
    p += round256(16 * (size_t)Q);
    float *sorted_out = reinterpret_cast<float *>(p);
    p += round256(rows);
    const hipStream_t s = static_cast<hipStream_t>(stream);
    // 1. the permutation to halfedge order, and the queries as records
    if (const htex_status st = from_hip(
            htex::launch_sort(H, nullptr, 0, Q, queries->h, queries->u, queries->v,
                              queries->footprint, perm, nullptr, nullptr, nullptr, nullptr,
                              records, p, s),
            "sort launch"))
        return st;
    // 2. the batch sampled in halfedge order, each lane reading its query's
    // record through the permutation
    a.order = perm;
    a.qrec = records;
    a.out = sorted_out;
    if (const htex_status st = launch_prepared(a, pool, filter, 0, stream)) return st;
    // 3. the results back in input order
    return from_hip(htex::launch_unpermute(perm, Q, pool->channels, sorted_out, out, s),
                    "unpermute launch");
}

namespace {

htex_status check_aniso(const htex_pool *pool, const htex_queries *q, const float *jac,
                        int32_t max_aniso, uint32_t flags, const float *out)
{
    htex_status st = check_queries(q, HTEX_BILINEAR);
    if (st) return st;
    if (const htex_status fs = check_flags(flags)) return fs;
    if (!pool->has_mips) return fail(HTEX_E_ARG, "anisotropic filtering needs a pool with mips");
    if (max_aniso < 1 || max_aniso > HTEX_MAX_ANISO)
        return fail(HTEX_E_ARG, "max_aniso %d outside [1, %d]", max_aniso, HTEX_MAX_ANISO);
    if (q->Q > 0) {
        if (!jac || !aligned(jac, 16)) return fail(HTEX_E_ARG, "jac must be 16-byte aligned");
        if (!out || !aligned(out, 4 * (size_t)pool->channels))
            return fail(HTEX_E_ARG, "out must be %d-byte aligned", 4 * pool->channels);
    }
    return HTEX_OK;
}

}  // namespace

htex_status htex_sample_aniso(const htex_mesh *mesh, const htex_pool *pool,
                              const htex_queries *queries, const float *jac, int32_t max_aniso,
                              uint32_t flags, float *out, int32_t *nprobe, int32_t *err_count,
                              void *stream)
{
    htex_status st = check_mesh(mesh);
    if (!st) st = check_pool(pool, mesh);
    if (st) return st;
    if (!queries) return fail(HTEX_E_ARG, "queries is NULL");
    st = check_aniso(pool, queries, jac, max_aniso, flags, out);
    if (st) return st;
    if (nprobe && !aligned(nprobe, 4)) return fail(HTEX_E_ARG, "nprobe must be 4-byte aligned");
    if (queries->Q > 0 && mesh->H == 0) return fail(HTEX_E_ARG, "queries on an empty mesh");
    htex::SampleArgs a = make_args(mesh, pool, queries);
    a.qf = nullptr;
    a.out = out;
    a.err = err_count;
    return from_hip(htex::launch_sample_aniso(a, pool->dtype, jac, max_aniso, nprobe,
                                              static_cast<hipStream_t>(stream)),
                    "anisotropic sample launch");
}

htex_status htex_sample_aniso_prepared(int32_t H, const void *prep, const htex_pool *pool,
                                       const htex_queries *queries, const float *jac,
                                       int32_t max_aniso, uint32_t flags, float *out,
                                       int32_t *err_count, void *stream)
{
    htex_status st = check_pool(pool, nullptr);
    if (st) return st;
    if (!queries) return fail(HTEX_E_ARG, "queries is NULL");
    st = check_aniso(pool, queries, jac, max_aniso, flags, out);
    if (st) return st;
    if (H < 0) return fail(HTEX_E_ARG, "negative H");
    if (queries->Q > 0) {
        if (H == 0) return fail(HTEX_E_ARG, "queries on an empty mesh");
        if (!prep || !aligned(prep, 16)) return fail(HTEX_E_ARG, "prep must be 16-byte aligned");
    }
    htex::SampleArgs a{};
    a.H = H;
    a.channels = pool->channels;
    a.texels = pool->texels;
    a.scale = pool->scale;
    a.has_mips = pool->has_mips;
    a.total_texels = pool->total_texels;
    a.Q = queries->Q;
    a.qh = queries->h;
    a.qu = queries->u;
    a.qv = queries->v;
    a.out = out;
    a.err = err_count;
    a.prep = prep;
    return from_hip(htex::launch_sample_aniso(a, pool->dtype, jac, max_aniso, nullptr,
                                              static_cast<hipStream_t>(stream)),
                    "prepared anisotropic sample launch");
}

}  // extern "C"
