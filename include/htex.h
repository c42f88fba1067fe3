/*
 * htex.h -- C ABI of the MI355X Htex sampling library (libhtex.so).
 *
 * Htex (Barbier & Dupuy 2022) textures a polygon mesh with one square texture
 * per edge: the edge's halfedge/twin pair forms an intrinsic quad (Section
 * 3.2; a boundary halfedge pairs with itself).  A query names a halfedge h and
 * a barycentric point (u, v) of h's intrinsic triangle (Section 4.2); its
 * value is Alg. 3 (Section 4.4): three filtered fetches -- the quad of
 * Edge(h) at TriangleToQuadUV(h, (u, v)), the quad of Edge(Next h) at
 * TriangleToQuadUV(Next h, (v, -u)) and the quad of Edge(Prev h) at
 * TriangleToQuadUV(Prev h, (-v, u)) -- each read with a CLAMP_TO_BORDER
 * sampler of border 0 together with a border-normalization channel of ones,
 * summed, and divided by the summed normalization channel.  TriangleToQuadUV
 * (Alg. 2) keeps (u, v) when h > Twin(h) and returns (1-u, 1-v) otherwise.
 *
 * Conventions used throughout (the paper leaves them to the GPU's texture
 * unit; these are the OpenGL ones):
 *   - texture of edge e: n = 2^k texels per side, k = log2res[e] in [0, 15];
 *     the quad coordinate x in [0, 1] indexes columns i, y indexes rows j;
 *     texel (i, j) is centred at ((i + 1/2)/n, (j + 1/2)/n);
 *   - bilinear filtering of a point (x, y): taps (i0 + di, j0 + dj),
 *     i0 = floor(x n - 1/2), j0 = floor(y n - 1/2), weights (1-a or a)(1-b or b)
 *     with a = x n - 1/2 - i0, b = y n - 1/2 - j0; taps outside [0, n)^2 read
 *     the zero border and add nothing to the normalization channel either;
 *   - trilinear filtering (LINEAR_MIPMAP_LINEAR) with an isotropic footprint
 *     f (quad units, one per query): lambda = log2(f n); lambda <= 0 reads
 *     level 0, lambda >= k reads level k, otherwise levels floor(lambda) and
 *     floor(lambda) + 1 blended by lambda - floor(lambda).  f <= 0, NaN or
 *     subnormal reads level 0; f = +inf reads level k;
 *   - the normalization channel is computed (sum of in-bounds tap weights),
 *     never stored.
 *
 * Memory: every pointer inside htex_mesh / htex_pool / htex_queries and every
 * output pointer is DEVICE memory owned by the caller; the structs themselves
 * and pointers documented as "host" are host memory, read during the call
 * only.  The sampling entry points allocate nothing.  All launches are
 * asynchronous on `stream` (a hipStream_t; NULL = the null stream).
 *
 * Errors: arguments are checked on the host before anything is launched; a
 * failed check returns a negative status, launches nothing and records a
 * message readable with htex_last_error() (thread-local).  Per-query problems
 * (h outside [0, H), non-finite u or v) do not abort the call: that query's
 * output row is NaN and *err_count (if given) is incremented on the device.
 * A launch failure returns HTEX_E_DEVICE.
 */
#ifndef HTEX_H
#define HTEX_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t htex_status;

#define HTEX_OK 0
#define HTEX_E_ARG (-1)          /* bad argument: NULL, size, enum, alignment */
#define HTEX_E_TOPOLOGY (-2)     /* halfedge arrays violate an invariant      */
#define HTEX_E_RANGE (-3)        /* a size exceeds what the library supports  */
#define HTEX_E_DEVICE (-4)       /* a HIP call or kernel launch failed        */
#define HTEX_E_UNSUPPORTED (-5)  /* valid request the library does not serve  */
#define HTEX_E_BUSY (-6)         /* resource in use (serving)                 */
#define HTEX_E_NOMEM (-7)        /* memory budget exhausted (serving)         */

/* texel storage, per channel (a texel holds 4 channels, RGBA, or 1, e.g. a
 * displacement map) */
#define HTEX_F32 0        /* float32: 16 bytes per RGBA texel, 4 per scalar     */
#define HTEX_BF16 1       /* bfloat16: 8 bytes per RGBA texel, 2 per scalar     */
#define HTEX_FP8_E4M3 2   /* OCP E4M3 (no infinities, max 448): 4 bytes per    */
                          /* RGBA texel, 1 per scalar, times a float32 scale   */
                          /* per edge                                          */
/* filters */
#define HTEX_BILINEAR 0
#define HTEX_TRILINEAR 1
/* flags */
#define HTEX_QUERIES_SORTED (1u << 0)    /* hint: queries arrive ordered by h */
#define HTEX_QUERIES_SCATTERED (1u << 1) /* hint: neighbouring queries share  */
                                         /* no texels (random order); not    */
                                         /* together with _SORTED            */

/* Halfedge arrays (Section 2, Fig. 2), device, int32 [H] each.  Twin(h) = -1
 * marks a boundary halfedge; Edge(h) in [0, E) names h's quad and texture.
 * The sampler trusts these arrays; check them once with htex_mesh_validate. */
typedef struct htex_mesh {
    int32_t H, E;
    const int32_t *twin, *next, *prev, *edge;
} htex_mesh;

/* Per-edge texel pool.  Edge e's texels start at texel index base[e] (a
 * multiple of 16); its levels follow each other from level 0 (n x n) down to
 * level k (1 x 1) when has_mips, level 0 only otherwise; each level is
 * row-major (texel (i, j) at j * n + i), `channels` values per texel.  Level
 * l of an edge of log2 resolution k starts (4^(k+1) - 4^(k+1-l)) / 3 texels
 * after base[e].  htex_pool_layout computes a valid base[] (host).
 * texels: aligned to one texel's bytes (16 / 8 / 4 for RGBA float32 / BF16 /
 * FP8; 4 / 2 / 1 for one channel).
 * scale: FP8 only, float32 [E], texel value = decoded code * scale[e].
 * Results (and gradients of results) have `channels` floats per query:
 * Alg. 3 filters every channel with the same weights and normalization. */
typedef struct htex_pool {
    int32_t E;
    int32_t dtype;         /* HTEX_F32 / HTEX_BF16 / HTEX_FP8_E4M3 */
    int32_t has_mips;      /* 0 or 1 */
    int32_t max_log2res;   /* max over log2res[] (host-known bound, <= 15) */
    int32_t channels;      /* 4 (RGBA) or 1 */
    int32_t reserved;      /* 0 */
    int64_t total_texels;  /* size of the pool in texels */
    const uint8_t *log2res;   /* [E] */
    const int64_t *base;      /* [E] */
    const void *texels;
    const float *scale;       /* [E] or NULL */
} htex_pool;

/* A batch of queries, device, SoA.  footprint may be NULL (bilinear only). */
typedef struct htex_queries {
    int64_t Q;
    const int32_t *h;
    const float *u, *v;
    const float *footprint;
} htex_queries;

/* Optional per-query trace of the three fetches (s = 0 own quad, 1 Next,
 * 2 Prev; slot l = first / second mip level).  Integer fields are exact:
 * level = -1 and i0 = j0 = inb = 0 for an unused slot; inb bit (2 dj + di) is
 * set for every in-bounds tap (whatever its weight); i0/j0 are exact while
 * |u|, |v| <= 4 (beyond, the coordinate is clamped to +-4 first, which only
 * moves taps that are out of bounds anyway).  An invalid query has next =
 * prev = edge = level = -1 and zeros elsewhere.  phi is the trilinear
 * fraction, W the summed normalization channel, wf the per-fetch channel. */
typedef struct htex_debug_rec {
    int32_t next, prev;
    int32_t edge[3];
    int32_t flip[3];
    int32_t level[3][2];
    int32_t i0[3][2];
    int32_t j0[3][2];
    int32_t inb[3][2];
    float phi;
    float W;
    float wf[3];
    int32_t pad[3];
} htex_debug_rec; /* 160 bytes */

/* Message of the last failed call on this thread ("" if none). */
const char *htex_last_error(void);
const char *htex_status_string(htex_status s);

/* Host only.  Fills base_host_out[E] with texel offsets for the pool format
 * above (each edge padded to a multiple of 16 texels) and *total_texels_out
 * with the pool size.  log2res_host[E] must hold values in [0, 15]. */
htex_status htex_pool_layout(int32_t E, const uint8_t *log2res_host, int32_t has_mips,
                             int64_t *base_host_out, int64_t *total_texels_out);

/* Checks the halfedge invariants of Section 2 on the device and waits for the
 * result: Twin is an involution without fixed points where it is >= 0; Next
 * and Prev are inverse permutations; twins share their edge; every edge id in
 * [0, E) is used by exactly one twin pair or one lone boundary halfedge; every
 * face has at least 3 sides.  Returns HTEX_OK, or HTEX_E_TOPOLOGY with the
 * smallest offending halfedge in *first_bad_host (-1 for an unused edge id).
 * Allocates a small temporary device buffer (not for use under graph
 * capture). */
htex_status htex_mesh_validate(const htex_mesh *mesh, int32_t *first_bad_host,
                               void *stream);

/* Box-filtered mip chain, in place: for every edge and l = 1..k, texel (i, j)
 * of level l becomes the mean of texels (2i..2i+1, 2j..2j+1) of level l-1,
 * in float32, channel by channel.  The pool must be HTEX_F32 with has_mips = 1; `texels_rw` is
 * the same memory as pool->texels, writable. */
htex_status htex_build_mips(const htex_pool *pool, void *texels_rw, void *stream);

/* Intrinsic triangle of every halfedge (Section 3.1, Alg. 1): out[h] =
 * (v0, v1, v2) as 9 floats, v0 = positions[Vert(Next h)], v2 =
 * positions[Vert(h)], v1 = the mean of the positions of the vertices of h's
 * face (found by following Next from h), summed in float32 with every
 * rounding error kept, from the face's smallest halfedge, and rounded once
 * (every triangle of a face gets the same v1 bit for bit).  Section 4.2's
 * frame: the query (h, u, v) is the point u v2 + v v0 + (1 - u - v) v1.
 * vert: device int32 [H] (the Vert operator, not part of htex_mesh since
 * sampling never needs it); positions: device float32 [V][3]; out: device
 * float32 [H][9].
 * A face ring longer than 65536 halfedges, a walk leaving [0, H) or a
 * vertex id outside [0, V) gives a NaN row and increments *err_count
 * (device, nullable). */
htex_status htex_triangle_vertices(const htex_mesh *mesh, const int32_t *vert, int32_t V,
                                   const float *positions, float *out, int32_t *err_count,
                                   void *stream);

/* Transpose of htex_build_mips, for training a pool whose coarser levels
 * are box means of level 0: in place on `dtexels` (float32, the pool's
 * layout and channels, aligned to 4 C bytes), from the coarsest level
 * down, each texel of level l adds a quarter of its gradient to each of the
 * four level-(l-1) texels it averages.  Level 0 then holds the gradient
 * with respect to level 0 through every level (what an optimizer of level
 * 0 needs); with clear_coarse = 1 the coarser levels are zeroed as they
 * are folded, otherwise each keeps its own gradient plus what came from
 * the levels above it.  Needs has_mips; the pool's texels are not read. */
htex_status htex_mip_backward(const htex_pool *pool, float *dtexels, int32_t clear_coarse,
                              void *stream);

/* Corner pre-processing (Section 4.4, "Corner Pre-processing"), in place on
 * a float32 pool: on every level of n >= 2 texels per side, the corner
 * texels that lie on one mesh vertex, or on one face centroid, all receive
 * the mean of their values (float32 sums with every rounding error kept,
 * rounded once);
 * levels of different edges are grouped by equal n.  With one resolution
 * everywhere, filtering is then continuous at vertices and face centroids
 * too (the seams are continuous already), which displacement needs to stay
 * crack-free; 1x1 levels (one texel = four corners) are left unchanged.
 * Corner texels of the quad of edge e, whose larger halfedge g keeps its
 * barycentric (u, v) as quad coordinates (Alg. 2): (n-1, 0) at Vert(g),
 * (0, n-1) at Vert(Next g), (0, 0) at the centroid of g's face, (n-1, n-1)
 * at the centroid of the twin's face -- or, for a boundary edge, the mirror
 * image of (0, 0), written with the same value.  Vertices and faces are
 * found from the halfedge operators alone (rings of Twin(Prev g) and of
 * Next), so the mesh must be valid; a ring longer than 65536 halfedges or
 * one that leaves [0, H) increments *err_count (device, nullable) and is
 * left unchanged.  Run it after htex_build_mips (rebuilding the mips would
 * undo it on the coarser levels) and before quantizing (BF16 keeps equal
 * values equal; FP8's per-edge scales do not).  `texels_rw` is the same
 * memory as pool->texels, writable. */
htex_status htex_corner_average(const htex_mesh *mesh, const htex_pool *pool, void *texels_rw,
                                int32_t *err_count, void *stream);

/* Converts a float32 pool to `dtype` into `dst` (same layout, same base[],
 * same channels, total_texels texels).  HTEX_BF16: round to nearest even.  HTEX_FP8_E4M3:
 * per-edge scale s = (max |T| over every level and channel of the edge) / 448
 * computed in float32 and written to scale_out[e]; code = E4M3 of the
 * float32 quotient T / s, rounded to nearest even and saturated to +-448; an
 * all-zero edge gets s = 0 and zero codes.  Padding texels are written as 0.
 * scale_out is required for FP8 and ignored otherwise. */
htex_status htex_quantize(const htex_pool *src_f32, int32_t dtype, void *dst,
                          float *scale_out, void *stream);

/* Alg. 3 for every query (Section 4.4) -> out[q][0..C) (float32, Q x C for
 * a pool of C channels, aligned to 4 C bytes).  filter: HTEX_BILINEAR (level 0, footprint ignored) or
 * HTEX_TRILINEAR (needs has_mips and a footprint array).  Colour is blended
 * and normalized in float32 whatever the storage type.  debug (nullable):
 * Q records.  err_count (nullable, device int32): incremented once per
 * invalid query.  Results do not depend on the batch they are computed in. */
htex_status htex_sample(const htex_mesh *mesh, const htex_pool *pool,
                        const htex_queries *queries, int32_t filter, uint32_t flags,
                        float *out, htex_debug_rec *debug, int32_t *err_count,
                        void *stream);

/* Transpose of htex_sample with respect to the texels: for every valid query
 * and every in-bounds tap it reads, dtexels[tap][c] += (om w / W) * dout[q][c]
 * (om: level weight, w: bilinear weight, W: the query's normalization).
 * dtexels is float32 with the pool's layout and channels (aligned to 4 C
 * bytes) and is added to, with float32 atomics (summation order
 * unspecified); the pool must be HTEX_F32.  dout is float32 Q x C (aligned
 * to 4 C bytes).  With HTEX_QUERIES_SORTED, each workgroup first sums its
 * consecutive queries' contributions to small textures (at most 32 x 32
 * RGBA or 64 x 64 one-channel texels per level) in on-chip memory and adds
 * each texel once (fewer, uncontended atomics). */
htex_status htex_sample_backward(const htex_mesh *mesh, const htex_pool *pool,
                                 const htex_queries *queries, int32_t filter,
                                 uint32_t flags, const float *dout, float *dtexels,
                                 void *stream);

/* --------------------------------------------------------- query order --
 * Optional step before sampling: the paper's fragments arrive from a
 * rasterizer in triangle order (Section 4.4, "Rendering"); a batch in any
 * other order can be put in halfedge order so that neighbouring queries read
 * the same textures.  Sampling results do not depend on the order. */

/* Bytes of device workspace htex_sort_queries and htex_sort_batch need for
 * Q queries on a mesh of H halfedges (htex_sort_batch_by_key: pass the
 * number of keys for H). */
size_t htex_sort_workspace_bytes(int32_t H, int64_t Q);

/* perm[0..Q) = the stable ordering of the queries by h (queries with h
 * outside [0, H) last, in input order).  h: device int32 [Q]; perm: device
 * int32 [Q]; ws: device workspace of at least htex_sort_workspace_bytes(H, Q)
 * bytes, 256-byte aligned, not overlapping perm; its contents on entry do
 * not matter.  Q < 2^31. */
htex_status htex_sort_queries(int32_t H, int64_t Q, const int32_t *h, int32_t *perm, void *ws,
                              size_t ws_bytes, void *stream);

/* The sorted batch itself in one call: perm as htex_sort_queries, and
 * h_out[i] = h[perm[i]], likewise u_out, v_out and f_out (f_out only when
 * `in` has footprints; it may be NULL otherwise).  The counting read copies
 * each query into a 16-byte record and the last radix pass gathers each
 * sorted row's record (one 16-byte read per query), so no separate gather
 * through perm follows.  Every
 * output is device int32/float32 [Q], 4-byte aligned, and must not overlap
 * the input arrays, each other or the workspace (HTEX_E_ARG otherwise).
 * ws as for htex_sort_queries.  Q < 2^31. */
htex_status htex_sort_batch(int32_t H, const htex_queries *in, int32_t *perm, int32_t *h_out,
                            float *u_out, float *v_out, float *f_out, void *ws, size_t ws_bytes,
                            void *stream);

/* htex_sort_batch ordered by a key per halfedge instead of the halfedge:
 * query i sorts by key_of_h[h_i] (device int32 [H], values 0 .. nkeys - 1),
 * stably; queries whose h lies outside [0, H), or whose key lies outside
 * [0, nkeys), sort last, in input order.  With key_of_h = the mesh's edge
 * array (nkeys = E) both halfedges of an edge -- the two triangles of one
 * intrinsic quad, which share its texture (Sections 3.2 and 4.1) -- are
 * sampled back to back, which a sorted-batch kernel turns into fewer texel
 * line fetches.  perm and the sorted arrays
 * as htex_sort_batch; they must not overlap key_of_h either.  ws: at least
 * htex_sort_workspace_bytes(nkeys, Q) bytes, 256-byte aligned.  nkeys >= 1;
 * Q < 2^31. */
htex_status htex_sort_batch_by_key(int32_t H, int32_t nkeys, const int32_t *key_of_h,
                                   const htex_queries *in, int32_t *perm, int32_t *h_out,
                                   float *u_out, float *v_out, float *f_out, void *ws,
                                   size_t ws_bytes, void *stream);

/* htex_sort_batch for callers that cannot allocate device memory (code
 * under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc): no workspace argument; the radix passes use a scratch array
 * compiled into the library instead.  Same outputs as htex_sort_batch, bit
 * for bit.  Calls no hipMalloc, hipFree or allocating library routine.
 * Limits: at most HTEX_SORT_NOALLOC_MAX_Q queries (HTEX_E_RANGE above); the
 * array takes HTEX_SORT_NOALLOC_SCRATCH_MIB MiB of device memory on every
 * GPU where the library's sort kernels are loaded, until the process ends.
 * Every call on one GPU uses that GPU's one array: calls that overlap in
 * time on one GPU (other streams, other threads) race and corrupt each
 * other's results, so serialize them (calls on one stream are ordered).
 * Nothing in the array needs clearing between calls (each call clears or
 * writes all it reads).  Arguments as for htex_sort_batch. */
#define HTEX_SORT_NOALLOC_MAX_Q (1 << 20)
#define HTEX_SORT_NOALLOC_SCRATCH_MIB 39
htex_status htex_sort_batch_noalloc(int32_t H, const htex_queries *in, int32_t *perm,
                                    int32_t *h_out, float *u_out, float *v_out, float *f_out,
                                    void *stream);

/* Sorted copy of a batch: h_out[i] = h[perm[i]], same for u, v and the
 * footprint (f_out may be NULL when the batch has none). */
htex_status htex_permute_queries(const htex_queries *in, const int32_t *perm, int32_t *h_out,
                                 float *u_out, float *v_out, float *f_out, void *stream);

/* Results back to input order: row perm[i] of out = row i of in (float32,
 * Q rows of `channels` (1 or 4) floats, both aligned to 4 channels bytes,
 * not overlapping).  perm must be a permutation of [0, Q). */
htex_status htex_unpermute_results(int64_t Q, int32_t channels, const int32_t *perm,
                                   const float *in, float *out, void *stream);

/* Prepared fetch descriptors: the halfedge navigation of Alg. 3 resolved
 * once per (mesh, pool) so that a query reads one record instead of walking
 * Next/Prev/Twin/Edge and the edge table.  Record h (HTEX_PREP_BYTES bytes,
 * 16-byte aligned, layout private to the library) holds, for each of the
 * three fetches of halfedge h (own quad, Next(h), Prev(h)), the edge, the texture
 * base, its log2 resolution and the reflection bit of Alg. 2, plus Next(h)
 * and Prev(h).  It depends on the mesh and on the pool's log2res/base (not
 * on the texels: a quantized copy with the same layout shares it); rebuild
 * it when either changes.  Requires total_texels < 2^40. */
#define HTEX_PREP_BYTES 48

/* Writes H descriptor records to `prep` (device, caller-allocated, H *
 * HTEX_PREP_BYTES bytes, 16-byte aligned).  Trusts the mesh (validate it
 * first). */
htex_status htex_prepare(const htex_mesh *mesh, const htex_pool *pool, void *prep,
                         void *stream);

/* Same result as htex_sample (bit for bit) from prepared descriptors: the
 * fast path for repeated sampling of one mesh.  `H` is the number of
 * halfedges the records cover (queries with h outside [0, H) are invalid as
 * in htex_sample); the records buffer must hold H records.  A record whose
 * fetches would read past pool->total_texels (records prepared for another
 * pool layout) makes its query invalid (NaN row, *err_count incremented)
 * instead of reading outside the pool.  No debug trace.  The HTEX_QUERIES_SCATTERED hint picks
 * the kernel: by default every tap of a sampled level is read, which suits
 * coherent batches (ordered by halfedge, or rasterized, where neighbouring
 * queries share the cache lines); with the hint only in-bounds taps are
 * read, which saves line fetches when no two queries share texels.  Without
 * the hint, BF16 and FP8 pools and pools of at most 256 MB (which stay in
 * the caches, so the launch is bound by arithmetic rather than memory) take
 * a variant that deals the Next and Prev fetches out across the
 * wavefront.  Every kernel gives the same results. */
htex_status htex_sample_prepared(int32_t H, const void *prep, const htex_pool *pool,
                                 const htex_queries *queries, int32_t filter,
                                 uint32_t flags, float *out, int32_t *err_count,
                                 void *stream);

/* htex_sample_prepared for a batch in any order, sampled in halfedge order:
 * the library sorts the batch by halfedge (the order a rasterizer delivers,
 * Section 4.4, "Rendering", in which neighbouring queries read the same
 * textures), samples it with its sorted-batch kernels, each lane reading its
 * query as one 16-byte record through the permutation, and writes row i of
 * out for query i, as htex_sample_prepared would (the same bits).  Flags
 * are implied (none taken).  ws: device workspace of at least
 * htex_sample_reordered_workspace_bytes(H, Q, pool->channels) bytes,
 * 256-byte aligned, overlapping neither out nor the query arrays (its
 * contents on entry do not matter).  Q < 2^31 (HTEX_E_RANGE otherwise);
 * other arguments and errors as htex_sample_prepared. */
size_t htex_sample_reordered_workspace_bytes(int32_t H, int64_t Q, int32_t channels);
htex_status htex_sample_prepared_reordered(int32_t H, const void *prep, const htex_pool *pool,
                                           const htex_queries *queries, int32_t filter,
                                           float *out, void *ws, size_t ws_bytes,
                                           int32_t *err_count, void *stream);

/* ----------------------------------------------- anisotropic filtering --
 * The paper samples with the GPU's anisotropic filter (Section 5.1, Fig. 7).
 * Here that is the OpenGL anisotropic-filtering extension's filter applied
 * to each of Alg. 3's fetches.  Per query, jac[q] = (du/dx, dv/dx, du/dy,
 * dv/dy): the screen-space derivatives of the query's barycentric (u, v).
 * With px = |(du/dx, dv/dx)|, py = |(du/dy, dv/dy)|, pmax, pmin their
 * maximum and minimum and a the derivative vector of the longer axis:
 *   N = 1 if pmax = 0, else min(ceil(pmax / pmin), max_aniso) probes;
 *   probe i = 1..N at (u, v) + (i / (N + 1) - 1/2) a;
 *   each probe is Alg. 3 with trilinear fetches at footprint f = pmax / N
 *   (LOD as for htex_sample; the quad maps preserve lengths, so the same
 *   footprint holds in all three quads);
 *   out = (sum over probes and fetches of colour) / (same sum of the
 *   normalization channel).
 * N and the probe coordinates are computed in float32 with one rounding
 * per operation (squares, sums, square roots, quotients, offset, product
 * and sum; no fused multiply-add), so they are reproducible.  N = 1 is
 * exactly htex_sample's trilinear result at footprint f = pmax.  Each
 * probe's three fetches are added in Alg. 3's order, then the probes in
 * order, so a query's result does not depend on the rest of the batch.
 * Requires a pool with mips; footprint arrays in `queries` are ignored.
 * jac: device float32 [Q][4], 16-byte aligned.  A query with a non-finite
 * derivative is invalid (NaN row, *err_count incremented). */
#define HTEX_MAX_ANISO 16

/* nprobe (nullable, device int32 [Q]) receives N per query (0 if invalid). */
htex_status htex_sample_aniso(const htex_mesh *mesh, const htex_pool *pool,
                              const htex_queries *queries, const float *jac, int32_t max_aniso,
                              uint32_t flags, float *out, int32_t *nprobe, int32_t *err_count,
                              void *stream);

/* The same from prepared records (htex_prepare), bit for bit; records that
 * do not fit the pool make their queries invalid, as in
 * htex_sample_prepared. */
htex_status htex_sample_aniso_prepared(int32_t H, const void *prep, const htex_pool *pool,
                                       const htex_queries *queries, const float *jac,
                                       int32_t max_aniso, uint32_t flags, float *out,
                                       int32_t *err_count, void *stream);

/* ------------------------------------------------------------- serving --
 * A continuous-batching server over resident meshes.  Requests (a mesh id
 * and a batch of queries in host memory) are admitted in arrival order as
 * request slots and device memory (an arena of arena_bytes, 32 bytes per
 * query) free up; admitted requests are copied to the device (on
 * copy_streams upload streams; results come back on as many download
 * streams, both directions at once; whole requests in arrival order, or
 * round-robin chunks of copy_chunk_queries), and requests whose upload has
 * completed are gathered into batches, each computed by one launch over a
 * list of 256-query tiles that mixes requests and meshes; up to
 * compute_streams launches run at once, and requests arriving meanwhile
 * join a later batch.  Results are copied back into the caller's host
 * buffer; a request is complete when its result is in host memory.  Every
 * query is computed with the arithmetic of htex_sample_prepared, bit for
 * bit, so results are identical alone and in any mix.
 * A scheduler thread inside the library drives the device; the calls below
 * are thread-safe.  Not part of the paper (which renders frames); this is
 * the batched serving form of its sampling. */
typedef struct htex_server htex_server;

typedef struct htex_server_config {
    int32_t dtype;            /* texel storage of every mesh                   */
    int32_t filter;           /* HTEX_BILINEAR or HTEX_TRILINEAR              */
    int32_t max_inflight;     /* request slots (admitted, not yet complete)    */
    int32_t compute_streams;  /* concurrent batch launches, 1..4 (HIP maps a
                                 process's streams onto GPU_MAX_HW_QUEUES
                                 hardware queues, 4 by default, and streams
                                 sharing a queue serialize: 1 compute + 1 + 1
                                 copy streams in a process run with 8 queues
                                 measured best)                                */
    int64_t arena_bytes;      /* device bytes for request buffers (> 0)        */
    int64_t max_batch_queries;/* queries gathered into one launch (> 0)        */
    int32_t grid_blocks;      /* blocks per launch; 0 = 4 per compute unit     */
    int32_t max_meshes;       /* resident meshes (> 0)                         */
    int32_t copy_streams;     /* host<->device copy streams per direction, 1..4 */
    int32_t channels;         /* channels of every pool and result row: 1 or 4
                                 (0 means 4)                                   */
    int32_t copy_chunk_queries;/* > 0: requests are copied in chunks of this
                                 many queries, round-robin over the requests
                                 in flight, so the PCIe link is shared among
                                 them; 0: each request is copied whole, in
                                 arrival order                                 */
    int32_t reserved;         /* 0                                             */
} htex_server_config;

typedef struct htex_server_stats {
    int64_t submitted, completed, rejected;
    int64_t batches, queries_done;
    int64_t arena_peak_bytes;
    int32_t invalid_queries;  /* queries answered with NaN (bad h or u, v)     */
    int32_t pad;
} htex_server_stats;

/* Creates a server on the current device; allocates the arena and staging
 * buffers.  *out receives the handle. */
htex_status htex_server_create(const htex_server_config *cfg, htex_server **out);

/* Registers a resident mesh: its prepared records (htex_prepare, H records)
 * and its pool (dtype and channels must match the server's; trilinear needs
 * mips).  The
 * device memory stays owned by the caller and must outlive the server.  Up
 * to max_meshes calls; *mesh_id receives 0, 1, ... */
htex_status htex_server_add_mesh(htex_server *srv, int32_t H, const void *prep,
                                 const htex_pool *pool, int32_t *mesh_id);

/* Queues a request of Q queries on mesh `mesh_id`: h, u, v (and footprint
 * for trilinear) are HOST arrays of Q entries, out a HOST array of Q x C
 * floats (C = the server's channels); all must stay valid until the request completes (page-locked
 * memory gives asynchronous copies).  Never blocks.  Returns HTEX_E_NOMEM
 * if the request alone exceeds the arena, HTEX_E_ARG for a bad mesh id or
 * pointer.  *request_id receives a number increasing from 0. */
htex_status htex_server_submit(htex_server *srv, int32_t mesh_id, int64_t Q, const int32_t *h,
                               const float *u, const float *v, const float *footprint,
                               float *out, int64_t *request_id);

/* Non-blocking: moves up to `max` completed requests into ids[] and their
 * latency (seconds from submit to result in host memory) into latency_s[];
 * *n receives the count. */
htex_status htex_server_poll(htex_server *srv, int32_t max, int64_t *ids, double *latency_s,
                             int32_t *n);

/* Waits until every submitted request is complete (HTEX_E_BUSY after
 * timeout_s seconds). */
htex_status htex_server_drain(htex_server *srv, double timeout_s);

htex_status htex_server_stats_get(htex_server *srv, htex_server_stats *stats);

/* Finishes outstanding work, stops the scheduler and frees the server. */
htex_status htex_server_destroy(htex_server *srv);

#ifdef __cplusplus
}
#endif
#endif /* HTEX_H */
