// htex_corner.hip -- corner pre-processing of a float32 texel pool (Section
// 4.4, "Corner Pre-processing"): every corner texel that lies on one mesh
// vertex, or on one face centroid, takes the mean of those texels, level by
// level among levels of equal resolution n >= 2.  Afterwards filtering near
// a vertex or a centroid reads one value whichever quads it touches, which
// is what makes displaced surfaces crack-free.
//
// Which texel is which corner.  The larger halfedge g of an edge keeps its
// barycentric (u, v) as quad coordinates (Alg. 2), and Section 4.2 puts
// Vert(g) at (1, 0), Vert(Next g) at (0, 1) and the centroid of g's face
// (Alg. 1) at (0, 0); the twin's face centroid is at (1, 1).  On a level of
// n texels per side those points lie in texels (n-1, 0), (0, n-1), (0, 0)
// and (n-1, n-1).  A boundary quad mirrors its lower-left half, so its
// (n-1, n-1) corner is written with the value of its (0, 0) corner.  A 1x1
// level is left alone: its one texel is all four corners.
//
// Groups come from the halfedge operators alone.  A face is a Next cycle.
// The halfedges leaving a vertex are an orbit of R(g) = Twin(Prev g): a
// cycle around an interior vertex, and around a boundary vertex a chain that
// starts at the outgoing boundary halfedge (Twin = -1) and ends at the
// halfedge whose Prev is the incoming boundary halfedge.  A halfedge leaving
// the vertex meets it at its quad's (n-1, 0) corner when it is its edge's
// larger halfedge and at (0, n-1) otherwise; the incoming boundary
// halfedge's quad meets it at (0, n-1).
//
// One lane per halfedge.  The lane of a face's smallest halfedge, of an
// interior vertex's smallest outgoing halfedge, or of a boundary vertex's
// chain start owns that group: it sums the group's corner texels as float32
// pairs with every rounding error kept (walk order, so the result is
// deterministic) and writes the mean, rounded once, to every one of them.  Groups are disjoint sets of
// texels, so owners never read what another owner writes.  Walks are
// bounded: a ring longer than kMaxRing halfedges, or one that leaves
// [0, H), is counted as an error and its group is left unchanged.
#include <hip/hip_runtime.h>

#include "htex_internal.h"

namespace htex {
namespace {

constexpr int kBlock = 256;
constexpr int32_t kMaxRing = 1 << 16;

struct CornerArgs {
    const int32_t *twin, *next, *prev, *edge;
    int32_t H, E;
    const uint8_t *log2res;
    const int64_t *base;
    float *tex;
    int channels;
    int has_mips;
    int kmax;
    int32_t *err;
};

enum Corner { kC10 = 0, kC01 = 1, kC00 = 2, kC11 = 3 };

// Texel index of a corner of edge e's level of resolution 2^r, or -1 when
// the edge has no such level (or e is not an edge id).
__device__ __forceinline__ int64_t corner_texel(const CornerArgs &a, int32_t e, int r, int c)
{
    if ((uint32_t)e >= (uint32_t)a.E) return -1;
    const int k = a.log2res[e];
    const int l = k - r;
    if (l < 0 || (l > 0 && !a.has_mips)) return -1;
    const int64_t n = int64_t(1) << r;
    const int64_t lv = a.base[e] + level_offset(k, l);
    switch (c) {
    case kC10: return lv + n - 1;
    case kC01: return lv + (n - 1) * n;
    case kC00: return lv;
    default: return lv + (n - 1) * n + n - 1;
    }
}

// Visit the (edge, corner) pairs of a group with fn(e, corner, mirrored):
// `mirrored` marks a boundary quad's (0, 0) corner, whose (n-1, n-1) image
// must receive the same value.
template <typename Fn>
__device__ __forceinline__ void face_ring(const CornerArgs &a, int32_t g, Fn fn)
{
    int32_t x = g;
    do {
        const int32_t t = a.twin[x];
        fn(a.edge[x], x > t ? kC00 : kC11, t < 0);
        x = a.next[x];
    } while (x != g);
}

template <typename Fn>
__device__ __forceinline__ void vertex_ring(const CornerArgs &a, int32_t g, Fn fn)
{
    int32_t x = g;
    do {
        fn(a.edge[x], x > a.twin[x] ? kC10 : kC01, false);
        const int32_t p = a.prev[x];
        const int32_t t = a.twin[p];
        if (t < 0) {   // p is the incoming boundary halfedge
            fn(a.edge[p], kC01, false);
            break;
        }
        x = t;
    } while (x != g);
}

// True when g owns its face: it is the smallest halfedge of its Next cycle.
// *bad is set when the walk runs too long or leaves [0, H).
__device__ __forceinline__ bool owns_face(const CornerArgs &a, int32_t g, bool *bad)
{
    int32_t x = a.next[g];
    for (int32_t s = 0; s < kMaxRing; ++s) {
        if ((uint32_t)x >= (uint32_t)a.H) { *bad = true; return false; }
        if (x == g) return true;
        if (x < g) return false;
        x = a.next[x];
    }
    *bad = true;
    return false;
}

// True when g owns its origin vertex: it starts a boundary chain, or it is
// the smallest halfedge of an interior vertex's cycle.
__device__ __forceinline__ bool owns_vertex(const CornerArgs &a, int32_t g, bool *bad)
{
    const bool chain_start = a.twin[g] < 0;
    int32_t x = g;
    for (int32_t s = 0; s < kMaxRing; ++s) {
        const int32_t p = a.prev[x];
        if ((uint32_t)p >= (uint32_t)a.H) { *bad = true; return false; }
        const int32_t t = a.twin[p];
        if (t < 0) return chain_start;            // end of a chain
        if ((uint32_t)t >= (uint32_t)a.H) { *bad = true; return false; }
        if (t == g) return !chain_start;          // closed cycle
        if (!chain_start && t < g) return false;  // a smaller member owns it
        x = t;
    }
    *bad = true;
    return false;
}

template <bool FACE, typename Fn>
__device__ __forceinline__ void ring(const CornerArgs &a, int32_t g, Fn fn)
{
    if constexpr (FACE) face_ring(a, g, fn); else vertex_ring(a, g, fn);
}

template <bool FACE>
__device__ void average_group(const CornerArgs &a, int32_t g)
{
    const int C = a.channels;
    for (int r = 1; r <= a.kmax; ++r) {
        PairSum s[4];
        int32_t cnt = 0;
        ring<FACE>(a, g, [&](int32_t e, int c, bool) {
            const int64_t t = corner_texel(a, e, r, c);
            if (t < 0) return;
            for (int ch = 0; ch < C; ++ch) s[ch].add(a.tex[C * t + ch]);
            ++cnt;
        });
        if (cnt == 0) continue;
        float mean[4];
        for (int ch = 0; ch < 4; ++ch) mean[ch] = s[ch].mean(cnt);
        ring<FACE>(a, g, [&](int32_t e, int c, bool mirrored) {
            const int64_t t = corner_texel(a, e, r, c);
            if (t < 0) return;
            for (int ch = 0; ch < C; ++ch) a.tex[C * t + ch] = mean[ch];
            if (mirrored) {
                const int64_t m = corner_texel(a, e, r, kC11);
                for (int ch = 0; ch < C; ++ch) a.tex[C * m + ch] = mean[ch];
            }
        });
    }
}

__global__ void __launch_bounds__(kBlock) k_corners(CornerArgs a)
{
    const int64_t gi = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (gi >= a.H) return;
    const int32_t g = (int32_t)gi;
    bool bad = false;
    if (owns_face(a, g, &bad)) average_group<true>(a, g);
    if (owns_vertex(a, g, &bad)) average_group<false>(a, g);
    if (bad && a.err) atomicAdd(a.err, 1);
}

}  // namespace

hipError_t launch_corner_average(const htex_mesh &m, float *texels, const uint8_t *log2res,
                                 const int64_t *base, int channels, int has_mips, int kmax,
                                 int32_t *err, hipStream_t s)
{
    if (m.H == 0 || kmax < 1) return hipSuccess;
    CornerArgs a{m.twin, m.next, m.prev, m.edge, m.H, m.E, log2res, base, texels,
                 channels, has_mips, kmax, err};
    const uint32_t G = (uint32_t)((m.H + kBlock - 1) / kBlock);
    hipLaunchKernelGGL(k_corners, dim3(G), dim3(kBlock), 0, s, a);
    return hipGetLastError();
}

}  // namespace htex
