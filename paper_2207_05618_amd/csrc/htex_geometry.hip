// htex_geometry.hip -- the intrinsic triangle of every halfedge (Section 3.1,
// Alg. 1): v0 = Vert(Next h), v2 = Vert(h) and v1 = the mean of the vertices
// of h's face, found by following Next from h until it returns.  Section
// 4.2's barycentric frame puts (u, v, w) = (1, 0, 0) at v2, (0, 1, 0) at v0
// and (0, 0, 1) at v1, so a query (h, u, v) is the surface point
// u v2 + v v0 + (1 - u - v) v1.
//
// One lane per halfedge.  The centroid is summed as float32 pairs with every
// rounding error kept, starting at the face's smallest halfedge, and
// rounded once, so every triangle of a face gets the same v1 bit for bit.  The walk
// is bounded: a face ring longer than kMaxRing halfedges, a walk that leaves
// [0, H) or a vertex id outside [0, V) makes the lane write NaN and count
// an error.
#include <hip/hip_runtime.h>

#include "htex_internal.h"

namespace htex {
namespace {

constexpr int kBlock = 256;
constexpr int32_t kMaxRing = 1 << 16;

__global__ void __launch_bounds__(kBlock) k_triangle_vertices(htex_mesh m, const int32_t *vert,
                                                              int32_t V, const float *pos,
                                                              float *out, int32_t *err)
{
    const int64_t hi = (int64_t)blockIdx.x * kBlock + threadIdx.x;
    if (hi >= m.H) return;
    const int32_t h = (int32_t)hi;
    float *o = out + 9 * hi;
    // first walk: check the ring and find its smallest halfedge, so that
    // every triangle of the face sums the centroid in the same order
    bool ok = true;
    int32_t g = h, first = h, n = 0;
    do {
        if ((uint32_t)vert[g] >= (uint32_t)V || n >= kMaxRing) {
            ok = false;
            break;
        }
        first = min(first, g);
        ++n;
        g = m.next[g];
        if ((uint32_t)g >= (uint32_t)m.H) {
            ok = false;
            break;
        }
    } while (g != h);
    const int32_t v0 = ok ? vert[m.next[h]] : -1;   // Next(h) was checked by the walk
    const int32_t v2 = vert[h];
    if (!ok || (uint32_t)v2 >= (uint32_t)V) {
        const float nan = __uint_as_float(0x7fc00000u);
        for (int d = 0; d < 9; ++d) o[d] = nan;
        if (err) atomicAdd(err, 1);
        return;
    }
    PairSum c[3];
    g = first;
    do {
        const int64_t vg = vert[g];
        c[0].add(pos[3 * vg + 0]);
        c[1].add(pos[3 * vg + 1]);
        c[2].add(pos[3 * vg + 2]);
        g = m.next[g];
    } while (g != first);
    for (int d = 0; d < 3; ++d) {
        o[d] = pos[3 * (int64_t)v0 + d];
        o[3 + d] = c[d].mean(n);
        o[6 + d] = pos[3 * (int64_t)v2 + d];
    }
}

}  // namespace

hipError_t launch_triangle_vertices(const htex_mesh &m, const int32_t *vert, int32_t V,
                                    const float *pos, float *out, int32_t *err, hipStream_t s)
{
    if (m.H == 0) return hipSuccess;
    const uint32_t G = (uint32_t)((m.H + kBlock - 1) / kBlock);
    hipLaunchKernelGGL(k_triangle_vertices, dim3(G), dim3(kBlock), 0, s, m, vert, V, pos, out,
                       err);
    return hipGetLastError();
}

}  // namespace htex
