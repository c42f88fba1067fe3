/*
 * htex_oracle.c -- plain FP64 CPU oracle for batched Htex sampling.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the package smoke check and
 * the benchmark's CPU-baseline leg may load this library.  The product path
 * (the HIP library) never calls it, links it or shares code with it.
 *
 * What it computes, from the paper (Barbier & Dupuy, "Htex: Per-Halfedge
 * Texturing for Arbitrary Mesh Topologies", 2022):
 *   - halfedge operators Twin/Next/Prev/Edge (Section 2, Fig. 2);
 *   - the quad parameterization of a halfedge's intrinsic triangle
 *     (Section 4.2, Alg. 2 TriangleToQuadUV);
 *   - Htexture (Section 4.4, Alg. 3): three texture fetches -- the halfedge's
 *     own edge quad at its (u, v), the Next halfedge's quad at (v, -u) and the
 *     Prev halfedge's quad at (-v, u) -- each filtered with CLAMP_TO_BORDER and
 *     a zero border, summed with a border-normalization channel of ones, and
 *     divided by that channel (Section 4.4, "Texture and Sampler
 *     Initialization" and "Rendering");
 *   - the texture fetch itself is the OpenGL filter the paper relies on
 *     (Section 4.3 "Filtering"): texel centres at (i + 1/2) / n, bilinear
 *     weights, and for trilinear filtering the LINEAR_MIPMAP_LINEAR level pair
 *     chosen from the footprint.  The normalization channel is all ones, so
 *     its filtered value is the sum of the in-bounds tap weights; it is
 *     computed, not stored.
 *
 * Everything is FP64 on FP32 inputs promoted exactly; the pool is passed in
 * as doubles (the caller widens the stored FP32 / BF16 / FP8 values exactly).
 * Readings of points the paper leaves open are listed in the design notes of
 * the repository; the ones that shape this code are repeated where used.
 *
 * Parity of every function here is pinned by CPU tests (closed forms,
 * invariants, the Fig. 2 table, brute force, library routines); see tests/.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#include "htex_oracle.h"

/* ------------------------------------------------------------------ layout */

/* Offset, in texels, of mip level l inside an edge whose level 0 is 2^k wide:
 * levels follow each other from the finest to the coarsest, so level l starts
 * after sum_{m<l} 4^(k-m) texels. */
static int64_t level_offset(int k, int l)
{
    int64_t off = 0;
    for (int m = 0; m < l; ++m)
        off += (int64_t)1 << (2 * (k - m));
    return off;
}

/* ------------------------------------------------------ Alg. 2 (Sec. 4.2) */

/* TriangleToQuadUV: the halfedge with the larger id keeps (u, v) (lower-left
 * half of the quad); the other one is reflected to (1-u, 1-v).  A boundary
 * halfedge has Twin = -1 and therefore always keeps (u, v). */
static int triangle_to_quad_uv(int32_t g, const int32_t *twin, double a, double b,
                               double *x, double *y)
{
    if (g > twin[g]) {
        *x = a;
        *y = b;
        return 0;
    }
    *x = 1.0 - a;
    *y = 1.0 - b;
    return 1;
}

/* -------------------------------------------- level selection (Sec. 4.3) */

/* OpenGL LINEAR_MIPMAP_LINEAR on a texture of 2^k texels per side, for an
 * isotropic footprint f in quad units: lambda = log2(f * 2^k).  lambda <= 0
 * magnifies (level 0 only); lambda >= k clamps to the coarsest level; in
 * between the two levels floor(lambda), floor(lambda)+1 are blended with the
 * fraction of lambda.  The integer part comes from the exponent of f, so
 * f = m * 2^E with m in [1, 2), floor(lambda) = E + k, frac = log2(m). */
static int lod_levels(int filter, double f, int k, int lv[2], double om[2])
{
    lv[1] = -1;
    om[1] = 0.0;
    if (filter == ORA_BILINEAR || !(f > 0.0)) {
        lv[0] = 0;
        om[0] = 1.0;
        return 1;
    }
    if (isinf(f)) {
        lv[0] = k;
        om[0] = 1.0;
        return 1;
    }
    int E;
    double m = frexp(f, &E);   /* f = m * 2^E with m in [0.5, 1) */
    m *= 2.0;
    E -= 1;                     /* now m in [1, 2) */
    int li = E + k;
    if (li < 0) {
        lv[0] = 0;
        om[0] = 1.0;
        return 1;
    }
    if (li >= k) {
        lv[0] = k;
        om[0] = 1.0;
        return 1;
    }
    double p = log2(m);
    lv[0] = li;
    om[0] = 1.0 - p;
    lv[1] = li + 1;
    om[1] = p;
    return 2;
}

/* Debug trace of the level blend: the fraction log2(m) of lambda for any
 * positive, finite footprint that is a normal float32 number (whether or not
 * a texture's level pair is clamped); 0 otherwise or for bilinear. */
static double trilinear_fraction(int filter, double f)
{
    if (filter != ORA_TRILINEAR || !(f >= 0x1p-126) || isinf(f))
        return 0.0;
    int E;
    double m = 2.0 * frexp(f, &E);
    return log2(m);
}

/* ------------------------------------------ texture fetch (Sec. 4.3-4.4) */

/* One filtered fetch: what Alg. 3's Texture(e, <x, y>) returns for the colour
 * channels and for the border-normalization channel. */
typedef struct {
    int32_t g;        /* halfedge whose quad is read                    */
    int32_t e;        /* Edge(g): the texture                           */
    int k;            /* log2 of the level-0 resolution of e            */
    int flip;         /* 1 if Alg. 2 reflected the coordinates          */
    int nlev;         /* 1 or 2 mip levels                              */
    int lv[2];        /* levels (lv[1] = -1 if unused)                  */
    double om[2];     /* level weights                                  */
    double x, y;      /* quad coordinates                               */
    int32_t i0[2], j0[2], inb[2];  /* integer tap bases, in-bounds mask */
    double C[4];      /* filtered colour (weights not normalized)        */
    double W;         /* filtered normalization channel                  */
} fetch_rec;

/* Bilinear taps of one level: texel centres at (i + 1/2)/n, so the sample
 * point in texel units is s = x n - 1/2, t = y n - 1/2; taps (i0 + di, j0 + dj)
 * with i0 = floor(s), j0 = floor(t) carry weights (1-a or a)(1-b or b),
 * a = s - i0, b = t - j0.  Taps outside [0, n)^2 read the zero border. */
typedef struct {
    int64_t i0, j0;
    double a, b;
} taps;

static taps level_taps(double x, double y, int64_t n)
{
    taps T;
    double s = x * (double)n - 0.5, t = y * (double)n - 0.5;
    double fi = floor(s), fj = floor(t);
    T.a = s - fi;
    T.b = t - fj;
    /* points far outside the quad only produce out-of-bounds taps; keep the
     * integer conversion defined (exact for |coordinate| <= 4) */
    double lim = 8.0 * (double)n;
    if (fi < -lim) fi = -lim;
    if (fi > lim) fi = lim;
    if (fj < -lim) fj = -lim;
    if (fj > lim) fj = lim;
    T.i0 = (int64_t)fi;
    T.j0 = (int64_t)fj;
    return T;
}

static double tap_weight(const taps *T, int di, int dj)
{
    return (di ? T->a : 1.0 - T->a) * (dj ? T->b : 1.0 - T->b);
}

static void texture_fetch(const ora_pool *P, fetch_rec *F)
{
    memset(F->C, 0, sizeof F->C);
    F->W = 0.0;
    for (int s = 0; s < 2; ++s) {
        F->i0[s] = F->j0[s] = F->inb[s] = 0;
    }
    for (int s = 0; s < F->nlev; ++s) {
        int l = F->lv[s];
        int64_t n = (int64_t)1 << (F->k - l);
        const int C = P->channels;
        const double *T = P->texels + C * (P->base[F->e] + level_offset(F->k, l));
        taps tp = level_taps(F->x, F->y, n);
        int mask = 0;
        for (int dj = 0; dj < 2; ++dj)
            for (int di = 0; di < 2; ++di) {
                int64_t i = tp.i0 + di, j = tp.j0 + dj;
                if (i < 0 || i >= n || j < 0 || j >= n)
                    continue;
                double ow = F->om[s] * tap_weight(&tp, di, dj);
                const double *t = T + C * (j * n + i);
                for (int c = 0; c < C; ++c)
                    F->C[c] += ow * t[c];
                F->W += ow;
                mask |= 1 << (dj * 2 + di);
            }
        F->i0[s] = (int32_t)tp.i0;
        F->j0[s] = (int32_t)tp.j0;
        F->inb[s] = mask;
    }
}

/* Alg. 3 for one query, in the algorithm's order: the own quad at (u, v),
 * the Next halfedge's quad at (v, -u), the Prev halfedge's quad at (-v, u),
 * each mapped by Alg. 2; each fetch is formed on its own and added to the
 * running sum (c <- c + Texture(...)).  htexture_sums leaves the colour
 * channels C and the normalization channel W unnormalized; htexture
 * returns c_i / c_n. */
static void htexture_sums(const ora_mesh *M, const ora_pool *P, int filter, int32_t h,
                          double u, double v, double f, fetch_rec F[3], double C[4], double *Wtot)
{
    const int32_t g[3] = {h, M->next[h], M->prev[h]};
    const double a[3] = {u, v, -v};
    const double b[3] = {v, -u, u};
    double W = 0.0;
    for (int c = 0; c < 4; ++c)
        C[c] = 0.0;
    for (int q = 0; q < 3; ++q) {
        fetch_rec *R = &F[q];
        R->g = g[q];
        R->flip = triangle_to_quad_uv(g[q], M->twin, a[q], b[q], &R->x, &R->y);
        R->e = M->edge[g[q]];
        R->k = P->log2res[R->e];
        R->nlev = lod_levels(filter, f, R->k, R->lv, R->om);
        texture_fetch(P, R);
        for (int c = 0; c < P->channels; ++c)
            C[c] += R->C[c];
        W += R->W;
    }
    *Wtot = W;
}

static void htexture(const ora_mesh *M, const ora_pool *P, int filter, int32_t h,
                     double u, double v, double f, fetch_rec F[3], double out[4],
                     double *Wtot)
{
    double C[4];
    htexture_sums(M, P, filter, h, u, v, f, F, C, Wtot);
    for (int c = 0; c < P->channels; ++c)
        out[c] = C[c] / *Wtot;
}

static int query_valid(const ora_mesh *M, int32_t h, float u, float v)
{
    return h >= 0 && h < M->H && isfinite(u) && isfinite(v);
}

int64_t ora_sample(const ora_mesh *M, const ora_pool *P, int64_t Q, const int32_t *h,
                   const float *u, const float *v, const float *fp, int filter,
                   double *out, ora_debug *dbg, int nthreads)
{
    if (filter == ORA_TRILINEAR && !P->has_mips)
        return -1;
    int64_t errs = 0;
#ifdef _OPENMP
    if (nthreads > 0)
        omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(static) reduction(+ : errs)
#endif
    for (int64_t q = 0; q < Q; ++q) {
        ora_debug *d = dbg ? dbg + q : NULL;
        if (!query_valid(M, h[q], u[q], v[q])) {
            for (int c = 0; c < P->channels; ++c)
                out[P->channels * q + c] = NAN;
            if (d) {
                memset(d, 0, sizeof(*d));
                d->next = d->prev = -1;
                for (int s = 0; s < 3; ++s) {
                    d->edge[s] = -1;
                    d->level[s][0] = d->level[s][1] = -1;
                }
            }
            errs += 1;
            continue;
        }
        double f = fp ? (double)fp[q] : 0.0;
        fetch_rec F[3];
        double W = 0.0;
        htexture(M, P, filter, h[q], (double)u[q], (double)v[q], f, F, out + P->channels * q, &W);
        if (d) {
            d->next = F[1].g;
            d->prev = F[2].g;
            for (int s = 0; s < 3; ++s) {
                d->edge[s] = F[s].e;
                d->flip[s] = F[s].flip;
                for (int l = 0; l < 2; ++l) {
                    d->level[s][l] = F[s].lv[l];
                    d->i0[s][l] = F[s].i0[l];
                    d->j0[s][l] = F[s].j0[l];
                    d->inb[s][l] = F[s].inb[l];
                }
                d->wf[s] = F[s].W;
            }
            d->phi = trilinear_fraction(filter, f);
            d->W = W;
        }
    }
    return errs;
}

/* ------------------------------------------- anisotropic filtering (Sec. 5.1) */

/* The paper samples with the GPU's anisotropic texture filter (Fig. 7).  Read
 * here as the filter of the OpenGL anisotropic-filtering extension: from the
 * screen-space derivatives of the query's barycentric coordinates, the
 * footprint's two axis lengths px = |d(u,v)/dx| and py = |d(u,v)/dy|; N =
 * ceil(pmax / pmin) probes, at most max_aniso, spread evenly along the major
 * axis, each a trilinear fetch whose level comes from pmax / N.  The maps of
 * Alg. 2 and Alg. 3 are rotations and reflections of the quad, so lengths
 * and the probe points agree in the three quads: every fetch of Alg. 3
 * becomes the sum of its N probes, colour and normalization channel alike,
 * and the result is sum C / sum W over all probes of all three fetches.
 *
 * The decisions that pick integers -- N, and the probe coordinates from
 * which tap bases follow -- are taken in float32, one rounding per
 * operation (squares, sums, square roots, quotients, the probe offset and
 * its product and sum), so the oracle and the device take them alike. */
typedef struct {
    int n;        /* probes                                  */
    float f;      /* footprint of each probe (quad units)    */
    float au, av; /* major axis in barycentric coordinates   */
} aniso_plan;

static aniso_plan aniso_setup(float dudx, float dvdx, float dudy, float dvdy, int max_aniso)
{
    volatile float t0, t1;
    t0 = dudx * dudx;
    t1 = dvdx * dvdx;
    const float px = sqrtf(t0 + t1);
    t0 = dudy * dudy;
    t1 = dvdy * dvdy;
    const float py = sqrtf(t0 + t1);
    aniso_plan A;
    const int xmajor = px >= py;
    const float pmax = xmajor ? px : py, pmin = xmajor ? py : px;
    A.au = xmajor ? dudx : dudy;
    A.av = xmajor ? dvdx : dvdy;
    if (pmax == 0.0f) {
        A.n = 1;
        A.f = 0.0f;
        return A;
    }
    const float ratio = pmax / pmin;   /* +inf when pmin is 0 */
    A.n = ratio > (float)max_aniso ? max_aniso : (int)ceilf(ratio);
    if (A.n < 1)
        A.n = 1;
    A.f = pmax / (float)A.n;
    return A;
}

/* Probe i (1..n) of a plan: (u, v) + (i / (n + 1) - 1/2) * axis. */
static void aniso_probe(const aniso_plan *A, int i, float u, float v, float *ui, float *vi)
{
    volatile float t = (float)i / (float)(A->n + 1);
    t = t - 0.5f;
    volatile float du = t * A->au, dv = t * A->av;
    *ui = u + du;
    *vi = v + dv;
}

int64_t ora_sample_aniso(const ora_mesh *M, const ora_pool *P, int64_t Q, const int32_t *h,
                         const float *u, const float *v, const float *jac, int max_aniso,
                         double *out, int32_t *nprobe, int nthreads)
{
    if (!P->has_mips || max_aniso < 1)
        return -1;
    int64_t errs = 0;
    const int C = P->channels;
#ifdef _OPENMP
    if (nthreads > 0)
        omp_set_num_threads(nthreads);
#pragma omp parallel for schedule(static) reduction(+ : errs)
#endif
    for (int64_t q = 0; q < Q; ++q) {
        const float *J = jac + 4 * q;
        int ok = query_valid(M, h[q], u[q], v[q]);
        for (int c = 0; c < 4; ++c)
            ok = ok && isfinite(J[c]);
        if (!ok) {
            for (int c = 0; c < C; ++c)
                out[C * q + c] = NAN;
            if (nprobe)
                nprobe[q] = 0;
            errs += 1;
            continue;
        }
        aniso_plan A = aniso_setup(J[0], J[1], J[2], J[3], max_aniso);
        double Cs[4] = {0, 0, 0, 0}, Ws = 0.0;
        for (int i = 1; i <= A.n; ++i) {
            float ui, vi;
            aniso_probe(&A, i, u[q], v[q], &ui, &vi);
            fetch_rec F[3];
            double Ci[4], Wi;
            htexture_sums(M, P, ORA_TRILINEAR, h[q], (double)ui, (double)vi, (double)A.f, F, Ci,
                          &Wi);
            for (int c = 0; c < C; ++c)
                Cs[c] += Ci[c];
            Ws += Wi;
        }
        for (int c = 0; c < C; ++c)
            out[C * q + c] = Cs[c] / Ws;
        if (nprobe)
            nprobe[q] = A.n;
    }
    return errs;
}

/* ----------------------------------------------------------- backward */

/* The output of Alg. 3 is linear in the texels: out_c = sum over taps of
 * (om w / W) T_c.  The gradient of L with respect to a texel channel is the
 * sum, over every query and every in-bounds tap that reads it, of
 * (om w / W) dL/dout_c.  `dtex` (pool-shaped, one double per texel channel) is added
 * to; `dabs`, if given, receives the sum of the absolute values of the same
 * contributions (a scale for tolerances). */
int64_t ora_backward(const ora_mesh *M, const ora_pool *P, int64_t Q, const int32_t *h,
                     const float *u, const float *v, const float *fp, int filter,
                     const double *dout, double *dtex, double *dabs)
{
    if (filter == ORA_TRILINEAR && !P->has_mips)
        return -1;
    int64_t errs = 0;
    for (int64_t q = 0; q < Q; ++q) {
        if (!query_valid(M, h[q], u[q], v[q])) {
            errs += 1;
            continue;
        }
        double f = fp ? (double)fp[q] : 0.0;
        fetch_rec F[3];
        double out[4], W;
        htexture(M, P, filter, h[q], (double)u[q], (double)v[q], f, F, out, &W);
        for (int s3 = 0; s3 < 3; ++s3) {
            const fetch_rec *R = &F[s3];
            for (int s = 0; s < R->nlev; ++s) {
                int64_t n = (int64_t)1 << (R->k - R->lv[s]);
                int64_t off = P->base[R->e] + level_offset(R->k, R->lv[s]);
                taps tp = level_taps(R->x, R->y, n);
                for (int dj = 0; dj < 2; ++dj)
                    for (int di = 0; di < 2; ++di) {
                        int64_t i = tp.i0 + di, j = tp.j0 + dj;
                        if (i < 0 || i >= n || j < 0 || j >= n)
                            continue;
                        double w = R->om[s] * tap_weight(&tp, di, dj) / W;
                        int64_t t = off + j * n + i;
                        const int C = P->channels;
                        for (int c = 0; c < C; ++c) {
                            double gr = w * dout[C * q + c];
                            dtex[C * t + c] += gr;
                            if (dabs)
                                dabs[C * t + c] += fabs(gr);
                        }
                    }
            }
        }
    }
    return errs;
}

/* ----------------------------------------------------------------- mips */

/* Box-filtered mip chain: each texel of level l+1 is the mean of the 2x2
 * block of level l it covers (the paper relies on hardware mip-mapping and
 * does not say how levels are made; a 2x2 box is the standard
 * construction).  Works in place on a pool whose level 0 is filled. */
void ora_build_mips(const ora_pool *P, double *texels)
{
    for (int32_t e = 0; e < P->E; ++e) {
        int k = P->log2res[e];
        for (int l = 1; l <= k; ++l) {
            int64_t n = (int64_t)1 << (k - l);
            const int C = P->channels;
            double *src = texels + C * (P->base[e] + level_offset(k, l - 1));
            double *dst = texels + C * (P->base[e] + level_offset(k, l));
            for (int64_t j = 0; j < n; ++j)
                for (int64_t i = 0; i < n; ++i)
                    for (int c = 0; c < C; ++c) {
                        double s = src[C * ((2 * j) * (2 * n) + 2 * i) + c] +
                                   src[C * ((2 * j) * (2 * n) + 2 * i + 1) + c] +
                                   src[C * ((2 * j + 1) * (2 * n) + 2 * i) + c] +
                                   src[C * ((2 * j + 1) * (2 * n) + 2 * i + 1) + c];
                        dst[C * (j * n + i) + c] = 0.25 * s;
                    }
        }
    }
}

/* ------------------------------------- intrinsic triangles (Sec. 3.1, Alg. 1) */

/* The triangle of halfedge h (Alg. 1): v0 = the position of Vert(Next h),
 * v2 = that of Vert(h), and v1 = the mean of the positions of the vertices
 * of h's face, gathered by following Next from h until it returns.  Section
 * 4.2 gives its barycentric frame: (u, v, w) = (1, 0, 0) is v2, (0, 1, 0)
 * is v0 and (0, 0, 1) is v1.  pos is [V][3]; out is [H][3][3] = v0, v1, v2.
 * Returns the number of halfedges whose face walk does not return within
 * H steps or names a vertex outside [0, V) (their rows are NaN). */
int64_t ora_triangle_vertices(const ora_mesh *M, const int32_t *vert, int32_t V, const double *pos,
                              double *out)
{
    int64_t bad = 0;
    for (int32_t h = 0; h < M->H; ++h) {
        double *o = out + 9 * (int64_t)h;
        double c[3] = {0, 0, 0};
        int64_t n = 0;
        int32_t g = h;
        int ok = 1;
        do {
            if (g < 0 || g >= M->H || vert[g] < 0 || vert[g] >= V || n > M->H) {
                ok = 0;
                break;
            }
            for (int d = 0; d < 3; ++d)
                c[d] += pos[3 * (int64_t)vert[g] + d];
            n += 1;
            g = M->next[g];
        } while (g != h);
        const int32_t nx = M->next[h];
        if (!ok || nx < 0 || nx >= M->H || vert[nx] < 0 || vert[nx] >= V) {
            for (int d = 0; d < 9; ++d)
                o[d] = NAN;
            bad += 1;
            continue;
        }
        for (int d = 0; d < 3; ++d) {
            o[d] = pos[3 * (int64_t)vert[nx] + d];
            o[3 + d] = c[d] / (double)n;
            o[6 + d] = pos[3 * (int64_t)vert[h] + d];
        }
    }
    return bad;
}

/* Surface point of every texel centre (Section 4.2 read backwards): texel
 * (i, j) of a level of n texels sits at quad coordinates x = (i + 1/2) / n,
 * y = (j + 1/2) / n.  Where x + y <= 1 it lies on the triangle of the
 * edge's larger halfedge g with (u, v) = (x, y) (Alg. 2 keeps them);
 * elsewhere on the twin's triangle with (u, v) = (1 - x, 1 - y) (Alg. 2
 * reflects them); a boundary edge has no twin and mirrors its lower-left
 * half across x + y = 1, so such a texel takes the point of its mirror
 * image (n-1-j, n-1-i).  The point is u v2 + v v0 + (1 - u - v) v1 of that
 * triangle (Alg. 1, ora_triangle_vertices).  tri is [H][3][3]; out is
 * [total][3] (padding texels are left untouched). */
void ora_texel_positions(const ora_mesh *M, const double *tri, const ora_pool *P, double *out)
{
    for (int32_t g = 0; g < M->H; ++g) {
        const int32_t t = M->twin[g];
        if (!(g > t))
            continue;
        const int32_t e = M->edge[g];
        const int k = P->log2res[e];
        for (int l = 0; l <= (P->has_mips ? k : 0); ++l) {
            const int64_t n = (int64_t)1 << (k - l);
            const int64_t lv = P->base[e] + level_offset(k, l);
            for (int64_t j = 0; j < n; ++j)
                for (int64_t i = 0; i < n; ++i) {
                    int64_t si = i, sj = j;
                    if (t < 0 && i + j > n - 1) {
                        si = n - 1 - j;
                        sj = n - 1 - i;
                    }
                    const double x = (si + 0.5) / (double)n, y = (sj + 0.5) / (double)n;
                    int32_t hh = g;
                    double u = x, v = y;
                    if (x + y > 1.0) {
                        hh = t;
                        u = 1.0 - x;
                        v = 1.0 - y;
                    }
                    const double *T = tri + 9 * (int64_t)hh;
                    const double w = 1.0 - u - v;
                    for (int d = 0; d < 3; ++d)
                        out[3 * (lv + j * n + i) + d] = u * T[6 + d] + v * T[d] + w * T[3 + d];
                }
        }
    }
}

/* ------------------------------------------ corner pre-processing (Sec. 4.4) */

/* Quad corners on the mesh.  The halfedge g of an edge with the larger id
 * keeps its barycentric (u, v) as quad coordinates (Alg. 2), and Section 4.2
 * puts Vert(g) at (u, v) = (1, 0) and Vert(Next(g)) at (0, 1); the third
 * corner of its intrinsic triangle, the centroid of g's face (Alg. 1), is at
 * (0, 0), and the twin's face centroid at (1, 1).  On a level of n texels
 * per side these four points lie in the corner texels (i, j) = (n-1, 0),
 * (0, n-1), (0, 0) and (n-1, n-1).
 *
 * The pre-processing of Section 4.4 makes every corner texel that lies on
 * one mesh vertex, or on one face centroid, hold the same value: here the
 * mean of those texels, taken separately for each resolution n >= 2 (levels
 * of different edges with equal n are averaged together).  A 1x1 level is
 * left alone: its one texel is all four corners at once.  A boundary quad
 * mirrors its lower-left half, so its (n-1, n-1) corner is the image of its
 * (0, 0) corner and takes the same value without being counted twice.
 *
 * vert[h] and face[h] give the vertex and face ids of each halfedge (V and F
 * of them); the texels are updated in place. */
void ora_corner_average(const ora_mesh *M, const int32_t *vert, const int32_t *face, int32_t V,
                        int32_t F, const ora_pool *P, double *texels)
{
    int kmax = 0;
    for (int32_t e = 0; e < P->E; ++e)
        if (P->log2res[e] > kmax)
            kmax = P->log2res[e];
    const int64_t G = (int64_t)V + F;
    const int C = P->channels;
    double *sum = (double *)malloc(sizeof(double) * 4 * (size_t)(G > 0 ? G : 1));
    int64_t *cnt = (int64_t *)malloc(sizeof(int64_t) * (size_t)(G > 0 ? G : 1));
    for (int r = 1; r <= kmax; ++r) {
        const int64_t n = (int64_t)1 << r;
        memset(sum, 0, sizeof(double) * 4 * (size_t)G);
        memset(cnt, 0, sizeof(int64_t) * (size_t)G);
        for (int pass = 0; pass < 2; ++pass) {
            for (int32_t g = 0; g < M->H; ++g) {
                const int32_t t = M->twin[g];
                if (!(g > t))
                    continue; /* visit each edge once, through its larger halfedge */
                const int32_t e = M->edge[g];
                const int k = P->log2res[e];
                const int l = k - r;
                if (l < 0 || (l > 0 && !P->has_mips))
                    continue;
                const int64_t lv = P->base[e] + level_offset(k, l);
                const int64_t at[4] = {lv + (n - 1), lv + (n - 1) * n, lv, lv + (n - 1) * n + n - 1};
                const int64_t grp[4] = {vert[g], vert[M->next[g]], (int64_t)V + face[g],
                                        t >= 0 ? (int64_t)V + face[t] : -1};
                for (int c = 0; c < 4; ++c) {
                    if (grp[c] < 0) {
                        if (pass == 1) /* boundary mirror of the (0, 0) corner */
                            for (int ch = 0; ch < C; ++ch)
                                texels[C * at[3] + ch] = texels[C * at[2] + ch];
                        continue;
                    }
                    if (pass == 0) {
                        for (int ch = 0; ch < C; ++ch)
                            sum[4 * grp[c] + ch] += texels[C * at[c] + ch];
                        cnt[grp[c]] += 1;
                    } else {
                        for (int ch = 0; ch < C; ++ch)
                            texels[C * at[c] + ch] = sum[4 * grp[c] + ch] / (double)cnt[grp[c]];
                    }
                }
            }
        }
    }
    free(sum);
    free(cnt);
}

/* Transpose of the mip chain (ora_build_mips) for gradients: when the
 * coarser levels are box means of level 0, a gradient with respect to
 * every stored level folds into one with respect to level 0.  Level l-1
 * receives a quarter of the gradient of each level-l texel in each of the
 * four texels it averages, from the coarsest level down, so level 0 ends
 * with the total; each coarser level ends with its own gradient plus what
 * came through the levels above it.  In place on `dtex` (pool-shaped). */
void ora_mip_backward(const ora_pool *P, double *dtex)
{
    const int C = P->channels;
    for (int32_t e = 0; e < P->E; ++e) {
        int k = P->log2res[e];
        for (int l = k; l >= 1; --l) {
            int64_t n = (int64_t)1 << (k - l);
            const double *src = dtex + C * (P->base[e] + level_offset(k, l));
            double *dst = dtex + C * (P->base[e] + level_offset(k, l - 1));
            for (int64_t j = 0; j < n; ++j)
                for (int64_t i = 0; i < n; ++i)
                    for (int c = 0; c < C; ++c) {
                        double g = 0.25 * src[C * (j * n + i) + c];
                        dst[C * ((2 * j) * (2 * n) + 2 * i) + c] += g;
                        dst[C * ((2 * j) * (2 * n) + 2 * i + 1) + c] += g;
                        dst[C * ((2 * j + 1) * (2 * n) + 2 * i) + c] += g;
                        dst[C * ((2 * j + 1) * (2 * n) + 2 * i + 1) + c] += g;
                    }
        }
    }
}

/* -------------------------------------------------------- quantization */

/* bfloat16: the upper 16 bits of a binary32 after rounding its significand
 * to 8 bits, to nearest with ties to even.  NaN stays NaN (quiet). */
uint16_t ora_f32_to_bf16(float x)
{
    uint32_t b;
    memcpy(&b, &x, 4);
    if ((b & 0x7f800000u) == 0x7f800000u && (b & 0x007fffffu))
        return (uint16_t)((b >> 16) | 0x0040u);
    uint32_t low = b & 0xffffu, hi = b >> 16;
    if (low > 0x8000u || (low == 0x8000u && (hi & 1u)))
        hi += 1;   /* carries into the exponent correctly, up to infinity */
    return (uint16_t)hi;
}

double ora_bf16_to_f64(uint16_t c)
{
    uint32_t b = (uint32_t)c << 16;
    float x;
    memcpy(&x, &b, 4);
    return (double)x;
}

/* OCP 8-bit E4M3 ("E4M3FN"): 1 sign, 4 exponent (bias 7), 3 mantissa bits;
 * no infinities; S.1111.111 is NaN; largest finite magnitude 448; exponent
 * field 0 encodes subnormals m * 2^-9. */
double ora_e4m3_to_f64(uint8_t c)
{
    int s = c >> 7, e = (c >> 3) & 15, m = c & 7;
    double v;
    if (e == 15 && m == 7)
        return NAN;
    if (e == 0)
        v = ldexp((double)m, -9);
    else
        v = ldexp(1.0 + m / 8.0, e - 7);
    return s ? -v : v;
}

/* Round to the nearest finite E4M3 value, ties to the even code, magnitudes
 * beyond 448 saturating to 448.  Written as a search over the 127 finite
 * non-negative codes, which is the definition itself. */
uint8_t ora_f64_to_e4m3_sat(double x)
{
    if (isnan(x))
        return 0x7f;
    int neg = signbit(x) ? 1 : 0;
    double a = fabs(x);
    if (a > 448.0)
        a = 448.0;   /* saturation: the nearest finite value */
    int best = 0;
    double bd = INFINITY;
    for (int c = 0; c <= 0x7e; ++c) {
        double d = fabs(ora_e4m3_to_f64((uint8_t)c) - a);
        if (d < bd || (d == bd && (c & 1) == 0 && (best & 1) == 1)) {
            bd = d;
            best = c;
        }
    }
    return (uint8_t)(best | (neg << 7));
}

/* Per-edge FP8 quantization: scale s_e = max |T| over every level and
 * channel of edge e divided by 448, both in float32 (the precision the
 * device quantizer decides in); codes = E4M3(T / s_e) with the quotient
 * rounded to float32 first.  An all-zero edge gets s_e = 0 and zero codes.
 * `src` is the float32 pool, `codes` receives one byte per texel channel. */
void ora_quantize_e4m3(const ora_pool *P, const float *src, int64_t total_texels,
                       uint8_t *codes, float *scale)
{
    (void)total_texels;
    for (int32_t e = 0; e < P->E; ++e) {
        int k = P->log2res[e];
        int64_t cnt = 0;
        for (int l = 0; l <= (P->has_mips ? k : 0); ++l)
            cnt += (int64_t)1 << (2 * (k - l));
        const int C = P->channels;
        const float *t = src + C * P->base[e];
        float mx = 0.0f;
        for (int64_t i = 0; i < C * cnt; ++i) {
            float a = fabsf(t[i]);
            if (a > mx)
                mx = a;
        }
        float s = mx / 448.0f;
        scale[e] = s;
        uint8_t *o = codes + C * P->base[e];
        for (int64_t i = 0; i < C * cnt; ++i) {
            if (s == 0.0f) {
                o[i] = 0;
                continue;
            }
            volatile float qv = t[i] / s;
            o[i] = ora_f64_to_e4m3_sat((double)qv);
        }
    }
}

void ora_quantize_bf16(const float *src, int64_t count, uint16_t *dst)
{
    for (int64_t i = 0; i < count; ++i)
        dst[i] = ora_f32_to_bf16(src[i]);
}

/* -------------------------------------------------------- mesh checks */

/* Halfedge invariants (Section 2 and Fig. 2): Twin is an involution where
 * defined and links opposite directions (Vert(Twin h) = Vert(Next h));
 * Next/Prev are inverse permutations; twins share their edge; every edge id
 * is used by exactly one twin pair or one lone boundary halfedge; faces have
 * at least three sides.  Returns 0 or a negative code, with the first bad
 * halfedge in *first_bad. */
int ora_validate(const ora_mesh *M, const int32_t *vert, int32_t *first_bad)
{
    int32_t H = M->H, E = M->E;
    *first_bad = -1;
    int32_t *use = (int32_t *)calloc((size_t)(E > 0 ? E : 1), sizeof(int32_t));
    int rc = 0;
    for (int32_t h = 0; h < H && rc == 0; ++h) {
        int32_t t = M->twin[h], n = M->next[h], p = M->prev[h], e = M->edge[h];
        if (t < -1 || t >= H || n < 0 || n >= H || p < 0 || p >= H || e < 0 || e >= E ||
            t == h) {
            rc = -1;
        } else if (M->prev[n] != h || M->next[p] != h) {
            rc = -2;
        } else if (t >= 0 && (M->twin[t] != h || M->edge[t] != e ||
                              (vert && vert[t] != vert[n]))) {
            rc = -3;
        } else if (n == h || M->next[n] == h) {
            rc = -4; /* face with fewer than 3 sides */
        }
        if (rc) {
            *first_bad = h;
            break;
        }
        use[e] += 1;
    }
    if (rc == 0) {
        for (int32_t h = 0; h < H; ++h) {
            int32_t e = M->edge[h];
            int want = M->twin[h] >= 0 ? 2 : 1;
            if (use[e] != want) {
                rc = -5;
                *first_bad = h;
                break;
            }
        }
        for (int32_t e = 0; e < E && rc == 0; ++e)
            if (use[e] == 0) {
                rc = -6;
                *first_bad = -1;
            }
    }
    free(use);
    return rc;
}

/* Exact widening of stored codes to FP64 (the values the sampler reads). */
void ora_dequantize_bf16(const uint16_t *codes, int64_t count, double *out)
{
    for (int64_t i = 0; i < count; ++i)
        out[i] = ora_bf16_to_f64(codes[i]);
}

/* FP8 texel value = decoded code times the edge's scale (exact in FP64). */
void ora_dequantize_e4m3(const ora_pool *P, const uint8_t *codes, const float *scale,
                         double *out)
{
    for (int32_t e = 0; e < P->E; ++e) {
        int k = P->log2res[e];
        int64_t cnt = 0;
        for (int l = 0; l <= (P->has_mips ? k : 0); ++l)
            cnt += (int64_t)1 << (2 * (k - l));
        for (int64_t i = P->channels * P->base[e]; i < P->channels * (P->base[e] + cnt); ++i)
            out[i] = ora_e4m3_to_f64(codes[i]) * (double)scale[e];
    }
}

/* Alg. 3's Texture(e, <x, y>) on its own: one filtered fetch of edge e at quad
 * coordinates (x, y) with footprint f, returning the colour C[0..3] and the
 * border-normalization channel *W. */
void ora_texture_fetch(const ora_pool *P, int32_t e, int filter, double f, double x,
                       double y, double C[4], double *W)
{
    fetch_rec R;
    memset(&R, 0, sizeof R);
    R.e = e;
    R.k = P->log2res[e];
    R.x = x;
    R.y = y;
    R.nlev = lod_levels(filter, f, R.k, R.lv, R.om);
    texture_fetch(P, &R);
    for (int c = 0; c < 4; ++c)
        C[c] = c < P->channels ? R.C[c] : 0.0;
    *W = R.W;
}
