/*
 * htex_oracle.h -- interface of the FP64 CPU oracle (test infrastructure
 * only; see htex_oracle.c).  Independent of the HIP library's headers.
 */
#ifndef HTEX_ORACLE_H
#define HTEX_ORACLE_H
#include <stdint.h>

enum { ORA_BILINEAR = 0, ORA_TRILINEAR = 1 };

typedef struct {
    int32_t H, E;
    const int32_t *twin, *next, *prev, *edge; /* [H] halfedge operators */
} ora_mesh;

typedef struct {
    int32_t E, has_mips;
    int32_t channels;        /* values per texel: 4 (RGBA) or 1          */
    int32_t pad;
    const uint8_t *log2res;  /* [E] level-0 resolution 2^k             */
    const int64_t *base;     /* [E] texel offset of level 0 of edge e   */
    const double *texels;    /* [total][channels], levels fine to coarse */
} ora_pool;

/* Per-query trace of the three fetches (s = own, Next, Prev; l = level slot). */
typedef struct {
    int32_t next, prev;
    int32_t edge[3];
    int32_t flip[3];
    int32_t level[3][2];
    int32_t i0[3][2];
    int32_t j0[3][2];
    int32_t inb[3][2];
    double phi;
    double W;
    double wf[3];
} ora_debug;

int64_t ora_sample(const ora_mesh *M, const ora_pool *P, int64_t Q, const int32_t *h,
                   const float *u, const float *v, const float *f, int filter,
                   double *out, ora_debug *dbg, int nthreads);
int64_t ora_sample_aniso(const ora_mesh *M, const ora_pool *P, int64_t Q, const int32_t *h,
                         const float *u, const float *v, const float *jac, int max_aniso,
                         double *out, int32_t *nprobe, int nthreads);
int64_t ora_backward(const ora_mesh *M, const ora_pool *P, int64_t Q, const int32_t *h,
                     const float *u, const float *v, const float *f, int filter,
                     const double *dout, double *dtex, double *dabs);
void ora_build_mips(const ora_pool *P, double *texels);
void ora_mip_backward(const ora_pool *P, double *dtex);
uint16_t ora_f32_to_bf16(float x);
double ora_bf16_to_f64(uint16_t c);
double ora_e4m3_to_f64(uint8_t c);
uint8_t ora_f64_to_e4m3_sat(double x);
void ora_quantize_bf16(const float *src, int64_t count, uint16_t *dst);
void ora_quantize_e4m3(const ora_pool *P, const float *src, int64_t total_texels,
                       uint8_t *codes, float *scale);
void ora_dequantize_bf16(const uint16_t *codes, int64_t count, double *out);
void ora_dequantize_e4m3(const ora_pool *P, const uint8_t *codes, const float *scale,
                         double *out);
void ora_texture_fetch(const ora_pool *P, int32_t e, int filter, double f, double x,
                       double y, double C[4], double *W);
int64_t ora_triangle_vertices(const ora_mesh *M, const int32_t *vert, int32_t V, const double *pos,
                              double *out);
void ora_texel_positions(const ora_mesh *M, const double *tri, const ora_pool *P, double *out);
void ora_corner_average(const ora_mesh *M, const int32_t *vert, const int32_t *face, int32_t V,
                        int32_t F, const ora_pool *P, double *texels);
int ora_validate(const ora_mesh *M, const int32_t *vert, int32_t *first_bad);
#endif
