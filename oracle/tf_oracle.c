/*
 * Twofold fast arithmetic (Latkin, "Twofold fast arithmetic", 2014):
 * a plain, slow, scalar CPU oracle.
 *
 * TEST INFRASTRUCTURE.  This library exists to check the GPU library.  Only
 * the test suite, the smoke check and the benchmark's CPU-baseline leg load
 * it; the product path never calls, links or imports it, and it shares no
 * code, header or table with the GPU sources.
 *
 * Each function takes the paper's steps in the paper's order, one IEEE
 * operation at a time, in the working type (binary64 or binary32 mirror).
 * Compile with floating-point contraction off and without fast-math:
 *     gcc -O2 -std=c11 -ffp-contract=off -fno-fast-math -shared -fPIC
 * x86-64 evaluates float and double in SSE registers (no extended
 * precision), fma()/fmaf() are the C library's correctly rounded fused
 * multiply-add and sqrt()/sqrtf() are correctly rounded.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>

#define T double
#define SFX f64
#define FMA fma
#define SQRT sqrt
#include "tf_oracle_t.h"
#undef T
#undef SFX
#undef FMA
#undef SQRT

#define T float
#define SFX f32
#define FMA fmaf
#define SQRT sqrtf
#include "tf_oracle_t.h"
#undef T
#undef SFX
#undef FMA
#undef SQRT

/*
 * FP64 reference for judging binary32 twofolds.
 *
 * The paper notes that checking float arithmetic by recomputing it in
 * double is the easy route.  For binary32 inputs widened to binary64 the
 * binary64 twofold operation above gives Z0 + Z1 close to the exact z, with
 * an error far below a binary32 ulp; the reference deviation of a binary32
 * standard result z0 is then dz = (Z0 - z0) + Z1, computed in binary64.
 * A NULL low-part pointer means a dotted operand, as everywhere else.
 */
static double *widen(int64_t n, const float *x)
{
    if (!x) return 0;
    double *w = (double *)malloc((size_t)(n > 0 ? n : 1) * sizeof(double));
    for (int64_t i = 0; i < n; ++i) w[i] = (double)x[i];
    return w;
}

static void deviation(int64_t n, const double *Z0, const double *Z1,
                      const float *z0, double *dz)
{
    for (int64_t i = 0; i < n; ++i) dz[i] = (Z0[i] - (double)z0[i]) + Z1[i];
}

typedef void (*binary_f64)(int64_t, const double *, const double *,
                           const double *, const double *, double *, double *);

static void ref64_binary(binary_f64 op, int64_t n, const float *x0,
                         const float *x1, const float *y0, const float *y1,
                         const float *z0, double *dz)
{
    double *X0 = widen(n, x0), *X1 = widen(n, x1);
    double *Y0 = widen(n, y0), *Y1 = widen(n, y1);
    double *Z0 = (double *)malloc((size_t)(n > 0 ? n : 1) * sizeof(double));
    double *Z1 = (double *)malloc((size_t)(n > 0 ? n : 1) * sizeof(double));
    op(n, X0, X1, Y0, Y1, Z0, Z1);
    deviation(n, Z0, Z1, z0, dz);
    free(X0); free(X1); free(Y0); free(Y1); free(Z0); free(Z1);
}

void orc_ref64_add(int64_t n, const float *x0, const float *x1, const float *y0,
                   const float *y1, const float *z0, double *dz)
{ ref64_binary(orc_add_f64, n, x0, x1, y0, y1, z0, dz); }
void orc_ref64_sub(int64_t n, const float *x0, const float *x1, const float *y0,
                   const float *y1, const float *z0, double *dz)
{ ref64_binary(orc_sub_f64, n, x0, x1, y0, y1, z0, dz); }
void orc_ref64_mul(int64_t n, const float *x0, const float *x1, const float *y0,
                   const float *y1, const float *z0, double *dz)
{ ref64_binary(orc_mul_f64, n, x0, x1, y0, y1, z0, dz); }
void orc_ref64_div(int64_t n, const float *x0, const float *x1, const float *y0,
                   const float *y1, const float *z0, double *dz)
{ ref64_binary(orc_div_f64, n, x0, x1, y0, y1, z0, dz); }

void orc_ref64_sqrt(int64_t n, const float *x0, const float *x1,
                    const float *z0, double *dz)
{
    double *X0 = widen(n, x0), *X1 = widen(n, x1);
    double *Z0 = (double *)malloc((size_t)(n > 0 ? n : 1) * sizeof(double));
    double *Z1 = (double *)malloc((size_t)(n > 0 ? n : 1) * sizeof(double));
    orc_sqrt_f64(n, X0, X1, Z0, Z1);
    deviation(n, Z0, Z1, z0, dz);
    free(X0); free(X1); free(Z0); free(Z1);
}

void orc_ref64_axpy(int64_t n, const float *a, const float *x0, const float *x1,
                    const float *y0, const float *y1, const float *z0,
                    double *dz)
{
    double A[2] = {(double)a[0], (double)a[1]};
    double *X0 = widen(n, x0), *X1 = widen(n, x1);
    double *Y0 = widen(n, y0), *Y1 = widen(n, y1);
    double *Z0 = (double *)malloc((size_t)(n > 0 ? n : 1) * sizeof(double));
    double *Z1 = (double *)malloc((size_t)(n > 0 ? n : 1) * sizeof(double));
    orc_axpy_f64(n, A, X0, X1, Y0, Y1, Z0, Z1);
    deviation(n, Z0, Z1, z0, dz);
    free(X0); free(X1); free(Y0); free(Y1); free(Z0); free(Z1);
}

void orc_ref64_horner(int64_t n, int degree, const float *c, const float *x0,
                      const float *x1, const float *z0, double *dz)
{
    double C[64];
    for (int k = 0; k <= degree && k < 64; ++k) C[k] = (double)c[k];
    double *X0 = widen(n, x0), *X1 = widen(n, x1);
    double *Z0 = (double *)malloc((size_t)(n > 0 ? n : 1) * sizeof(double));
    double *Z1 = (double *)malloc((size_t)(n > 0 ? n : 1) * sizeof(double));
    orc_horner_f64(n, degree, C, X0, X1, Z0, Z1);
    deviation(n, Z0, Z1, z0, dz);
    free(X0); free(X1); free(Z0); free(Z1);
}

void orc_ref64_sum(int64_t n, const float *x0, const float *x1, const float *z0,
                   double *dz)
{
    double *X0 = widen(n, x0), *X1 = widen(n, x1);
    double Z[2];
    orc_sum_f64(n, X0, X1, Z);
    deviation(1, &Z[0], &Z[1], z0, dz);
    free(X0); free(X1);
}

void orc_ref64_dot(int64_t n, const float *x0, const float *x1, const float *y0,
                   const float *y1, const float *z0, double *dz)
{
    double *X0 = widen(n, x0), *X1 = widen(n, x1);
    double *Y0 = widen(n, y0), *Y1 = widen(n, y1);
    double Z[2];
    orc_dot_f64(n, X0, X1, Y0, Y1, Z);
    deviation(1, &Z[0], &Z[1], z0, dz);
    free(X0); free(X1); free(Y0); free(Y1);
}
