/*
 * Ill-conditioned dot-product instances, after the idea of the GenDot
 * generator of Ogita, Rump and Oishi ("Accurate sum and dot product", SIAM
 * J. Sci. Comput. 26(6), 2005), in this project's own construction.
 *
 * This is input generation only: it holds none of the twofold method's
 * arithmetic.  The exact running dot is kept in a wide two's-complement
 * fixed-point integer, and exact products come from 53x53-bit integer
 * mantissa products, so no error-free floating-point transform is used.
 *
 * Construction for n entries (n even), exponent range e_max (chosen by the
 * caller from the target condition number) and h = n/2:
 *   - for i < h: x_i = u_i 2^{e_i}, y_i = v_i 2^{e_i}, where u, v are the
 *     caller's uniform draws in (-1, 1) and e_i the caller's exponents in
 *     [0, e_max];
 *   - for i >= h: e_i falls linearly from e_max (at i = h) to 0 (at n-1);
 *     x_i = u_i 2^{e_i} and y_i = fl((v_i 2^{e_i} + T - S~) / x_i) where S~
 *     is the exact dot S of all earlier entries read to at least 64 bits
 *     and T = 4 A / cond with A = sum_{i<h} |x_i y_i|, so the partial sums
 *     cancel down to about T + O(1) and 2 sum|x_i y_i| / |x^T y| comes out
 *     near cond (for large cond the caller narrows e_max instead);
 *   - S is then updated exactly with x_i y_i.
 * The binary32 variant computes the second-half y_i in binary32.
 *
 * Build: gcc -O2 -std=c11 -ffp-contract=off -shared -fPIC
 */
#include <math.h>
#include <stdint.h>
#include <string.h>

/* Fixed point: value = sum_k limb[k] 2^(64k - BIAS), two's complement. */
#define NLIMB 40
#define BIAS 1280 /* lowest weight 2^-1280, below the last bit of any
                     product of two finite doubles whose larger factor is
                     at least 2^-150; the top limb reaches 2^1280 */

typedef struct { uint64_t limb[NLIMB]; } acc_t;

typedef unsigned __int128 u128;

/* Split a finite double into sign, 53-bit integer mantissa and exponent of
 * its lowest bit: |x| = m 2^e. */
static void decompose(double x, int *neg, uint64_t *m, int *e)
{
    uint64_t bits;
    memcpy(&bits, &x, 8);
    *neg = (int)(bits >> 63);
    int ef = (int)((bits >> 52) & 0x7ff);
    uint64_t f = bits & ((1ull << 52) - 1);
    if (ef == 0) { /* subnormal or zero */
        *m = f;
        *e = -1074;
    } else {
        *m = f | (1ull << 52);
        *e = ef - 1075;
    }
}

/* acc += (neg ? -1 : 1) * P * 2^(pos - BIAS) where P < 2^128. */
static void acc_add(acc_t *a, int neg, u128 P, int pos)
{
    if (P == 0) return;
    if (pos < 0) { /* below the accumulator: unreachable for these inputs */
        P = -pos < 128 ? P >> -pos : 0;
        pos = 0;
        if (P == 0) return;
    }
    int L = pos / 64, sh = pos % 64;
    uint64_t w[3];
    if (sh == 0) {
        w[0] = (uint64_t)P;
        w[1] = (uint64_t)(P >> 64);
        w[2] = 0;
    } else {
        w[0] = (uint64_t)P << sh;
        w[1] = (uint64_t)(P >> (64 - sh));
        w[2] = (uint64_t)((P >> 64) >> (64 - sh));
    }
    if (!neg) {
        uint64_t carry = 0;
        for (int k = 0; k < NLIMB - L; ++k) {
            uint64_t add = k < 3 ? w[k] : 0;
            if (k >= 3 && carry == 0) break;
            u128 s = (u128)a->limb[L + k] + add + carry;
            a->limb[L + k] = (uint64_t)s;
            carry = (uint64_t)(s >> 64);
        }
    } else {
        uint64_t borrow = 0;
        for (int k = 0; k < NLIMB - L; ++k) {
            uint64_t sub = k < 3 ? w[k] : 0;
            if (k >= 3 && borrow == 0) break;
            uint64_t old = a->limb[L + k];
            uint64_t r = old - sub - borrow;
            borrow = (old < sub || (old - sub) < borrow) ? 1 : 0;
            a->limb[L + k] = r;
        }
    }
}

/* acc += x * y exactly. */
static void acc_add_product(acc_t *a, double x, double y)
{
    int nx, ny, ex, ey;
    uint64_t mx, my;
    decompose(x, &nx, &mx, &ex);
    decompose(y, &ny, &my, &ey);
    if (mx == 0 || my == 0) return;
    acc_add(a, nx ^ ny, (u128)mx * my, ex + ey + BIAS);
}

/* Nearest binary64 value of the accumulator (ties to even). */
static int acc_bit(const acc_t *t, int p) { return (int)((t->limb[p / 64] >> (p % 64)) & 1); }

static double acc_to_double(const acc_t *a)
{
    acc_t t = *a;
    int neg = (int)(t.limb[NLIMB - 1] >> 63);
    if (neg) { /* two's complement negation */
        uint64_t carry = 1;
        for (int k = 0; k < NLIMB; ++k) {
            u128 s = (u128)(~t.limb[k]) + carry;
            t.limb[k] = (uint64_t)s;
            carry = (uint64_t)(s >> 64);
        }
    }
    int H = NLIMB - 1;
    while (H >= 0 && t.limb[H] == 0) --H;
    if (H < 0) return 0.0;
    int top = 64 * H + (63 - __builtin_clzll(t.limb[H])); /* leading bit */
    int lsb = top - 52;                                     /* 53-bit window */
    uint64_t mant = 0;
    for (int p = top; p >= lsb; --p)
        mant = (mant << 1) | (uint64_t)(p >= 0 ? acc_bit(&t, p) : 0);
    int guard = lsb - 1 >= 0 ? acc_bit(&t, lsb - 1) : 0;
    int sticky = 0;
    int below = lsb - 2; /* highest bit position under the guard bit */
    if (below >= 0) {
        int L = below / 64;
        int r = below % 64;
        uint64_t mask = r == 63 ? ~0ull : ((1ull << (r + 1)) - 1);
        if (t.limb[L] & mask) sticky = 1;
        for (int k = L - 1; k >= 0 && !sticky; --k)
            if (t.limb[k]) sticky = 1;
    }
    if (guard && (sticky || (mant & 1))) mant += 1;
    double v = ldexp((double)mant, lsb - BIAS);
    return neg ? -v : v;
}

/* Fast deterministic approximation of the accumulator from its top three
 * significant limbs of magnitude (relative error below 2^-64); used only to
 * steer the construction, never reported. */
static double acc_approx(const acc_t *a)
{
    int neg = (int)(a->limb[NLIMB - 1] >> 63);
    uint64_t fill = neg ? ~0ull : 0ull;
    int H = NLIMB - 1;
    while (H > 0 && a->limb[H] == fill) --H;
    if (!neg && a->limb[H] == 0) return 0.0;
    int low = H - 2 > 0 ? H - 2 : 0;
    /* magnitude of limbs [low, H]; for a negative value the one's complement
     * of those limbs, which is short of the magnitude by less than one unit
     * of limb `low` */
    double v = 0.0;
    for (int k = H; k >= low; --k) {
        uint64_t w = neg ? ~a->limb[k] : a->limb[k];
        v = v * 18446744073709551616.0 + (double)w;
    }
    v = ldexp(v, 64 * low - BIAS);
    return neg ? -v : v;
}

/* Second-half exponent: falls linearly from e_max at i = h to 0 at n-1. */
static int e_second(int64_t i, int64_t n, int64_t h, int e_max)
{
    int64_t span = n - 1 - h;
    if (span <= 0) return 0;
    return (int)llround((double)e_max * (double)(n - 1 - i) / (double)span);
}

/*
 * Binary64 instance.  u, v: n uniform draws in (-1, 1); e1: h = n/2
 * first-half exponents in [0, e_max].  The final exact dot is rounded once,
 * to nearest-even.  Writes x, y and
 * stats[0] = achieved condition number 2 sum|x_i y_i| / |x^T y|,
 * stats[1] = fl(x^T y) (exact dot rounded once),
 * stats[2] = e_max.
 */
void tfgen_illdot_f64(int64_t n, int e_max, double cond, const double *u,
                      const double *v, const int32_t *e1, double *x, double *y,
                      double *stats)
{
    acc_t S;
    memset(&S, 0, sizeof S);
    int64_t h = n / 2;
    double abs_sum = 0.0, target = 0.0;
    for (int64_t i = 0; i < n; ++i) {
        if (i == h) target = 4.0 * abs_sum / cond;
        if (i < h) {
            x[i] = ldexp(u[i], e1[i]);
            y[i] = ldexp(v[i], e1[i]);
        } else {
            int e = e_second(i, n, h, e_max);
            x[i] = ldexp(u[i], e);
            double s = acc_approx(&S);
            double t = (ldexp(v[i], e) + target) - s;
            y[i] = x[i] != 0.0 ? t / x[i] : 0.0;
        }
        acc_add_product(&S, x[i], y[i]);
        abs_sum += fabs(x[i] * y[i]);
    }
    double dot = acc_to_double(&S);
    stats[0] = dot != 0.0 ? 2.0 * abs_sum / fabs(dot) : INFINITY;
    stats[1] = dot;
    stats[2] = (double)e_max;
}

/* Binary32 instance: as above with x, y in binary32 and the second-half
 * y_i computed in binary32 arithmetic. */
void tfgen_illdot_f32(int64_t n, int e_max, double cond, const float *u,
                      const float *v, const int32_t *e1, float *x, float *y,
                      double *stats)
{
    acc_t S;
    memset(&S, 0, sizeof S);
    int64_t h = n / 2;
    double abs_sum = 0.0;
    float target = 0.0f;
    for (int64_t i = 0; i < n; ++i) {
        if (i == h) target = (float)(4.0 * abs_sum / cond);
        if (i < h) {
            x[i] = ldexpf(u[i], e1[i]);
            y[i] = ldexpf(v[i], e1[i]);
        } else {
            int e = e_second(i, n, h, e_max);
            x[i] = ldexpf(u[i], e);
            float s = (float)acc_approx(&S);
            float t = (ldexpf(v[i], e) + target) - s;
            y[i] = x[i] != 0.0f ? t / x[i] : 0.0f;
        }
        acc_add_product(&S, (double)x[i], (double)y[i]);
        abs_sum += fabs((double)x[i] * (double)y[i]);
    }
    double dot = acc_to_double(&S);
    stats[0] = dot != 0.0 ? 2.0 * abs_sum / fabs(dot) : INFINITY;
    stats[1] = dot;
    stats[2] = (double)e_max;
}

/*
 * Exact split of products for twofold sum instances: hi_i = fl(x_i y_i)
 * and lo_i = x_i y_i - hi_i, the remainder obtained from the integer
 * product (representable unless it underflows).
 */
void tfgen_product_split_f64(int64_t n, const double *x, const double *y,
                             double *hi, double *lo)
{
    for (int64_t i = 0; i < n; ++i) {
        double p = x[i] * y[i];
        hi[i] = p;
        acc_t A;
        memset(&A, 0, sizeof A);
        acc_add_product(&A, x[i], y[i]);
        acc_add_product(&A, p, -1.0);
        lo[i] = acc_to_double(&A);
    }
}

void tfgen_product_split_f32(int64_t n, const float *x, const float *y,
                             float *hi, float *lo)
{
    for (int64_t i = 0; i < n; ++i) {
        float p = x[i] * y[i];
        hi[i] = p;
        /* a product of two binary32 values is exact in binary64 */
        double exact = (double)x[i] * (double)y[i];
        lo[i] = (float)(exact - (double)p);
    }
}

/* Exact dot of binary64 vectors rounded once to binary64 (for reporting). */
double tfgen_exact_dot_f64(int64_t n, const double *x, const double *y)
{
    acc_t S;
    memset(&S, 0, sizeof S);
    for (int64_t i = 0; i < n; ++i) acc_add_product(&S, x[i], y[i]);
    return acc_to_double(&S);
}
