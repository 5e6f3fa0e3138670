/*
 * Body of the twofold-arithmetic oracle, written once and instantiated for
 * each working type by tf_oracle.c.  TEST INFRASTRUCTURE: see tf_oracle.c.
 *
 * Before including, define
 *   T     the working type (double or float)
 *   SFX   the suffix of every exported name (f64 or f32)
 *   FMA   the correctly rounded fused multiply-add of T
 *   SQRT  the correctly rounded square root of T
 *
 * Every operation below is one IEEE operation of T rounded to nearest-even.
 * The file must be compiled with floating-point contraction off, so that
 * a*b+c is a multiply followed by an add, exactly as written.
 *
 * Notation follows the paper: a twofold z is the unevaluated sum z0 + z1,
 * z0 is the standard result and z1 approximates dz0 = z - z0.  A "dotted"
 * operand is a plain number (its low part is absent).
 */

#define TF_CAT2(a, b) a##_##b
#define TF_CAT(a, b) TF_CAT2(a, b)
#define NM(base) TF_CAT(base, SFX)

typedef struct { T z0; T z1; } NM(pair);
#define PAIR NM(pair)

/* ---------------------------------------------------------------------
 * Error-free transforms (Background section, Algorithms 1.2, 2.2, 3, 4, 5)
 * ------------------------------------------------------------------- */

/* Two-Sum (Algorithm 1.2): s = fl(a+b) and t = a+b-s exactly, for any a, b,
 * with no branch on the magnitudes. */
static PAIR NM(two_sum)(T a, T b)
{
    T s = a + b;
    T b_virt = s - a;       /* b', the part of s that came from b */
    T a_virt = s - b_virt;  /* a', the part of s that came from a */
    T b_lost = b - b_virt;  /* what b lost in the rounding */
    T a_lost = a - a_virt;  /* what a lost in the rounding */
    PAIR r;
    r.z0 = s;
    r.z1 = a_lost + b_lost;
    return r;
}

/* Two-Diff (Algorithm 2.2): d = fl(a-b) and t = a-b-d exactly, for any a, b.
 * Reading: the printed Algorithm 2.2 forms the two lost parts as b-b' and
 * a'-a, which yields -t (a-b = d - t).  Here the lost parts are taken with
 * the orientation of Algorithm 2.1 and of Shewchuk's Two-Diff: b'-b for the
 * subtrahend and a-a' for the minuend, so that a-b = d + t holds. */
static PAIR NM(two_diff)(T a, T b)
{
    T d = a - b;
    T b_virt = a - d;        /* b', the subtrahend as seen through d */
    T a_virt = b_virt + d;   /* a', the minuend rebuilt from b' and d */
    T b_lost = b_virt - b;
    T a_lost = a - a_virt;
    PAIR r;
    r.z0 = d;
    r.z1 = a_lost + b_lost;
    return r;
}

/* Two-Product-FMA (Algorithm 3): p = fl(ab), e = ab - p via one fma. */
static PAIR NM(two_prod)(T a, T b)
{
    PAIR r;
    r.z0 = a * b;
    r.z1 = FMA(a, b, -r.z0);
    return r;
}

/* Division with exact remainder (Algorithm 4): q = fl(a/b), r = a - qb. */
static PAIR NM(div_rem)(T a, T b)
{
    PAIR r;
    r.z0 = a / b;
    r.z1 = FMA(-r.z0, b, a);
    return r;
}

/* Square root with exact residual (Algorithm 5): c = sqrt(a), d = a - c^2. */
static PAIR NM(sqrt_rem)(T a)
{
    PAIR r;
    r.z0 = SQRT(a);
    r.z1 = FMA(-r.z0, r.z0, a);
    return r;
}

/* ---------------------------------------------------------------------
 * Add / subtract (Algorithms ATF1, ATF1.1, STF1, STF1.1)
 * The sums of the low parts associate to the left, as the paper states
 * for its Dekker-style formulas.
 * ------------------------------------------------------------------- */

/* ATF1: twofold + twofold. z0 = x0 (+) y0; z1 = (x1 (+) y1) (+) err(x0+y0). */
static PAIR NM(add_tt)(T x0, T x1, T y0, T y1)
{
    PAIR s = NM(two_sum)(x0, y0);
    PAIR z;
    z.z0 = s.z0;
    z.z1 = (x1 + y1) + s.z1;
    return z;
}

/* ATF1.1: twofold + dotted. z1 = x1 (+) err(x0+y0). */
static PAIR NM(add_td)(T x0, T x1, T y0)
{
    PAIR s = NM(two_sum)(x0, y0);
    PAIR z;
    z.z0 = s.z0;
    z.z1 = x1 + s.z1;
    return z;
}

/* ATF1.1 with the roles of the operands exchanged: dotted x + twofold y. */
static PAIR NM(add_dt)(T x0, T y0, T y1)
{
    PAIR s = NM(two_sum)(x0, y0);
    PAIR z;
    z.z0 = s.z0;
    z.z1 = y1 + s.z1;
    return z;
}

/* Both dotted: the exact transform itself (the 2x section notes that
 * dotted inputs give the exact transforms). */
static PAIR NM(add_dd)(T x0, T y0) { return NM(two_sum)(x0, y0); }

/* STF1: twofold - twofold. z0 = x0 (-) y0; z1 = (x1 (-) y1) (+) err(x0-y0). */
static PAIR NM(sub_tt)(T x0, T x1, T y0, T y1)
{
    PAIR d = NM(two_diff)(x0, y0);
    PAIR z;
    z.z0 = d.z0;
    z.z1 = (x1 - y1) + d.z1;
    return z;
}

/* STF1.1: twofold - dotted. z1 = x1 (+) err(x0-y0). */
static PAIR NM(sub_td)(T x0, T x1, T y0)
{
    PAIR d = NM(two_diff)(x0, y0);
    PAIR z;
    z.z0 = d.z0;
    z.z1 = x1 + d.z1;
    return z;
}

/* Dotted x - twofold y: dz0 = err(x0-y0) - y1, so z1 = err (-) y1. */
static PAIR NM(sub_dt)(T x0, T y0, T y1)
{
    PAIR d = NM(two_diff)(x0, y0);
    PAIR z;
    z.z0 = d.z0;
    z.z1 = d.z1 - y1;
    return z;
}

static PAIR NM(sub_dd)(T x0, T y0) { return NM(two_diff)(x0, y0); }

/* ---------------------------------------------------------------------
 * Multiply (Algorithms MTF1, MTF1.1)
 * Only the products that reach the result are formed: p00 with its error
 * e00, and the plain products p01, p10, p11.
 * ------------------------------------------------------------------- */

/* MTF1: z0 = p00; z1 = (e00 (+) p11) (+) (p01 (+) p10). */
static PAIR NM(mul_tt)(T x0, T x1, T y0, T y1)
{
    PAIR p = NM(two_prod)(x0, y0);   /* p00, e00 */
    T p01 = x0 * y1;
    T p10 = x1 * y0;
    T p11 = x1 * y1;
    PAIR z;
    z.z0 = p.z0;
    z.z1 = (p.z1 + p11) + (p01 + p10);
    return z;
}

/* MTF1.1: y1 = 0, so p01 and p11 vanish: z1 = e00 (+) p10. */
static PAIR NM(mul_td)(T x0, T x1, T y0)
{
    PAIR p = NM(two_prod)(x0, y0);
    PAIR z;
    z.z0 = p.z0;
    z.z1 = p.z1 + x1 * y0;
    return z;
}

/* MTF1.1 with the operands exchanged: x1 = 0, z1 = e00 (+) p01. */
static PAIR NM(mul_dt)(T x0, T y0, T y1)
{
    PAIR p = NM(two_prod)(x0, y0);
    PAIR z;
    z.z0 = p.z0;
    z.z1 = p.z1 + x0 * y1;
    return z;
}

static PAIR NM(mul_dd)(T x0, T y0) { return NM(two_prod)(x0, y0); }

/* ---------------------------------------------------------------------
 * Divide (Algorithms DTF1, DTF1.1, DTF1.1.1)
 * ------------------------------------------------------------------- */

/* DTF1: z0 = x0 (/) y0; r0 = x0 - z0 y0 and r1 = x1 - z0 y1, each with one
 * fma; c0 = r0 (+) r1; d0 = y0 (+) y1; z1 = c0 (/) d0. */
static PAIR NM(div_tt)(T x0, T x1, T y0, T y1)
{
    T z0 = x0 / y0;
    T r0 = FMA(-z0, y0, x0);
    T r1 = FMA(-z0, y1, x1);
    T c0 = r0 + r1;
    T d0 = y0 + y1;
    PAIR z;
    z.z0 = z0;
    z.z1 = c0 / d0;
    return z;
}

/* DTF1.1: y1 = 0. r = x0 - z0 y0 (exact); c = r (+) x1; z1 = c (/) y0. */
static PAIR NM(div_td)(T x0, T x1, T y0)
{
    T z0 = x0 / y0;
    T r = FMA(-z0, y0, x0);
    T c = r + x1;
    PAIR z;
    z.z0 = z0;
    z.z1 = c / y0;
    return z;
}

/* Dotted x over twofold y: DTF1 with x1 = +0 (reading; the paper lists the
 * overload but gives no separate formula). */
static PAIR NM(div_dt)(T x0, T y0, T y1)
{
    return NM(div_tt)(x0, (T)0, y0, y1);
}

/* DTF1.1.1: both dotted. z1 = (x0 - z0 y0) (/) y0; z0 + z1 is coupled. */
static PAIR NM(div_dd)(T x0, T y0)
{
    T z0 = x0 / y0;
    T r1 = FMA(-z0, y0, x0);
    PAIR z;
    z.z0 = z0;
    z.z1 = r1 / y0;
    return z;
}

/* ---------------------------------------------------------------------
 * Square root (Algorithms RPF1, RPF1.1, RTF1)
 * ------------------------------------------------------------------- */

/* RPF1 on a coupled argument (u0, u1): one Newton step,
 * v0 = sqrt(u0); v1 = (u1 (+) (u0 - v0^2)) (/) (2 (*) v0). */
static PAIR NM(sqrt_coupled)(T u0, T u1)
{
    T v0 = SQRT(u0);
    T h = FMA(-v0, v0, u0);
    PAIR v;
    v.z0 = v0;
    v.z1 = (u1 + h) / ((T)2 * v0);
    return v;
}

/* RTF1: z0 = sqrt(x0); renormalise x into u with Two-Sum; v = RPF1(u);
 * w = STF1.1(v, z0), i.e. w0 = v0 (-) z0 and w1 = v1 (+) err(v0 - z0);
 * z1 = w0 (+) w1. */
static PAIR NM(sqrt_t)(T x0, T x1)
{
    T z0 = SQRT(x0);
    PAIR u = NM(two_sum)(x0, x1);
    PAIR v = NM(sqrt_coupled)(u.z0, u.z1);
    PAIR w = NM(sub_td)(v.z0, v.z1, z0);
    PAIR z;
    z.z0 = z0;
    z.z1 = w.z0 + w.z1;
    return z;
}

/* RPF1.1: dotted argument. z1 = (x0 - z0^2) (/) (2 (*) z0). */
static PAIR NM(sqrt_d)(T x0)
{
    T z0 = SQRT(x0);
    T h = FMA(-z0, z0, x0);
    PAIR z;
    z.z0 = z0;
    z.z1 = h / ((T)2 * z0);
    return z;
}

/* ---------------------------------------------------------------------
 * Array forms of the elementwise operations.  A NULL low-part pointer
 * means the operand is dotted, which selects the *.1 / *.1.1 variant.
 * ------------------------------------------------------------------- */

#define TF_BINARY_ARRAY(op)                                                    \
    void NM(orc_##op)(int64_t n, const T *x0, const T *x1, const T *y0,        \
                      const T *y1, T *z0, T *z1)                               \
    {                                                                          \
        for (int64_t i = 0; i < n; ++i) {                                      \
            PAIR z;                                                            \
            if (x1 && y1)                                                      \
                z = NM(op##_tt)(x0[i], x1[i], y0[i], y1[i]);                   \
            else if (x1)                                                       \
                z = NM(op##_td)(x0[i], x1[i], y0[i]);                          \
            else if (y1)                                                       \
                z = NM(op##_dt)(x0[i], y0[i], y1[i]);                          \
            else                                                               \
                z = NM(op##_dd)(x0[i], y0[i]);                                 \
            z0[i] = z.z0;                                                      \
            z1[i] = z.z1;                                                      \
        }                                                                      \
    }

TF_BINARY_ARRAY(add)
TF_BINARY_ARRAY(sub)
TF_BINARY_ARRAY(mul)
TF_BINARY_ARRAY(div)

void NM(orc_sqrt)(int64_t n, const T *x0, const T *x1, T *z0, T *z1)
{
    for (int64_t i = 0; i < n; ++i) {
        PAIR z = x1 ? NM(sqrt_t)(x0[i], x1[i]) : NM(sqrt_d)(x0[i]);
        z0[i] = z.z0;
        z1[i] = z.z1;
    }
}

/* The error-free transforms themselves, exposed for the identity checks. */
#define TF_EFT_ARRAY2(fn)                                                      \
    void NM(orc_##fn)(int64_t n, const T *a, const T *b, T *hi, T *lo)         \
    {                                                                          \
        for (int64_t i = 0; i < n; ++i) {                                      \
            PAIR r = NM(fn)(a[i], b[i]);                                       \
            hi[i] = r.z0;                                                      \
            lo[i] = r.z1;                                                      \
        }                                                                      \
    }
TF_EFT_ARRAY2(two_sum)
TF_EFT_ARRAY2(two_diff)
TF_EFT_ARRAY2(two_prod)
TF_EFT_ARRAY2(div_rem)

void NM(orc_sqrt_rem)(int64_t n, const T *a, T *hi, T *lo)
{
    for (int64_t i = 0; i < n; ++i) {
        PAIR r = NM(sqrt_rem)(a[i]);
        hi[i] = r.z0;
        lo[i] = r.z1;
    }
}

/* ---------------------------------------------------------------------
 * Composite streaming operations, built only from the operations above.
 * ------------------------------------------------------------------- */

/* axpy: z_i = a*x_i + y_i with a twofold scalar a = (a[0], a[1]).
 * t = MTF1(a, x_i) (MTF1.1 when x is dotted); z_i = ATF1(t, y_i)
 * (ATF1.1 when y is dotted). */
void NM(orc_axpy)(int64_t n, const T *a, const T *x0, const T *x1,
                  const T *y0, const T *y1, T *z0, T *z1)
{
    for (int64_t i = 0; i < n; ++i) {
        PAIR t = x1 ? NM(mul_tt)(a[0], a[1], x0[i], x1[i])
                    : NM(mul_td)(a[0], a[1], x0[i]);
        PAIR z = y1 ? NM(add_tt)(t.z0, t.z1, y0[i], y1[i])
                    : NM(add_td)(t.z0, t.z1, y0[i]);
        z0[i] = z.z0;
        z1[i] = z.z1;
    }
}

/* Horner evaluation of c[0] + c[1] x + ... + c[d] x^d with dotted
 * coefficients: r = (c[d], +0); for k = d-1 down to 0,
 * r = ATF1.1(MTF1(r, x_i), c[k])  (MTF1.1 when x is dotted). */
void NM(orc_horner)(int64_t n, int degree, const T *c, const T *x0,
                    const T *x1, T *z0, T *z1)
{
    for (int64_t i = 0; i < n; ++i) {
        PAIR r;
        r.z0 = c[degree];
        r.z1 = (T)0;
        for (int k = degree - 1; k >= 0; --k) {
            PAIR m = x1 ? NM(mul_tt)(r.z0, r.z1, x0[i], x1[i])
                        : NM(mul_td)(r.z0, r.z1, x0[i]);
            r = NM(add_td)(m.z0, m.z1, c[k]);
        }
        z0[i] = r.z0;
        z1[i] = r.z1;
    }
}

/* ---------------------------------------------------------------------
 * Reductions: a fixed pairwise tree over element indices.
 *
 * The leaves are cut into tiles of 256 consecutive indices [256j, 256j+256);
 * a short last tile is padded with zero leaves.  Inside a tile the tree is
 * complete: level 1 joins leaves 2i and 2i+1, level 2 joins the level-1
 * nodes 2i and 2i+1, and so on for 8 levels.  The tile results are then
 * joined by the same adjacent pairing, their count padded with (+0, +0) up
 * to a power of two.  n = 0 gives (+0, +0).  Every node is ATF1 of its left
 * and right child, except that dotted leaves enter through Two-Sum at
 * level 1 (dotted + dotted).
 * ------------------------------------------------------------------- */

#define TF_TILE 256

/* Reduce m pairs in place by adjacent pairing; m is a power of two. */
static PAIR NM(tree_pairs)(PAIR *node, int64_t m)
{
    for (int64_t w = m; w > 1; w /= 2)
        for (int64_t i = 0; i < w / 2; ++i)
            node[i] = NM(add_tt)(node[2 * i].z0, node[2 * i].z1,
                                 node[2 * i + 1].z0, node[2 * i + 1].z1);
    return node[0];
}

static int64_t NM(pow2_ceil)(int64_t v)
{
    int64_t p = 1;
    while (p < v) p *= 2;
    return p;
}

/* Kinds of leaf: 0 = dotted value x_i; 1 = twofold (x0_i, x1_i);
 * 2 = product of dotted x_i and y_i (Two-Product);
 * 3 = product of twofolds (MTF1); 4 = twofold x times dotted y (MTF1.1);
 * 5 = dotted x times twofold y (MTF1.1 exchanged). */
static PAIR NM(leaf)(int kind, int64_t i, const T *x0, const T *x1,
                     const T *y0, const T *y1)
{
    PAIR l;
    switch (kind) {
    case 1: l.z0 = x0[i]; l.z1 = x1[i]; break;
    case 2: l = NM(two_prod)(x0[i], y0[i]); break;
    case 3: l = NM(mul_tt)(x0[i], x1[i], y0[i], y1[i]); break;
    case 4: l = NM(mul_td)(x0[i], x1[i], y0[i]); break;
    case 5: l = NM(mul_dt)(x0[i], y0[i], y1[i]); break;
    default: l.z0 = x0[i]; l.z1 = (T)0; break;
    }
    return l;
}

static PAIR NM(reduce_tree)(int kind, int64_t n, const T *x0, const T *x1,
                            const T *y0, const T *y1)
{
    PAIR zero;
    zero.z0 = (T)0;
    zero.z1 = (T)0;
    if (n <= 0) return zero;

    int64_t tiles = (n + TF_TILE - 1) / TF_TILE;
    int64_t padded = NM(pow2_ceil)(tiles);
    PAIR *part = (PAIR *)malloc((size_t)padded * sizeof(PAIR));
    PAIR node[TF_TILE];

    for (int64_t j = 0; j < tiles; ++j) {
        int64_t base = j * TF_TILE;
        if (kind == 0) {
            /* dotted leaves: level 1 is Two-Sum of the two leaf values */
            for (int64_t i = 0; i < TF_TILE / 2; ++i) {
                int64_t a = base + 2 * i, b = a + 1;
                T va = a < n ? x0[a] : (T)0;
                T vb = b < n ? x0[b] : (T)0;
                node[i] = NM(two_sum)(va, vb);
            }
            part[j] = NM(tree_pairs)(node, TF_TILE / 2);
        } else {
            for (int64_t i = 0; i < TF_TILE; ++i)
                node[i] = base + i < n
                              ? NM(leaf)(kind, base + i, x0, x1, y0, y1)
                              : zero;
            part[j] = NM(tree_pairs)(node, TF_TILE);
        }
    }
    for (int64_t j = tiles; j < padded; ++j) part[j] = zero;
    PAIR r = NM(tree_pairs)(part, padded);
    free(part);
    return r;
}

/* Twofold sum of (x0, x1), or of the dotted x0 when x1 is NULL.
 * out[0] = z0, out[1] = z1. */
void NM(orc_sum)(int64_t n, const T *x0, const T *x1, T *out)
{
    PAIR r = NM(reduce_tree)(x1 ? 1 : 0, n, x0, x1, 0, 0);
    out[0] = r.z0;
    out[1] = r.z1;
}

/* Twofold dot product: leaves are the twofold products of x_i and y_i
 * (Two-Product for dotted inputs, MTF1 / MTF1.1 otherwise). */
void NM(orc_dot)(int64_t n, const T *x0, const T *x1, const T *y0,
                 const T *y1, T *out)
{
    int kind = x1 && y1 ? 3 : x1 ? 4 : y1 ? 5 : 2;
    PAIR r = NM(reduce_tree)(kind, n, x0, x1, y0, y1);
    out[0] = r.z0;
    out[1] = r.z1;
}

/* Sequential twofold accumulator (Applications, Summation): starting from
 * (+0, +0), add the twofold t = (t0, t1) `steps` times with ATF1. */
void NM(orc_accumulate)(int64_t steps, T t0, T t1, T *out)
{
    PAIR s;
    s.z0 = (T)0;
    s.z1 = (T)0;
    for (int64_t k = 0; k < steps; ++k) s = NM(add_tt)(s.z0, s.z1, t0, t1);
    out[0] = s.z0;
    out[1] = s.z1;
}

/* ---------------------------------------------------------------------
 * Coupled ("p") algorithms and renormalisation (Dekker arithmetic section;
 * Algorithms 1.1, MPF1, DPF1, RPF1).  A coupled twofold has |z1| at most
 * half an ulp of z0; the p-algorithms drop the terms that are negligible
 * for such operands.  Operation codes: 0 add, 1 sub, 2 mul, 3 div, 4 sqrt.
 * ------------------------------------------------------------------- */

/* Fast Two-Sum (Algorithm 1.1), exact when |a| >= |b|:
 * s = a (+) b; b' = s (-) a; t = b (-) b'. */
static PAIR NM(fast_two_sum)(T a, T b)
{
    T s = a + b;
    T bv = s - a;
    PAIR r;
    r.z0 = s;
    r.z1 = b - bv;
    return r;
}

TF_EFT_ARRAY2(fast_two_sum)

/* MPF1: the product x1 y1 is dropped; z0 = p00; z1 = e00 (+) (p01 (+) p10). */
static PAIR NM(mul_pp)(T x0, T x1, T y0, T y1)
{
    PAIR p = NM(two_prod)(x0, y0);
    T p01 = x0 * y1;
    T p10 = x1 * y0;
    PAIR z;
    z.z0 = p.z0;
    z.z1 = p.z1 + (p01 + p10);
    return z;
}

/* DPF1: the divisor's low part is not added back into the denominator;
 * z0 = x0 (/) y0; r0 = fma(-z0, y0, x0); r1 = fma(-z0, y1, x1);
 * c0 = r0 (+) r1; z1 = c0 (/) y0. */
static PAIR NM(div_pp)(T x0, T x1, T y0, T y1)
{
    T z0 = x0 / y0;
    T r0 = FMA(-z0, y0, x0);
    T r1 = FMA(-z0, y1, x1);
    T c0 = r0 + r1;
    PAIR z;
    z.z0 = z0;
    z.z1 = c0 / y0;
    return z;
}

/* One coupled operation.  xt / yt say whether the operand is a twofold
 * (otherwise its low part is ignored and the dotted form applies):
 *   add, sub: ATF1 / STF1 and their 1.1 forms, which the paper keeps for
 *             coupled input;
 *   mul: MPF1; one dotted operand: MPF1.1 = MTF1.1; both: Two-Product;
 *   div: DPF1; dotted divisor: DTF1.1; dotted dividend: DPF1 with x1 = +0;
 *        both dotted: DTF1.1.1;
 *   sqrt: RPF1 on x; dotted: RPF1.1. */
static PAIR NM(coupled_op)(int op, T x0, T x1, int xt, T y0, T y1, int yt)
{
    switch (op) {
    case 0:
        return xt && yt ? NM(add_tt)(x0, x1, y0, y1) : xt ? NM(add_td)(x0, x1, y0)
               : yt ? NM(add_dt)(x0, y0, y1) : NM(add_dd)(x0, y0);
    case 1:
        return xt && yt ? NM(sub_tt)(x0, x1, y0, y1) : xt ? NM(sub_td)(x0, x1, y0)
               : yt ? NM(sub_dt)(x0, y0, y1) : NM(sub_dd)(x0, y0);
    case 2:
        return xt && yt ? NM(mul_pp)(x0, x1, y0, y1) : xt ? NM(mul_td)(x0, x1, y0)
               : yt ? NM(mul_dt)(x0, y0, y1) : NM(mul_dd)(x0, y0);
    case 3:
        return xt && yt ? NM(div_pp)(x0, x1, y0, y1) : xt ? NM(div_td)(x0, x1, y0)
               : yt ? NM(div_pp)(x0, (T)0, y0, y1) : NM(div_dd)(x0, y0);
    default:
        return xt ? NM(sqrt_coupled)(x0, x1) : NM(sqrt_d)(x0);
    }
}

/* One twofold operation of the same code, for the chains below. */
static PAIR NM(twofold_op)(int op, T x0, T x1, T y0, T y1, int yt)
{
    switch (op) {
    case 0: return yt ? NM(add_tt)(x0, x1, y0, y1) : NM(add_td)(x0, x1, y0);
    case 1: return yt ? NM(sub_tt)(x0, x1, y0, y1) : NM(sub_td)(x0, x1, y0);
    case 2: return yt ? NM(mul_tt)(x0, x1, y0, y1) : NM(mul_td)(x0, x1, y0);
    case 3: return yt ? NM(div_tt)(x0, x1, y0, y1) : NM(div_td)(x0, x1, y0);
    default: return NM(sqrt_t)(x0, x1);
    }
}

/* Array form: z = coupled op(x, y), renormalised with Fast Two-Sum when
 * `renorm` is set (Dekker mode: the output is then non-overlapping, and z0
 * is no longer the standard result).  NULL low part: dotted operand. */
void NM(orc_coupled)(int op, int renorm, int64_t n, const T *x0, const T *x1,
                     const T *y0, const T *y1, T *z0, T *z1)
{
    for (int64_t i = 0; i < n; ++i) {
        PAIR z = NM(coupled_op)(op, x0[i], x1 ? x1[i] : (T)0, x1 != 0,
                                op == 4 ? (T)0 : y0[i], y1 ? y1[i] : (T)0, y1 != 0);
        if (renorm) z = NM(fast_two_sum)(z.z0, z.z1);
        z0[i] = z.z0;
        z1[i] = z.z1;
    }
}

/* Renormalisation of twofolds with Fast Two-Sum: (s, t) = (z0 (+) z1, ...). */
void NM(orc_renorm)(int64_t n, const T *z0, const T *z1, T *s, T *t)
{
    for (int64_t i = 0; i < n; ++i) {
        PAIR r = NM(fast_two_sum)(z0[i], z1[i]);
        s[i] = r.z0;
        t[i] = r.z1;
    }
}

/* ---------------------------------------------------------------------
 * Chains: one operation applied over and over to a value that stays in
 * registers, the compute-bound regime of the performance criteria
 * (Introduction; Performance).  For every i the state starts at
 * z = (x0_i, x1_i), or (x0_i, +0) when x1 is NULL, and each of `reps` steps
 * sets z = z (op) y_i (sqrt: z = sqrt(z)); y is dotted when y1 is NULL.
 * mode 0: twofold algorithms (ATF1, STF1, MTF1, DTF1, RTF1 and the *.1
 *         forms for a dotted y);
 * mode 1: coupled algorithms (ATF1, STF1, MPF1, DPF1, RPF1);
 * mode 2: Dekker mode, each coupled step followed by Fast Two-Sum.
 * ------------------------------------------------------------------- */
void NM(orc_chain)(int op, int mode, int64_t n, int64_t reps, const T *x0,
                   const T *x1, const T *y0, const T *y1, T *z0, T *z1)
{
    int yt = y1 != 0;
    for (int64_t i = 0; i < n; ++i) {
        PAIR z;
        z.z0 = x0[i];
        z.z1 = x1 ? x1[i] : (T)0;
        T b0 = op == 4 ? (T)0 : y0[i], b1 = yt ? y1[i] : (T)0;
        for (int64_t k = 0; k < reps; ++k) {
            if (mode == 0) {
                z = NM(twofold_op)(op, z.z0, z.z1, b0, b1, yt);
            } else {
                z = NM(coupled_op)(op, z.z0, z.z1, 1, b0, b1, yt);
                if (mode == 2) z = NM(fast_two_sum)(z.z0, z.z1);
            }
        }
        z0[i] = z.z0;
        z1[i] = z.z1;
    }
}

/* Plain chain: z = x_i, then z = z (op) y_i (sqrt: sqrt(z)), `reps` times. */
void NM(orc_plain_chain)(int op, int64_t n, int64_t reps, const T *x, const T *y, T *z)
{
    for (int64_t i = 0; i < n; ++i) {
        T v = x[i];
        for (int64_t k = 0; k < reps; ++k) {
            switch (op) {
            case 0: v = v + y[i]; break;
            case 1: v = v - y[i]; break;
            case 2: v = v * y[i]; break;
            case 3: v = v / y[i]; break;
            default: v = SQRT(v);
            }
        }
        z[i] = v;
    }
}

/* ---------------------------------------------------------------------
 * Applications, batched: many independent small problems, each solved
 * with the twofold operations in the order the formulas give.
 * ------------------------------------------------------------------- */

/* Back-substitution for upper-triangular m x m systems U x = f
 * (Applications, Linear Ax=f; the Jordan block is the bidiagonal case):
 * for i = m-1 down to 0: s = f_i; for j = i+1 .. m-1:
 * s = STF1(s, MTF1(U_ij, x_j)); then x_i = DTF1(s, U_ii).
 * The state s and the x_j are twofolds; f_i starts as (f0, f1 or +0).  A
 * NULL U1 makes the matrix dotted (MTF1.1 with the dotted operand first,
 * DTF1.1).  Layout, with k the system: U entry (i, j) at
 * [(i*m + j)*nsys + k], f_i and x_i at [i*nsys + k]. */
void NM(orc_trsv_upper)(int64_t nsys, int m, const T *U0, const T *U1,
                        const T *f0, const T *f1, T *x0, T *x1)
{
    for (int64_t k = 0; k < nsys; ++k) {
        for (int i = m - 1; i >= 0; --i) {
            PAIR s;
            s.z0 = f0[(int64_t)i * nsys + k];
            s.z1 = f1 ? f1[(int64_t)i * nsys + k] : (T)0;
            for (int j = i + 1; j < m; ++j) {
                int64_t a = ((int64_t)i * m + j) * nsys + k, b = (int64_t)j * nsys + k;
                PAIR p = U1 ? NM(mul_tt)(U0[a], U1[a], x0[b], x1[b])
                            : NM(mul_dt)(U0[a], x0[b], x1[b]);
                s = NM(sub_tt)(s.z0, s.z1, p.z0, p.z1);
            }
            int64_t d = ((int64_t)i * m + i) * nsys + k;
            PAIR x = U1 ? NM(div_tt)(s.z0, s.z1, U0[d], U1[d]) : NM(div_td)(s.z0, s.z1, U0[d]);
            x0[(int64_t)i * nsys + k] = x.z0;
            x1[(int64_t)i * nsys + k] = x.z1;
        }
    }
}

/* Roots of a x^2 + b x + c = 0 by the school formula (Applications, Square
 * root), every operand a twofold and every step a twofold operation:
 * q = STF1(MTF1(b, b), MTF1(MTF1((4, 0), a), c)); d = RTF1(q);
 * e = MTF1((2, 0), a); nb = (-b0, -b1);
 * r = DTF1(STF1(nb, d), e) and s = DTF1(ATF1(nb, d), e).
 * A negative discriminant gives NaN, which flows into both roots. */
void NM(orc_quadratic)(int64_t n, const T *a0, const T *a1, const T *b0, const T *b1,
                       const T *c0, const T *c1, T *r0, T *r1, T *s0, T *s1)
{
    for (int64_t i = 0; i < n; ++i) {
        PAIR bb = NM(mul_tt)(b0[i], b1[i], b0[i], b1[i]);
        PAIR a4 = NM(mul_tt)((T)4, (T)0, a0[i], a1[i]);
        PAIR ac = NM(mul_tt)(a4.z0, a4.z1, c0[i], c1[i]);
        PAIR q = NM(sub_tt)(bb.z0, bb.z1, ac.z0, ac.z1);
        PAIR d = NM(sqrt_t)(q.z0, q.z1);
        PAIR e = NM(mul_tt)((T)2, (T)0, a0[i], a1[i]);
        T nb0 = -b0[i], nb1 = -b1[i];
        PAIR u = NM(sub_tt)(nb0, nb1, d.z0, d.z1);
        PAIR v = NM(add_tt)(nb0, nb1, d.z0, d.z1);
        PAIR r = NM(div_tt)(u.z0, u.z1, e.z0, e.z1);
        PAIR s = NM(div_tt)(v.z0, v.z1, e.z0, e.z1);
        r0[i] = r.z0;
        r1[i] = r.z1;
        s0[i] = s.z0;
        s1[i] = s.z1;
    }
}

/* ---------------------------------------------------------------------
 * Twofold fused multiply-add, z = x y + w (an extension: the paper defines
 * the four operations and the square root only).  z0 = fma(x0, y0, w0) is
 * the standard result; the error of that fma, x0 y0 + w0 - z0, is the sum
 * of two floats (Boldo and Muller, "Exact and approximated error of the
 * FMA", IEEE TC 2011) and its rounded value eps = r2 comes from their
 * ErrFma steps:
 *   (u1, u2) = TP(x0, y0); (a1, a2) = TS(w0, u2); (b1, b2) = TS(u1, a1);
 *   g = (b1 (-) z0) (+) b2; r2 = g (+) a2.
 * The remaining terms follow MTF1 and ATF1:
 *   z1 = ((eps (+) p11) (+) (p01 (+) p10)) (+) w1,
 * with the products of an absent (dotted) low part left out. */
static PAIR NM(fma_t)(T x0, T x1, int xt, T y0, T y1, int yt, T w0, T w1, int wt)
{
    T z0 = FMA(x0, y0, w0);
    PAIR u = NM(two_prod)(x0, y0);
    PAIR a = NM(two_sum)(w0, u.z1);
    PAIR b = NM(two_sum)(u.z0, a.z0);
    T g = (b.z0 - z0) + b.z1;
    T eps = g + a.z1;
    T t = eps;
    if (xt && yt) t = (t + x1 * y1) + (x0 * y1 + x1 * y0);
    else if (xt) t = t + x1 * y0;
    else if (yt) t = t + x0 * y1;
    if (wt) t = t + w1;
    PAIR z;
    z.z0 = z0;
    z.z1 = t;
    return z;
}

void NM(orc_fma)(int64_t n, const T *x0, const T *x1, const T *y0, const T *y1,
                 const T *w0, const T *w1, T *z0, T *z1)
{
    for (int64_t i = 0; i < n; ++i) {
        PAIR z = NM(fma_t)(x0[i], x1 ? x1[i] : (T)0, x1 != 0, y0[i], y1 ? y1[i] : (T)0,
                           y1 != 0, w0[i], w1 ? w1[i] : (T)0, w1 != 0);
        z0[i] = z.z0;
        z1[i] = z.z1;
    }
}

/* The plain fma, the standard result the twofold one extends. */
void NM(orc_plain_fma)(int64_t n, const T *x, const T *y, const T *w, T *z)
{ for (int64_t i = 0; i < n; ++i) z[i] = FMA(x[i], y[i], w[i]); }

/* ---------------------------------------------------------------------
 * Plain (dotted-only) counterparts: the standard results, the same
 * operation order as the z0 part of the twofold forms.
 * ------------------------------------------------------------------- */

void NM(orc_plain_add)(int64_t n, const T *x, const T *y, T *z)
{ for (int64_t i = 0; i < n; ++i) z[i] = x[i] + y[i]; }
void NM(orc_plain_sub)(int64_t n, const T *x, const T *y, T *z)
{ for (int64_t i = 0; i < n; ++i) z[i] = x[i] - y[i]; }
void NM(orc_plain_mul)(int64_t n, const T *x, const T *y, T *z)
{ for (int64_t i = 0; i < n; ++i) z[i] = x[i] * y[i]; }
void NM(orc_plain_div)(int64_t n, const T *x, const T *y, T *z)
{ for (int64_t i = 0; i < n; ++i) z[i] = x[i] / y[i]; }
void NM(orc_plain_sqrt)(int64_t n, const T *x, T *z)
{ for (int64_t i = 0; i < n; ++i) z[i] = SQRT(x[i]); }

void NM(orc_plain_axpy)(int64_t n, T a, const T *x, const T *y, T *z)
{ for (int64_t i = 0; i < n; ++i) z[i] = a * x[i] + y[i]; }

void NM(orc_plain_horner)(int64_t n, int degree, const T *c, const T *x, T *z)
{
    for (int64_t i = 0; i < n; ++i) {
        T r = c[degree];
        for (int k = degree - 1; k >= 0; --k) r = r * x[i] + c[k];
        z[i] = r;
    }
}

static T NM(plain_tree)(int64_t n, const T *x, const T *y)
{
    if (n <= 0) return (T)0;
    int64_t tiles = (n + TF_TILE - 1) / TF_TILE;
    int64_t padded = NM(pow2_ceil)(tiles);
    T *part = (T *)malloc((size_t)padded * sizeof(T));
    T node[TF_TILE];
    for (int64_t j = 0; j < tiles; ++j) {
        for (int64_t i = 0; i < TF_TILE; ++i) {
            int64_t k = j * TF_TILE + i;
            node[i] = k < n ? (y ? x[k] * y[k] : x[k]) : (T)0;
        }
        for (int w = TF_TILE; w > 1; w /= 2)
            for (int i = 0; i < w / 2; ++i) node[i] = node[2 * i] + node[2 * i + 1];
        part[j] = node[0];
    }
    for (int64_t j = tiles; j < padded; ++j) part[j] = (T)0;
    for (int64_t w = padded; w > 1; w /= 2)
        for (int64_t i = 0; i < w / 2; ++i) part[i] = part[2 * i] + part[2 * i + 1];
    T r = part[0];
    free(part);
    return r;
}

void NM(orc_plain_sum)(int64_t n, const T *x, T *out) { out[0] = NM(plain_tree)(n, x, 0); }
void NM(orc_plain_dot)(int64_t n, const T *x, const T *y, T *out)
{ out[0] = NM(plain_tree)(n, x, y); }

#undef PAIR
#undef NM
#undef TF_CAT
#undef TF_CAT2
#undef TF_BINARY_ARRAY
#undef TF_EFT_ARRAY2
#undef TF_TILE
