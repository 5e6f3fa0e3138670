// Device-side twofold arithmetic for gfx950.
//
// A twofold z = z.hi + z.lo holds the standard result in hi (the paper's z0)
// and the estimate of its deviation in lo (z1).  Every function is a fixed,
// branch-free sequence of IEEE binary64/binary32 operations; the library is
// compiled with contraction off, so each + - * / below is one correctly
// rounded instruction (or the compiler's correctly rounded division / square
// root expansion) and each fma is one v_fma.  Results are therefore bitwise
// reproducible and independent of how the work is spread over the GPU.
#pragma once

#include <hip/hip_runtime.h>

namespace tf {

template <typename T>
struct Pair {
    T hi;  // z0: the standard result
    T lo;  // z1: estimate of z - z0
};

template <typename T>
__device__ __forceinline__ T fma_rn(T a, T b, T c);
template <>
__device__ __forceinline__ double fma_rn<double>(double a, double b, double c) { return __builtin_fma(a, b, c); }
template <>
__device__ __forceinline__ float fma_rn<float>(float a, float b, float c) { return __builtin_fmaf(a, b, c); }

template <typename T>
__device__ __forceinline__ T sqrt_rn(T a);
template <>
__device__ __forceinline__ double sqrt_rn<double>(double a) { return __builtin_sqrt(a); }
template <>
__device__ __forceinline__ float sqrt_rn<float>(float a) { return __builtin_sqrtf(a); }

// ---- error-free transforms (Background section) --------------------------

// Two-Sum, Algorithm 1.2: s = a (+) b and the exact rounding error, for any
// a and b (no magnitude test, so no branch).
template <typename T>
__device__ __forceinline__ Pair<T> two_sum(T a, T b) {
    const T s = a + b;
    const T bb = s - a;            // b as it survives inside s
    const T aa = s - bb;           // a as it survives inside s
    const T da = a - aa;           // part of a rounded away
    const T db = b - bb;           // part of b rounded away
    return {s, da + db};
}

// Two-Diff, Algorithm 2.2 with the error oriented so that a - b = d + t: the
// minuend's lost part is a - a', the subtrahend's is b' - b.
template <typename T>
__device__ __forceinline__ Pair<T> two_diff(T a, T b) {
    const T d = a - b;
    const T bb = a - d;            // b as it survives inside d
    const T aa = bb + d;           // a rebuilt from d and that b
    const T da = a - aa;
    const T db = bb - b;
    return {d, da + db};
}

// Two-Product, Algorithm 3: p = a (*) b, e = fma(a, b, -p).
template <typename T>
__device__ __forceinline__ Pair<T> two_prod(T a, T b) {
    const T p = a * b;
    return {p, fma_rn(a, b, -p)};
}

// ---- add / subtract: ATF1, ATF1.1, STF1, STF1.1 ---------------------------
// Dotted operands are passed as plain values.  Chains of low-part sums
// associate to the left.

template <typename T>
__device__ __forceinline__ Pair<T> add_tt(T x0, T x1, T y0, T y1) {
    const Pair<T> s = two_sum(x0, y0);
    return {s.hi, (x1 + y1) + s.lo};
}
template <typename T>
__device__ __forceinline__ Pair<T> add_td(T x0, T x1, T y0) {
    const Pair<T> s = two_sum(x0, y0);
    return {s.hi, x1 + s.lo};
}
template <typename T>
__device__ __forceinline__ Pair<T> add_dt(T x0, T y0, T y1) {
    const Pair<T> s = two_sum(x0, y0);
    return {s.hi, y1 + s.lo};
}
template <typename T>
__device__ __forceinline__ Pair<T> add_dd(T x0, T y0) { return two_sum(x0, y0); }

template <typename T>
__device__ __forceinline__ Pair<T> sub_tt(T x0, T x1, T y0, T y1) {
    const Pair<T> d = two_diff(x0, y0);
    return {d.hi, (x1 - y1) + d.lo};
}
template <typename T>
__device__ __forceinline__ Pair<T> sub_td(T x0, T x1, T y0) {
    const Pair<T> d = two_diff(x0, y0);
    return {d.hi, x1 + d.lo};
}
template <typename T>
__device__ __forceinline__ Pair<T> sub_dt(T x0, T y0, T y1) {
    const Pair<T> d = two_diff(x0, y0);
    return {d.hi, d.lo - y1};
}
template <typename T>
__device__ __forceinline__ Pair<T> sub_dd(T x0, T y0) { return two_diff(x0, y0); }

// ---- multiply: MTF1, MTF1.1 -----------------------------------------------

template <typename T>
__device__ __forceinline__ Pair<T> mul_tt(T x0, T x1, T y0, T y1) {
    const Pair<T> p = two_prod(x0, y0);            // p00, e00
    const T cross = x0 * y1 + x1 * y0;             // p01 (+) p10
    const T low = p.lo + x1 * y1;                  // e00 (+) p11
    return {p.hi, low + cross};
}
template <typename T>
__device__ __forceinline__ Pair<T> mul_td(T x0, T x1, T y0) {
    const Pair<T> p = two_prod(x0, y0);
    return {p.hi, p.lo + x1 * y0};
}
template <typename T>
__device__ __forceinline__ Pair<T> mul_dt(T x0, T y0, T y1) {
    const Pair<T> p = two_prod(x0, y0);
    return {p.hi, p.lo + x0 * y1};
}
template <typename T>
__device__ __forceinline__ Pair<T> mul_dd(T x0, T y0) { return two_prod(x0, y0); }

// ---- divide: DTF1, DTF1.1, DTF1.1.1 ---------------------------------------

template <typename T>
__device__ __forceinline__ Pair<T> div_tt(T x0, T x1, T y0, T y1) {
    const T q = x0 / y0;
    const T r0 = fma_rn(-q, y0, x0);               // exact remainder
    const T r1 = fma_rn(-q, y1, x1);
    return {q, (r0 + r1) / (y0 + y1)};
}
template <typename T>
__device__ __forceinline__ Pair<T> div_td(T x0, T x1, T y0) {
    const T q = x0 / y0;
    const T r = fma_rn(-q, y0, x0);
    return {q, (r + x1) / y0};
}
template <typename T>
__device__ __forceinline__ Pair<T> div_dt(T x0, T y0, T y1) { return div_tt(x0, T(0), y0, y1); }
template <typename T>
__device__ __forceinline__ Pair<T> div_dd(T x0, T y0) {
    const T q = x0 / y0;
    const T r = fma_rn(-q, y0, x0);
    return {q, r / y0};
}

// ---- square root: RTF1, RPF1.1 ---------------------------------------------

template <typename T>
__device__ __forceinline__ Pair<T> sqrt_t(T x0, T x1) {
    const T q = sqrt_rn(x0);
    const Pair<T> u = two_sum(x0, x1);             // renormalised argument
    const T v0 = sqrt_rn(u.hi);
    const T h = fma_rn(-v0, v0, u.hi);             // exact residual of v0
    const T v1 = (u.lo + h) / (T(2) * v0);         // one Newton step (RPF1)
    const Pair<T> w = sub_td(v0, v1, q);           // (v0 + v1) - z0 by STF1.1
    return {q, w.hi + w.lo};
}
template <typename T>
__device__ __forceinline__ Pair<T> sqrt_d(T x0) {
    const T q = sqrt_rn(x0);
    const T h = fma_rn(-q, q, x0);
    return {q, h / (T(2) * q)};
}

// ---- coupled ("p") algorithms and renormalisation ----------------------------
// For coupled operands (|x1| at most half an ulp of x0) the p-algorithms
// drop what is negligible; Fast Two-Sum renormalises a result (Dekker mode).

// Fast Two-Sum, Algorithm 1.1: exact when |a| >= |b|.
template <typename T>
__device__ __forceinline__ Pair<T> fast_two_sum(T a, T b) {
    const T s = a + b;
    const T bb = s - a;            // b as it survives inside s
    return {s, b - bb};
}
// MPF1: MTF1 without x1 y1; z1 = e00 (+) (p01 (+) p10).
template <typename T>
__device__ __forceinline__ Pair<T> mul_pp(T x0, T x1, T y0, T y1) {
    const Pair<T> p = two_prod(x0, y0);
    const T cross = x0 * y1 + x1 * y0;
    return {p.hi, p.lo + cross};
}
// DPF1: DTF1 dividing by y0 alone; z1 = (r0 (+) r1) (/) y0.
template <typename T>
__device__ __forceinline__ Pair<T> div_pp(T x0, T x1, T y0, T y1) {
    const T q = x0 / y0;
    const T r0 = fma_rn(-q, y0, x0);
    const T r1 = fma_rn(-q, y1, x1);
    return {q, (r0 + r1) / y0};
}
// RPF1: one Newton step from sqrt(x0), z1 = (x1 (+) (x0 - z0^2)) (/) (2 z0).
template <typename T>
__device__ __forceinline__ Pair<T> sqrt_p(T x0, T x1) {
    const T q = sqrt_rn(x0);
    const T h = fma_rn(-q, q, x0);
    return {q, (x1 + h) / (T(2) * q)};
}

// ---- twofold fma: z = x y + w (an extension of the paper's operations) --------
// z0 = fma(x0, y0, w0).  The error of that fma is rounded with Boldo and
// Muller's ErrFma steps (the exact error is r2 + r3 with r2 its rounded
// value): (u1, u2) = TP(x0, y0); (a1, a2) = TS(w0, u2); (b1, b2) = TS(u1, a1);
// r2 = ((b1 - z0) + b2) + a2.  The low-part terms follow MTF1, then w1.
template <typename T, bool XT, bool YT, bool WT>
__device__ __forceinline__ Pair<T> fma_t(T x0, T x1, T y0, T y1, T w0, T w1) {
    const T z0 = fma_rn(x0, y0, w0);
    const Pair<T> u = two_prod(x0, y0);
    const Pair<T> a = two_sum(w0, u.lo);
    const Pair<T> b = two_sum(u.hi, a.hi);
    T t = ((b.hi - z0) + b.lo) + a.lo;
    if constexpr (XT && YT) t = (t + x1 * y1) + (x0 * y1 + x1 * y0);
    else if constexpr (XT) t = t + x1 * y0;
    else if constexpr (YT) t = t + x0 * y1;
    if constexpr (WT) t = t + w1;
    return {z0, t};
}

}  // namespace tf
