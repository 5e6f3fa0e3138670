// Kernel templates and launch helpers shared by the library's translation
// units (elementwise, streaming, reductions).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "tf.h"
#include "tf_math.hpp"

namespace tf {

constexpr int kBlock = 256;  // threads per block: 4 waves of 64

// 16-byte vector of T: the unit of every coalesced load and store.
template <typename T>
struct Vec;
template <>
struct Vec<double> {
    typedef double type __attribute__((ext_vector_type(2)));
    static constexpr int N = 2;
};
template <>
struct Vec<float> {
    typedef float type __attribute__((ext_vector_type(4)));
    static constexpr int N = 4;
};

// Streaming data is touched once: non-temporal loads and stores keep it
// from displacing other lines in the caches.
#ifndef TF_NT_LOAD
#define TF_NT_LOAD 1
#endif
#ifndef TF_NT_STORE
#define TF_NT_STORE 1
#endif

template <typename T>
__device__ __forceinline__ typename Vec<T>::type vload(const T *p, int64_t vi) {
    const typename Vec<T>::type *q = reinterpret_cast<const typename Vec<T>::type *>(p) + vi;
#if TF_NT_LOAD
    return __builtin_nontemporal_load(q);
#else
    return *q;
#endif
}
template <typename T>
__device__ __forceinline__ void vstore(T *p, int64_t vi, typename Vec<T>::type v) {
    typename Vec<T>::type *q = reinterpret_cast<typename Vec<T>::type *>(p) + vi;
#if TF_NT_STORE
    __builtin_nontemporal_store(v, q);
#else
    *q = v;
#endif
}

// Operation codes.  0..4 are the twofold operations; 5..7 the coupled
// multiply, divide and square root (MPF1, DPF1, RPF1; coupled add and
// subtract are ATF1 / STF1 themselves); OP_RENORM added to any of these
// passes the result through Fast Two-Sum (Dekker mode); OP_FAST_TWO_SUM
// renormalises the twofold x alone.
enum Op {
    OP_ADD = 0,
    OP_SUB = 1,
    OP_MUL = 2,
    OP_DIV = 3,
    OP_SQRT = 4,
    OP_MUL_P = 5,
    OP_DIV_P = 6,
    OP_SQRT_P = 7,
    OP_RENORM = 8,
    OP_FAST_TWO_SUM = 16,
};

// Operations with one operand.
constexpr bool op_unary(int op) {
    return op == OP_FAST_TWO_SUM || (op & 7) == OP_SQRT || (op & 7) == OP_SQRT_P;
}

// One element of a binary operation; XT / YT: operand is twofold (else
// dotted).  For unary operations only x is used.
template <typename T, int OP, bool XT, bool YT>
__device__ __forceinline__ Pair<T> apply(T x0, T x1, T y0, T y1) {
    if constexpr (OP == OP_FAST_TWO_SUM) {
        return fast_two_sum(x0, x1);
    } else if constexpr ((OP & OP_RENORM) != 0) {
        const Pair<T> z = apply<T, OP & 7, XT, YT>(x0, x1, y0, y1);
        return fast_two_sum(z.hi, z.lo);
    } else if constexpr (OP == OP_MUL_P) {
        if constexpr (XT && YT) return mul_pp(x0, x1, y0, y1);
        else if constexpr (XT) return mul_td(x0, x1, y0);
        else if constexpr (YT) return mul_dt(x0, y0, y1);
        else return mul_dd(x0, y0);
    } else if constexpr (OP == OP_DIV_P) {
        if constexpr (XT && YT) return div_pp(x0, x1, y0, y1);
        else if constexpr (XT) return div_td(x0, x1, y0);
        else if constexpr (YT) return div_pp(x0, T(0), y0, y1);
        else return div_dd(x0, y0);
    } else if constexpr (OP == OP_SQRT_P) {
        if constexpr (XT) return sqrt_p(x0, x1);
        else return sqrt_d(x0);
    } else if constexpr (OP == OP_ADD) {
        if constexpr (XT && YT) return add_tt(x0, x1, y0, y1);
        else if constexpr (XT) return add_td(x0, x1, y0);
        else if constexpr (YT) return add_dt(x0, y0, y1);
        else return add_dd(x0, y0);
    } else if constexpr (OP == OP_SUB) {
        if constexpr (XT && YT) return sub_tt(x0, x1, y0, y1);
        else if constexpr (XT) return sub_td(x0, x1, y0);
        else if constexpr (YT) return sub_dt(x0, y0, y1);
        else return sub_dd(x0, y0);
    } else if constexpr (OP == OP_MUL) {
        if constexpr (XT && YT) return mul_tt(x0, x1, y0, y1);
        else if constexpr (XT) return mul_td(x0, x1, y0);
        else if constexpr (YT) return mul_dt(x0, y0, y1);
        else return mul_dd(x0, y0);
    } else if constexpr (OP == OP_DIV) {
        if constexpr (XT && YT) return div_tt(x0, x1, y0, y1);
        else if constexpr (XT) return div_td(x0, x1, y0);
        else if constexpr (YT) return div_dt(x0, y0, y1);
        else return div_dd(x0, y0);
    } else {
        if constexpr (XT) return sqrt_t(x0, x1);
        else return sqrt_d(x0);
    }
}

template <typename T, int OP>
__device__ __forceinline__ T apply_plain(T x, T y) {
    if constexpr (OP == OP_ADD) return x + y;
    else if constexpr (OP == OP_SUB) return x - y;
    else if constexpr (OP == OP_MUL) return x * y;
    else if constexpr (OP == OP_DIV) return x / y;
    else return sqrt_rn(x);
}

// axpy element: t = MTF1(a, x) (MTF1.1 for dotted x), z = ATF1(t, y)
// (ATF1.1 for dotted y).
template <typename T, bool XT, bool YT>
__device__ __forceinline__ Pair<T> axpy_one(T a0, T a1, T x0, T x1, T y0, T y1) {
    const Pair<T> t = XT ? mul_tt(a0, a1, x0, x1) : mul_td(a0, a1, x0);
    return YT ? add_tt(t.hi, t.lo, y0, y1) : add_td(t.hi, t.lo, y0);
}

// Horner element: r = (c[d], +0); r = ATF1.1(MTF1(r, x), c[k]) for
// k = d-1 .. 0 (MTF1.1 for dotted x).  Coefficients travel by value.
template <typename T>
struct Coeffs {
    T c[TF_MAX_DEGREE + 1];
};

template <typename T, bool XT>
__device__ __forceinline__ Pair<T> horner_one(const Coeffs<T> &C, int degree, T x0, T x1) {
    Pair<T> r{C.c[degree], T(0)};
    for (int k = degree - 1; k >= 0; --k) {
        const Pair<T> m = XT ? mul_tt(r.hi, r.lo, x0, x1) : mul_td(r.hi, r.lo, x0);
        r = add_td(m.hi, m.lo, C.c[k]);
    }
    return r;
}

// Grid for `work` items of `per_block` each, optionally capped (grid-stride
// loops in the kernels cover the rest).
inline unsigned grid_for(int64_t work, int64_t per_block, int64_t cap) {
    int64_t g = (work + per_block - 1) / per_block;
    if (g < 1) g = 1;
    if (cap > 0 && g > cap) g = cap;
    if (g > 0x7fffffff) g = 0x7fffffff;
    return (unsigned)g;
}

}  // namespace tf
