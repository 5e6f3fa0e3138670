// Kernel templates and launch helpers shared by the library's translation
// units (elementwise, streaming, reductions).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

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

template <typename T>
__device__ __forceinline__ typename Vec<T>::type vload(const T *p, int64_t vi) {
    return __builtin_nontemporal_load(reinterpret_cast<const typename Vec<T>::type *>(p) + vi);
}
template <typename T>
__device__ __forceinline__ void vstore(T *p, int64_t vi, typename Vec<T>::type v) {
    __builtin_nontemporal_store(v, reinterpret_cast<typename Vec<T>::type *>(p) + vi);
}

enum Op { OP_ADD = 0, OP_SUB = 1, OP_MUL = 2, OP_DIV = 3, OP_SQRT = 4 };

// One element of a binary operation; XT / YT: operand is twofold (else
// dotted).  For OP_SQRT only x is used.
template <typename T, int OP, bool XT, bool YT>
__device__ __forceinline__ Pair<T> apply(T x0, T x1, T y0, T y1) {
    if constexpr (OP == OP_ADD) {
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
