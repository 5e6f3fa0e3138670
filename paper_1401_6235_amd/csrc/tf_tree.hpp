// The fixed pairwise reduction tree, device side: one 256-leaf tile per
// wave and a binary counter for aligned groups of tiles.  Used by the
// reduction kernels and by the serving kernel, so both evaluate the same
// tree bit for bit.
//
// One wave reduces one tile: lane l holds leaves 4l .. 4l+3 (one 16-byte
// load for binary32, two for binary64), forms tree levels 1-2 in registers
// and levels 3-8 with a butterfly over the lanes (xor 1..32); both lanes of
// a pair evaluate the node with the same left/right order, so all 64 lanes
// end with identical bits.
#pragma once

#include "tf_internal.hpp"

namespace tf {

constexpr int kTile = 256;

template <int LEAF>
struct LeafTraits {
    static constexpr bool plain = LEAF == LEAF_PSUM || LEAF == LEAF_PDOT;
    static constexpr bool has_x1 = LEAF == LEAF_SUM_T || LEAF == LEAF_DOT_TT || LEAF == LEAF_DOT_TD;
    static constexpr bool has_y0 = LEAF >= LEAF_DOT_DD && LEAF != LEAF_PSUM;
    static constexpr bool has_y1 = LEAF == LEAF_DOT_TT || LEAF == LEAF_DOT_DT;
};

// A tree node: ATF1 of the left and right child, or the plain sum.
template <typename T, bool PLAIN>
__device__ __forceinline__ Pair<T> node(const Pair<T> &l, const Pair<T> &r) {
    if constexpr (PLAIN) return {l.hi + r.hi, T(0)};
    else return add_tt(l.hi, l.lo, r.hi, r.lo);
}

template <typename T, int LEAF>
__device__ __forceinline__ Pair<T> leaf(T a0, T a1, T b0, T b1) {
    if constexpr (LEAF == LEAF_SUM_T) return {a0, a1};
    else if constexpr (LEAF == LEAF_DOT_DD) return two_prod(a0, b0);
    else if constexpr (LEAF == LEAF_DOT_TT) return mul_tt(a0, a1, b0, b1);
    else if constexpr (LEAF == LEAF_DOT_TD) return mul_td(a0, a1, b0);
    else if constexpr (LEAF == LEAF_DOT_DT) return mul_dt(a0, b0, b1);
    else if constexpr (LEAF == LEAF_PDOT) return {a0 * b0, T(0)};
    else return {a0, T(0)};
}

// Four consecutive values starting at `first` (a multiple of 4); values at
// or beyond n read as +0.
template <typename T>
__device__ __forceinline__ void load4(const T *p, int64_t first, int64_t n, bool vec, T v[4]) {
    if (vec) {
        if constexpr (sizeof(T) == 8) {
            const typename Vec<T>::type a = vload(p, first / 2), b = vload(p, first / 2 + 1);
            v[0] = a[0];
            v[1] = a[1];
            v[2] = b[0];
            v[3] = b[1];
        } else {
            const typename Vec<T>::type a = vload(p, first / 4);
            v[0] = a[0];
            v[1] = a[1];
            v[2] = a[2];
            v[3] = a[3];
        }
    } else {
#pragma unroll
        for (int k = 0; k < 4; ++k) v[k] = first + k < n ? p[first + k] : T(0);
    }
}

// Binary64 tiles other than dotted sums load each half of the tile with
// one contiguous 16-byte-per-lane instruction (measured faster on MI355X
// than four consecutive leaves per lane, which strides lanes by 32 bytes).
#ifndef TF_RED_HALVES
#define TF_RED_HALVES 1
#endif

// Butterfly over the 64 lanes: after step d (1, 2, .., 32) every lane holds
// the node joining its group of 2d lanes; the lower group is the left child.
template <typename T, bool PLAIN>
__device__ __forceinline__ Pair<T> butterfly(Pair<T> v, int lane) {
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        Pair<T> o;
        o.hi = __shfl_xor(v.hi, d);
        o.lo = PLAIN ? T(0) : __shfl_xor(v.lo, d);
        const bool left = (lane & d) == 0;
        const Pair<T> l{left ? v.hi : o.hi, left ? v.lo : o.lo};
        const Pair<T> r{left ? o.hi : v.hi, left ? o.lo : v.lo};
        v = node<T, PLAIN>(l, r);
    }
    return v;
}

// Two consecutive values starting at `first` (even); beyond n read as +0.
template <typename T>
__device__ __forceinline__ void load2(const T *p, int64_t first, int64_t n, bool vec, T v[2]) {
    if (vec) {
        const typename Vec<T>::type a = vload(p, first / 2);
        v[0] = a[0];
        v[1] = a[1];
    } else {
        v[0] = first < n ? p[first] : T(0);
        v[1] = first + 1 < n ? p[first + 1] : T(0);
    }
}

// Level-1 node over leaves (a, b) of a tile.
template <typename T, int LEAF>
__device__ __forceinline__ Pair<T> level1(const T a0[], const T a1[], const T b0[], const T b1[], int i) {
    using Tr = LeafTraits<LEAF>;
    if constexpr (LEAF == LEAF_SUM_D) return two_sum(a0[i], a0[i + 1]);
    else return node<T, Tr::plain>(leaf<T, LEAF>(a0[i], a1[i], b0[i], b1[i]),
                                   leaf<T, LEAF>(a0[i + 1], a1[i + 1], b0[i + 1], b1[i + 1]));
}

// Value of one 256-leaf tile, identical in every lane of the wave.
template <typename T, int LEAF>
__device__ __forceinline__ Pair<T> tile_value(int64_t tile, int64_t n, bool aligned, const T *x0,
                                              const T *x1, const T *y0, const T *y1) {
    using Tr = LeafTraits<LEAF>;
    const int lane = threadIdx.x & 63;
    const bool vec = aligned && (tile + 1) * kTile <= n;
    if constexpr (sizeof(T) == 8 && TF_RED_HALVES && LEAF != LEAF_SUM_D) {
        // binary64, each 16-byte load instruction contiguous over the wave:
        // lane l holds leaves 2l, 2l+1 of each half of the tile; level 1 in
        // registers, levels 2-7 by one butterfly per half, level 8 joins
        // the halves.
        Pair<T> h[2];
#pragma unroll
        for (int k = 0; k < 2; ++k) {
            const int64_t first = tile * kTile + 128 * k + 2 * lane;
            T a0[2], a1[2] = {}, b0[2] = {}, b1[2] = {};
            load2(x0, first, n, vec, a0);
            if constexpr (Tr::has_x1) load2(x1, first, n, vec, a1);
            if constexpr (Tr::has_y0) load2(y0, first, n, vec, b0);
            if constexpr (Tr::has_y1) load2(y1, first, n, vec, b1);
            h[k] = level1<T, LEAF>(a0, a1, b0, b1, 0);
        }
#pragma unroll
        for (int k = 0; k < 2; ++k) h[k] = butterfly<T, Tr::plain>(h[k], lane);
        return node<T, Tr::plain>(h[0], h[1]);
    } else {
        const int64_t first = tile * kTile + 4 * lane;
        T a0[4], a1[4] = {}, b0[4] = {}, b1[4] = {};
        load4(x0, first, n, vec, a0);
        if constexpr (Tr::has_x1) load4(x1, first, n, vec, a1);
        if constexpr (Tr::has_y0) load4(y0, first, n, vec, b0);
        if constexpr (Tr::has_y1) load4(y1, first, n, vec, b1);
        const Pair<T> m0 = level1<T, LEAF>(a0, a1, b0, b1, 0);
        const Pair<T> m1 = level1<T, LEAF>(a0, a1, b0, b1, 2);
        return butterfly<T, Tr::plain>(node<T, Tr::plain>(m0, m1), lane);
    }
}

// Binary counter over consecutive subtree values: after the values of an
// aligned power-of-two group have been pushed in index order, slot[log2 m]
// holds their pairwise-tree value.  Uniform control flow.
template <typename T, bool PLAIN, int SLOTS>
struct Counter {
    Pair<T> slot[SLOTS];
    __device__ __forceinline__ void push(int64_t t, Pair<T> v) {
        bool placed = false;
#pragma unroll
        for (int k = 0; k < SLOTS; ++k) {
            if (!placed) {
                if ((t >> k) & 1) {
                    v = node<T, PLAIN>(slot[k], v);
                } else {
                    slot[k] = v;
                    placed = true;
                }
            }
        }
    }
    __device__ __forceinline__ Pair<T> result(int log2m) const {
        Pair<T> r = slot[0];
#pragma unroll
        for (int k = 1; k < SLOTS; ++k)
            if (log2m == k) r = slot[k];
        return r;
    }
};

__device__ __forceinline__ int ilog2(int64_t v) { return 63 - __clzll(v); }

// Value of the aligned subtree of `per_block` tiles (a power of two) that
// starts at tile b * per_block, computed by one block of 4 waves; valid in
// thread 0.  Each wave folds per_block / 4 consecutive tiles (or one) with a
// binary counter and thread 0 joins the wave results.  Tiles at or beyond
// `tiles` are (+0, +0).  Contains __syncthreads: call from every thread.
template <typename T, int LEAF>
__device__ __forceinline__ Pair<T> block_subtree(int64_t b, int per_block, int64_t n, int64_t tiles,
                                                 bool aligned, const T *x0, const T *x1, const T *y0,
                                                 const T *y1) {
    constexpr bool PLAIN = LeafTraits<LEAF>::plain;
    __shared__ Pair<T> wres[4];
    const int wave = threadIdx.x >> 6;
    const int per_wave = per_block >= 4 ? per_block / 4 : 1;
    const int waves = per_block / per_wave;
    if (wave < waves) {
        const int64_t t0 = b * per_block + (int64_t)wave * per_wave;
        Counter<T, PLAIN, 5> acc;
        for (int t = 0; t < per_wave; ++t) {
            const int64_t tile = t0 + t;
            const Pair<T> v = tile < tiles ? tile_value<T, LEAF>(tile, n, aligned, x0, x1, y0, y1)
                                           : Pair<T>{T(0), T(0)};
            acc.push(t, v);
        }
        if ((threadIdx.x & 63) == 0) wres[wave] = acc.result(ilog2(per_wave));
    }
    __syncthreads();
    Pair<T> r = wres[0];
    if (waves == 2) r = node<T, PLAIN>(wres[0], wres[1]);
    if (waves == 4) r = node<T, PLAIN>(node<T, PLAIN>(wres[0], wres[1]), node<T, PLAIN>(wres[2], wres[3]));
    __syncthreads();
    return r;
}

// Join of the aligned group of group * active partials (powers of two)
// starting at b * group * active: each of the first `active` threads folds
// `group` consecutive partials with a binary counter, then the block pairs
// the thread results level by level.  Partials at index >= count are
// (+0, +0).  Valid in thread 0; call from every thread.
template <typename T, bool PLAIN>
__device__ __forceinline__ Pair<T> block_join(int64_t b, int64_t count, int group, int active,
                                              const Pair<T> *in) {
    __shared__ Pair<T> s[kBlock];
    const int t = threadIdx.x;
    Pair<T> v{T(0), T(0)};
    if (t < active) {
        const int64_t first = (b * active + t) * group;
        Counter<T, PLAIN, 7> acc;
        for (int k = 0; k < group; ++k) {
            const int64_t i = first + k;
            acc.push(k, i < count ? in[i] : Pair<T>{T(0), T(0)});
        }
        v = acc.result(ilog2(group));
    }
    s[t] = v;
    __syncthreads();
    for (int w = active; w > 1; w >>= 1) {
        Pair<T> r{T(0), T(0)};
        if (t < w / 2) r = node<T, PLAIN>(s[2 * t], s[2 * t + 1]);
        __syncthreads();
        if (t < w / 2) s[t] = r;
        __syncthreads();
    }
    const Pair<T> r = s[0];
    __syncthreads();
    return r;
}

}  // namespace tf
