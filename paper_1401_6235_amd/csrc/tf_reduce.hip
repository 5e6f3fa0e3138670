// Twofold sum and dot over the fixed pairwise tree.
//
// The tree is defined by element indices only (tiles of 256 leaves, complete
// adjacent pairing inside a tile, tile results paired the same way up to a
// power of two), so every launch geometry below evaluates the very same
// tree and the result is bitwise reproducible.
//
// Mapping onto gfx950:
//   * one wave reduces one tile: lane l holds leaves 4l .. 4l+3 (one 16-byte
//     load for binary32, two for binary64), forms tree levels 1-2 in
//     registers and levels 3-8 with a butterfly over the lanes (xor 1..32);
//     both lanes of a pair evaluate the node with the same left/right
//     order, so all 64 lanes end with identical bits;
//   * one block of 4 waves reduces an aligned group of `per_block` tiles
//     (a subtree): each wave folds its consecutive tiles with a binary
//     counter (subtrees of 1, 2, 4, ... tiles merged as they complete), and
//     thread 0 joins the (at most 4) wave results;
//   * the per-block partials are joined by the same pairing in one more
//     pass (a second pass only when there are more than 16384 of them).
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

// Value of one 256-leaf tile, identical in every lane of the wave.
template <typename T, int LEAF>
__device__ __forceinline__ Pair<T> tile_value(int64_t tile, int64_t n, bool aligned, const T *x0,
                                              const T *x1, const T *y0, const T *y1) {
    using Tr = LeafTraits<LEAF>;
    const int lane = threadIdx.x & 63;
    const int64_t first = tile * kTile + 4 * lane;
    const bool vec = aligned && (tile + 1) * kTile <= n;
    T a0[4], a1[4] = {}, b0[4] = {}, b1[4] = {};
    load4(x0, first, n, vec, a0);
    if constexpr (Tr::has_x1) load4(x1, first, n, vec, a1);
    if constexpr (Tr::has_y0) load4(y0, first, n, vec, b0);
    if constexpr (Tr::has_y1) load4(y1, first, n, vec, b1);

    Pair<T> m0, m1;
    if constexpr (LEAF == LEAF_SUM_D) {
        m0 = two_sum(a0[0], a0[1]);
        m1 = two_sum(a0[2], a0[3]);
    } else {
        m0 = node<T, Tr::plain>(leaf<T, LEAF>(a0[0], a1[0], b0[0], b1[0]),
                                leaf<T, LEAF>(a0[1], a1[1], b0[1], b1[1]));
        m1 = node<T, Tr::plain>(leaf<T, LEAF>(a0[2], a1[2], b0[2], b1[2]),
                                leaf<T, LEAF>(a0[3], a1[3], b0[3], b1[3]));
    }
    Pair<T> v = node<T, Tr::plain>(m0, m1);
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        Pair<T> o;
        o.hi = __shfl_xor(v.hi, d);
        o.lo = Tr::plain ? T(0) : __shfl_xor(v.lo, d);
        const bool left = (lane & d) == 0;
        const Pair<T> l{left ? v.hi : o.hi, left ? v.lo : o.lo};
        const Pair<T> r{left ? o.hi : v.hi, left ? o.lo : v.lo};
        v = node<T, Tr::plain>(l, r);
    }
    return v;
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

template <typename T>
__device__ __forceinline__ void write_out(T *out, const Pair<T> &v, bool plain) {
    out[0] = v.hi;
    if (!plain) out[1] = v.lo;
}

// Tiles -> one partial per block (or the final result when there is one).
template <typename T, int LEAF>
__global__ __launch_bounds__(kBlock) void reduce_tiles_kernel(int64_t n, int64_t tiles, int per_block,
                                                              int aligned, const T *x0, const T *x1,
                                                              const T *y0, const T *y1,
                                                              Pair<T> *partial, T *out) {
    constexpr bool PLAIN = LeafTraits<LEAF>::plain;
    __shared__ Pair<T> wres[4];
    const int wave = threadIdx.x >> 6;
    const int per_wave = per_block >= 4 ? per_block / 4 : 1;
    const int waves = per_block / per_wave;
    if (wave < waves) {
        const int64_t t0 = (int64_t)blockIdx.x * per_block + (int64_t)wave * per_wave;
        Counter<T, PLAIN, 5> acc;
        for (int t = 0; t < per_wave; ++t) {
            const int64_t tile = t0 + t;
            const Pair<T> v = tile < tiles ? tile_value<T, LEAF>(tile, n, aligned != 0, x0, x1, y0, y1)
                                           : Pair<T>{T(0), T(0)};
            acc.push(t, v);
        }
        if ((threadIdx.x & 63) == 0) wres[wave] = acc.result(ilog2(per_wave));
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        Pair<T> r = wres[0];
        if (waves == 2) r = node<T, PLAIN>(wres[0], wres[1]);
        if (waves == 4) r = node<T, PLAIN>(node<T, PLAIN>(wres[0], wres[1]), node<T, PLAIN>(wres[2], wres[3]));
        if (out) write_out(out, r, PLAIN);
        else partial[blockIdx.x] = r;
    }
}

// Partials -> partials of the next level: block b joins the aligned group of
// group * active partials starting at b * group * active; each thread folds
// `group` consecutive partials, then the block pairs the thread results.
// Partials at index >= count are (+0, +0).
template <typename T, bool PLAIN>
__global__ __launch_bounds__(kBlock) void reduce_partials_kernel(int64_t count, int group, int active,
                                                                 const Pair<T> *in, Pair<T> *partial,
                                                                 T *out) {
    __shared__ Pair<T> s[kBlock];
    const int t = threadIdx.x;
    Pair<T> v{T(0), T(0)};
    if (t < active) {
        const int64_t first = ((int64_t)blockIdx.x * active + t) * group;
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
    if (t == 0) {
        if (out) write_out(out, s[0], PLAIN);
        else partial[blockIdx.x] = s[0];
    }
}

static int64_t pow2_ceil(int64_t v) {
    int64_t p = 1;
    while (p < v) p <<= 1;
    return p;
}

RedShape reduce_shape(int64_t n) {
    RedShape s;
    s.tiles = (n + kTile - 1) / kTile;
    const int64_t P = pow2_ceil(s.tiles > 0 ? s.tiles : 1);
    int64_t pb = config().red_tiles_per_block;
    if (pb > P) pb = P;
    s.per_block = pb;
    s.blocks = (s.tiles + pb - 1) / pb;
    s.padded = P / pb;
    return s;
}

template <typename T, int LEAF>
static void launch_reduce(const Launch &L, int64_t n, const T *x0, const T *x1, const T *y0,
                          const T *y1, T *out, Pair<T> *work) {
    constexpr bool PLAIN = LeafTraits<LEAF>::plain;
    if (n == 0) {  // empty: the partial pass over zero partials writes (+0, +0)
        hipLaunchKernelGGL((reduce_partials_kernel<T, PLAIN>), dim3(1), dim3(kBlock), 0, L.stream,
                           (int64_t)0, 1, 1, (const Pair<T> *)nullptr, (Pair<T> *)nullptr, out);
        return;
    }
    const RedShape s = reduce_shape(n);
    const bool single = s.padded == 1;
    hipLaunchKernelGGL((reduce_tiles_kernel<T, LEAF>), dim3((unsigned)s.blocks), dim3(kBlock), 0, L.stream,
                       n, s.tiles, (int)s.per_block, (int)L.aligned, x0, x1, y0, y1, work,
                       single ? out : (T *)nullptr);
    int64_t count = s.blocks, padded = s.padded;
    Pair<T> *src = work;
    while (padded > 1) {
        int64_t group = padded / kBlock;
        if (group < 1) group = 1;
        if (group > 64) group = 64;
        int64_t active = padded / group;
        if (active > kBlock) active = kBlock;
        const int64_t span = group * active;
        const int64_t next_padded = padded / span;
        const int64_t next_count = (count + span - 1) / span;
        Pair<T> *dst = src + count;
        const bool last = next_padded == 1;
        hipLaunchKernelGGL((reduce_partials_kernel<T, PLAIN>), dim3((unsigned)next_count), dim3(kBlock), 0,
                           L.stream, count, (int)group, (int)active, (const Pair<T> *)src, dst,
                           last ? out : (T *)nullptr);
        src = dst;
        count = next_count;
        padded = next_padded;
    }
}

template <typename T>
void run_reduce(const Launch &L, int leaf_kind, int64_t n, const void *x0, const void *x1,
                const void *y0, const void *y1, void *out, void *work) {
    const T *a0 = (const T *)x0, *a1 = (const T *)x1, *b0 = (const T *)y0, *b1 = (const T *)y1;
    T *o = (T *)out;
    Pair<T> *w = (Pair<T> *)work;
    switch (leaf_kind) {
    case LEAF_SUM_D: launch_reduce<T, LEAF_SUM_D>(L, n, a0, a1, b0, b1, o, w); break;
    case LEAF_SUM_T: launch_reduce<T, LEAF_SUM_T>(L, n, a0, a1, b0, b1, o, w); break;
    case LEAF_DOT_DD: launch_reduce<T, LEAF_DOT_DD>(L, n, a0, a1, b0, b1, o, w); break;
    case LEAF_DOT_TT: launch_reduce<T, LEAF_DOT_TT>(L, n, a0, a1, b0, b1, o, w); break;
    case LEAF_DOT_TD: launch_reduce<T, LEAF_DOT_TD>(L, n, a0, a1, b0, b1, o, w); break;
    case LEAF_DOT_DT: launch_reduce<T, LEAF_DOT_DT>(L, n, a0, a1, b0, b1, o, w); break;
    case LEAF_PSUM: launch_reduce<T, LEAF_PSUM>(L, n, a0, a1, b0, b1, o, w); break;
    default: launch_reduce<T, LEAF_PDOT>(L, n, a0, a1, b0, b1, o, w); break;
    }
}
template void run_reduce<double>(const Launch &, int, int64_t, const void *, const void *, const void *,
                                 const void *, void *, void *);
template void run_reduce<float>(const Launch &, int, int64_t, const void *, const void *, const void *,
                                const void *, void *, void *);

}  // namespace tf
