// The fixed pairwise reduction tree, device side.  Used by the reduction
// kernels and by the serving kernel, so both evaluate the same tree bit for
// bit.
//
// Two mappings of 256-leaf tiles onto a wave, chosen by the number of tiles
// a wave reduces:
//  * tile pairs (two or more tiles per wave): a wave takes two adjacent
//    tiles at once, transposes them through LDS so that each lane holds 8
//    consecutive leaves, forms levels 1-3 in registers and levels 4-8 by a
//    butterfly over 32 lanes;
//  * single tiles: lane l holds leaves 4l .. 4l+3 (or two leaves of each
//    half of the tile), levels 1-2 in registers, the rest by a butterfly
//    over the 64 lanes.
// In every butterfly both lanes of a pair evaluate the node with the same
// left/right order, so all lanes end with identical bits; a wave then keeps
// tile t's value in lane t and joins its tiles with one more butterfly.
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
    static constexpr int arrays = 1 + has_x1 + has_y0 + has_y1;
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

// Exchange with lane ^ D.  With TF_RED_DPP, xor 1 and 2 are DPP quad
// permutes (no LDS), xor 4, 8 and 16 ds_swizzle in bit-mask mode (no
// address computation), xor 32 a ds_bpermute; otherwise every distance is
// a ds_bpermute (__shfl_xor).  The value moved is the same either way.
#ifndef TF_RED_DPP
#define TF_RED_DPP 1
#endif

template <int D>
__device__ __forceinline__ int lane_xor_u32(int x) {
#if TF_RED_DPP
    if constexpr (D == 1) return __builtin_amdgcn_update_dpp(0, x, 0xB1, 0xF, 0xF, false);  // [1,0,3,2]
    else if constexpr (D == 2) return __builtin_amdgcn_update_dpp(0, x, 0x4E, 0xF, 0xF, false);  // [2,3,0,1]
    else if constexpr (D < 32) return __builtin_amdgcn_ds_swizzle(x, 0x1F | (D << 10));
    else return __shfl_xor(x, D);
#else
    return __shfl_xor(x, D);
#endif
}

template <int D, typename T>
__device__ __forceinline__ T lane_xor(T v) {
    if constexpr (sizeof(T) == 8) {
        const long long b = __double_as_longlong(v);
        const int lo = lane_xor_u32<D>((int)(b & 0xffffffffll));
        const int hi = lane_xor_u32<D>((int)(b >> 32));
        return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
    } else {
        return __int_as_float(lane_xor_u32<D>(__float_as_int(v)));
    }
}

// One butterfly step at distance D: every lane ends with the node joining
// its group of 2D lanes; the lower group is the left child, so both lanes of
// a pair evaluate the node in the same order and get the same bits.
template <int D, typename T, bool PLAIN>
__device__ __forceinline__ Pair<T> butterfly_step(Pair<T> v, int lane) {
    Pair<T> o;
    o.hi = lane_xor<D>(v.hi);
    o.lo = PLAIN ? T(0) : lane_xor<D>(v.lo);
    const bool left = (lane & D) == 0;
    const Pair<T> l{left ? v.hi : o.hi, left ? v.lo : o.lo};
    const Pair<T> r{left ? o.hi : v.hi, left ? o.lo : v.lo};
    return node<T, PLAIN>(l, r);
}

// Butterfly over the 64 lanes: after step d (1, 2, .., 32) every lane holds
// the node joining its group of 2d lanes.
template <typename T, bool PLAIN>
__device__ __forceinline__ Pair<T> butterfly(Pair<T> v, int lane) {
    v = butterfly_step<1, T, PLAIN>(v, lane);
    v = butterfly_step<2, T, PLAIN>(v, lane);
    v = butterfly_step<4, T, PLAIN>(v, lane);
    v = butterfly_step<8, T, PLAIN>(v, lane);
    v = butterfly_step<16, T, PLAIN>(v, lane);
    return butterfly_step<32, T, PLAIN>(v, lane);
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

// The leaves of one tile held by this lane: binary32 and dotted binary64
// sums hold 4 consecutive leaves (4l .. 4l+3); other binary64 tiles hold
// leaves 2l, 2l+1 of each half of the tile (entries 0, 1 and 2, 3), so each
// 16-byte load instruction is contiguous over the wave.
template <typename T>
struct TileData {
    T a0[4], a1[4], b0[4], b1[4];
};

template <typename T, int LEAF>
constexpr bool halves_layout() {
    return sizeof(T) == 8 && TF_RED_HALVES && LEAF != LEAF_SUM_D;
}

template <typename T, int LEAF>
__device__ __forceinline__ void tile_load(TileData<T> &D, int64_t tile, int64_t n, bool aligned,
                                          const T *x0, const T *x1, const T *y0, const T *y1) {
    using Tr = LeafTraits<LEAF>;
    const int lane = threadIdx.x & 63;
    const bool vec = aligned && (tile + 1) * kTile <= n;
#pragma unroll
    for (int k = 0; k < 4; ++k) D.a1[k] = D.b0[k] = D.b1[k] = T(0);
    if constexpr (halves_layout<T, LEAF>()) {
#pragma unroll
        for (int h = 0; h < 2; ++h) {
            const int64_t first = tile * kTile + 128 * h + 2 * lane;
            load2(x0, first, n, vec, D.a0 + 2 * h);
            if constexpr (Tr::has_x1) load2(x1, first, n, vec, D.a1 + 2 * h);
            if constexpr (Tr::has_y0) load2(y0, first, n, vec, D.b0 + 2 * h);
            if constexpr (Tr::has_y1) load2(y1, first, n, vec, D.b1 + 2 * h);
        }
    } else {
        const int64_t first = tile * kTile + 4 * lane;
        load4(x0, first, n, vec, D.a0);
        if constexpr (Tr::has_x1) load4(x1, first, n, vec, D.a1);
        if constexpr (Tr::has_y0) load4(y0, first, n, vec, D.b0);
        if constexpr (Tr::has_y1) load4(y1, first, n, vec, D.b1);
    }
}

// Tree value of a loaded tile, identical in every lane of the wave.
template <typename T, int LEAF>
__device__ __forceinline__ Pair<T> tile_reduce(const TileData<T> &D) {
    using Tr = LeafTraits<LEAF>;
    const int lane = threadIdx.x & 63;
    if constexpr (halves_layout<T, LEAF>()) {
        // level 1 in registers, levels 2-7 by one butterfly per half (the two
        // are independent and interleave), level 8 joins the halves
        Pair<T> h0 = level1<T, LEAF>(D.a0, D.a1, D.b0, D.b1, 0);
        Pair<T> h1 = level1<T, LEAF>(D.a0, D.a1, D.b0, D.b1, 2);
        h0 = butterfly<T, Tr::plain>(h0, lane);
        h1 = butterfly<T, Tr::plain>(h1, lane);
        return node<T, Tr::plain>(h0, h1);
    } else {
        const Pair<T> m0 = level1<T, LEAF>(D.a0, D.a1, D.b0, D.b1, 0);
        const Pair<T> m1 = level1<T, LEAF>(D.a0, D.a1, D.b0, D.b1, 2);
        return butterfly<T, Tr::plain>(node<T, Tr::plain>(m0, m1), lane);
    }
}

// Value of one 256-leaf tile, identical in every lane of the wave.
template <typename T, int LEAF>
__device__ __forceinline__ Pair<T> tile_value(int64_t tile, int64_t n, bool aligned, const T *x0,
                                              const T *x1, const T *y0, const T *y1) {
    TileData<T> D;
    tile_load<T, LEAF>(D, tile, n, aligned, x0, x1, y0, y1);
    return tile_reduce<T, LEAF>(D);
}

__device__ __forceinline__ int ilog2(int64_t v) { return 63 - __clzll(v); }

// ---- tile groups: 8 (binary64) or 16 (binary32) consecutive leaves per lane
//
// One wave reduces a group of adjacent tiles at once: 2 tiles (512 leaves)
// in binary64, 4 tiles (1024 leaves) in binary32, so every pass reads 4 KiB
// of each array.  Each array is loaded with contiguous 16-byte vectors (lane
// l, vector k: leaves W (64 k + l) ..), passed through a wave-private LDS
// region and read back so that lane l holds leaves LPL l .. LPL l + LPL-1;
// the tree levels inside those leaves are formed in registers and the rest
// of each tile by a butterfly over its 256 / LPL lanes (DPP / swizzle only),
// leaving tile q's value in lanes q * 256 / LPL onwards.  The LDS region has
// one spare vector after every lane's group, spreading the transposed reads
// over the banks.
#ifndef TF_RED_PAIRS
#define TF_RED_PAIRS 1
#endif
#ifndef TF_RED_LDS_PAD
#define TF_RED_LDS_PAD 1
#endif
#ifndef TF_RED_PAIR_ARRAYS
#define TF_RED_PAIR_ARRAYS 2
#endif
#ifndef TF_RED_LPL_F32
#define TF_RED_LPL_F32 16
#endif

template <typename T>
struct PairLayout {
    using V = typename Vec<T>::type;
    static constexpr int W = Vec<T>::N;
    static constexpr int LPL = sizeof(T) == 8 ? 8 : TF_RED_LPL_F32;  // consecutive leaves per lane
    static constexpr int VPL = LPL / W;        // vectors per lane per array
    static constexpr int NV = 64 * VPL;        // vectors per array per pass
    static constexpr int TILES = 64 * LPL / kTile;  // tiles per pass
    static constexpr int LANES = kTile / LPL;       // lanes per tile
    static constexpr int SLOTS = TF_RED_LDS_PAD ? NV + NV / VPL : NV;
    __device__ static int slot(int v) { return TF_RED_LDS_PAD ? v + v / VPL : v; }
};

// One LDS region per kernel and block size, shared by every instantiation
// (one region per wave, sized for the larger of the two layouts).
constexpr int kPairSlots = PairLayout<double>::SLOTS > PairLayout<float>::SLOTS ? PairLayout<double>::SLOTS
                                                                                : PairLayout<float>::SLOTS;
template <int WAVES>
__device__ __forceinline__ void *pair_lds_base() {
    __shared__ __attribute__((aligned(16))) unsigned char buf[WAVES * kPairSlots * 16];
    return buf;
}

template <typename T>
struct PairData {
    typename Vec<T>::type r[4][PairLayout<T>::VPL];  // x0, x1, y0, y1 as loaded
};

template <typename T, int LEAF>
__device__ __forceinline__ void pair_load(PairData<T> &D, int64_t tile, int64_t n, bool aligned, const T *x0,
                                          const T *x1, const T *y0, const T *y1) {
    using Tr = LeafTraits<LEAF>;
    using L = PairLayout<T>;
    const int lane = threadIdx.x & 63;
    const int64_t first = tile * kTile;  // leaf index of the group's first leaf
    const bool vec = aligned && first + L::TILES * kTile <= n;
    const T *src[4] = {x0, x1, y0, y1};
    const bool has[4] = {true, Tr::has_x1, Tr::has_y0, Tr::has_y1};
#pragma unroll
    for (int a = 0; a < 4; ++a) {
        if (!has[a]) continue;
#pragma unroll
        for (int k = 0; k < L::VPL; ++k) {
            const int64_t v = first / L::W + k * 64 + lane;  // vector index
            if (vec) {
                D.r[a][k] = vload(src[a], v);
            } else {
#pragma unroll
                for (int e = 0; e < L::W; ++e) {
                    const int64_t i = v * L::W + e;
                    D.r[a][k][e] = i < n ? src[a][i] : T(0);
                }
            }
        }
    }
}

template <typename T>
__device__ __forceinline__ T readlane_t(T v, int l) {
    if constexpr (sizeof(T) == 8) {
        const long long b = __double_as_longlong(v);
        const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffll), l);
        const int hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
        return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
    } else {
        return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), l));
    }
}

// Values of the tiles of a loaded group: lanes q * L::LANES .. hold tile q's.
// `lds` is this wave's region of L::SLOTS vectors.
template <typename T, int LEAF>
__device__ __forceinline__ Pair<T> pair_reduce(const PairData<T> &D, typename Vec<T>::type *lds) {
    using Tr = LeafTraits<LEAF>;
    using L = PairLayout<T>;
    const int lane = threadIdx.x & 63;
    const bool has[4] = {true, Tr::has_x1, Tr::has_y0, Tr::has_y1};
    T lv[4][L::LPL];
#pragma unroll
    for (int a = 0; a < 4; ++a) {
        if (!has[a]) {
#pragma unroll
            for (int i = 0; i < L::LPL; ++i) lv[a][i] = T(0);
            continue;
        }
#pragma unroll
        for (int k = 0; k < L::VPL; ++k) lds[L::slot(k * 64 + lane)] = D.r[a][k];
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
#pragma unroll
        for (int j = 0; j < L::VPL; ++j) {
            const typename Vec<T>::type v = lds[L::slot(lane * L::VPL + j)];
#pragma unroll
            for (int e = 0; e < L::W; ++e) lv[a][j * L::W + e] = v[e];
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
    // the lane's subtree: level 1 from the leaves, then adjacent pairing
    Pair<T> t[L::LPL / 2];
#pragma unroll
    for (int i = 0; i < L::LPL / 2; ++i) t[i] = level1<T, LEAF>(lv[0], lv[1], lv[2], lv[3], 2 * i);
#pragma unroll
    for (int w = L::LPL / 2; w > 1; w /= 2) {
#pragma unroll
        for (int i = 0; i < w / 2; ++i) t[i] = node<T, Tr::plain>(t[2 * i], t[2 * i + 1]);
    }
    Pair<T> v = t[0];
    if constexpr (L::LANES > 1) v = butterfly_step<1, T, Tr::plain>(v, lane);
    if constexpr (L::LANES > 2) v = butterfly_step<2, T, Tr::plain>(v, lane);
    if constexpr (L::LANES > 4) v = butterfly_step<4, T, Tr::plain>(v, lane);
    if constexpr (L::LANES > 8) v = butterfly_step<8, T, Tr::plain>(v, lane);
    if constexpr (L::LANES > 16) v = butterfly_step<16, T, Tr::plain>(v, lane);
    if constexpr (L::LANES > 32) v = butterfly_step<32, T, Tr::plain>(v, lane);
    return v;
}

// Butterfly over the first m lanes (m a power of two, at most 64): the
// adjacent-pairing tree of the values held by lanes 0 .. m-1, left in each of
// them.  Lanes at or beyond m pair among themselves and are not used.
template <typename T, bool PLAIN>
__device__ __forceinline__ Pair<T> butterfly_m(Pair<T> v, int lane, int m) {
    if (m > 1) v = butterfly_step<1, T, PLAIN>(v, lane);
    if (m > 2) v = butterfly_step<2, T, PLAIN>(v, lane);
    if (m > 4) v = butterfly_step<4, T, PLAIN>(v, lane);
    if (m > 8) v = butterfly_step<8, T, PLAIN>(v, lane);
    if (m > 16) v = butterfly_step<16, T, PLAIN>(v, lane);
    if (m > 32) v = butterfly_step<32, T, PLAIN>(v, lane);
    return v;
}

// Join of the wave results of a block (`waves` a power of two, at most
// MAXW): adjacent pairs, level by level, the same tree as the leaves'.
// Wave w's result is exchanged through LDS at wres[w * stride]; lane k of
// every wave then takes wave k's result and a butterfly over the first
// `waves` lanes forms the tree (one pair per lane in registers, whatever
// MAXW), whose root lane 0 holds and hands to the whole wave.
template <typename T, bool PLAIN, int MAXW>
__device__ __forceinline__ Pair<T> join_waves_via(Pair<T> mine, int waves, Pair<T> *wres, int stride) {
    static_assert(MAXW <= 64, "one wave result per lane");
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    if (wave < waves && lane == 0) wres[wave * stride] = mine;
    __syncthreads();
    Pair<T> v = lane < waves ? wres[lane * stride] : Pair<T>{T(0), T(0)};
    v = butterfly_m<T, PLAIN>(v, lane, waves);
    __syncthreads();
    return Pair<T>{readlane_t(v.hi, 0), readlane_t(v.lo, 0)};
}

template <typename T, bool PLAIN, int MAXW = 4>
__device__ __forceinline__ Pair<T> join_waves(Pair<T> mine, int waves) {
    __shared__ Pair<T> wres[MAXW];
    return join_waves_via<T, PLAIN, MAXW>(mine, waves, wres, 1);
}

// Value of the aligned subtree of `per_block` tiles (a power of two, at most
// 64 * WAVES) that starts at tile b * per_block, computed by one block of
// WAVES waves; valid in thread 0.  Each wave takes per_block / WAVES
// consecutive tiles (or one); lane t keeps the value of the wave's tile t,
// and a butterfly over those lanes gives the wave's subtree.  Tiles at or
// beyond `tiles` are (+0, +0).  Contains __syncthreads: call from every
// thread.
// ONE_PASS: every wave reduces exactly one group of tile pairs (per_block ==
// WAVES * PairLayout<T>::TILES, leaves from at most two arrays); the
// pipelined loop and its second buffer are left out, which frees registers
// for more waves per SIMD.  PIPE = false keeps the loop but not the second
// buffer (each group or tile loaded when it is reached), for callers whose
// register budget is tight.
template <typename T, int LEAF, int WAVES = 4, bool ONE_PASS = false, bool PIPE = true>
__device__ __forceinline__ Pair<T> block_subtree(int64_t b, int per_block, int64_t n, int64_t tiles,
                                                 bool aligned, const T *x0, const T *x1, const T *y0,
                                                 const T *y1) {
    constexpr bool PLAIN = LeafTraits<LEAF>::plain;
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int per_wave = per_block >= WAVES ? per_block / WAVES : 1;
    const int waves = per_block / per_wave;
    Pair<T> mine{T(0), T(0)};
    // Where a kernel has the tile-pair LDS region, each wave hands its result
    // to the join through the start of its own region (which it no longer
    // needs): no separate LDS array, so 8-wave blocks take exactly 40 KiB and
    // four fit in a compute unit's 160 KiB.
    constexpr bool PAIR_LDS = TF_RED_PAIRS && LeafTraits<LEAF>::arrays <= TF_RED_PAIR_ARRAYS;
    auto join = [&](Pair<T> m, int w) {
        if constexpr (PAIR_LDS)
            return join_waves_via<T, PLAIN, WAVES>(m, w, reinterpret_cast<Pair<T> *>(pair_lds_base<WAVES>()),
                                                   (int)(PairLayout<T>::SLOTS * 16 / sizeof(Pair<T>)));
        else
            return join_waves<T, PLAIN, WAVES>(m, w);
    };
#if TF_RED_PAIRS
    // Tile pairs pay off where the tree dominates the per-leaf work: leaves
    // read from one or two arrays (sums, dot of plain vectors).  Leaves with
    // three or four input arrays (twofold products) are already near the
    // read bandwidth on single tiles, and the extra transposes cost more
    // than the saved tree levels (measured on MI355X).
    using PL = PairLayout<T>;
    if (LeafTraits<LEAF>::arrays <= TF_RED_PAIR_ARRAYS && per_wave >= PL::TILES) {  // per_wave: a power of two
        typename Vec<T>::type *lds =
            reinterpret_cast<typename Vec<T>::type *>(pair_lds_base<WAVES>()) + wave * PL::SLOTS;
        const int64_t t0 = b * per_block + (int64_t)wave * per_wave;
        if constexpr (ONE_PASS) {
            if (t0 < tiles) {
                PairData<T> cur;
                pair_load<T, LEAF>(cur, t0, n, aligned, x0, x1, y0, y1);
                const Pair<T> v = pair_reduce<T, LEAF>(cur, lds);
#pragma unroll
                for (int q = 0; q < PL::TILES; ++q) {
                    const Pair<T> val{readlane_t(v.hi, q * PL::LANES), readlane_t(v.lo, q * PL::LANES)};
                    if (lane == q && t0 + q < tiles) mine = val;
                }
            }
            mine = butterfly_m<T, PLAIN>(mine, lane, PL::TILES);
            return join(mine, waves);
        }
        if constexpr (!PIPE) {
            for (int p = 0; PL::TILES * p < per_wave; ++p) {
                const int64_t tile = t0 + PL::TILES * p;
                if (tile < tiles) {
                    PairData<T> cur;
                    pair_load<T, LEAF>(cur, tile, n, aligned, x0, x1, y0, y1);
                    const Pair<T> v = pair_reduce<T, LEAF>(cur, lds);
#pragma unroll
                    for (int q = 0; q < PL::TILES; ++q) {
                        const Pair<T> val{readlane_t(v.hi, q * PL::LANES), readlane_t(v.lo, q * PL::LANES)};
                        if (lane == PL::TILES * p + q && tile + q < tiles) mine = val;
                    }
                }
            }
            mine = butterfly_m<T, PLAIN>(mine, lane, per_wave);
            return join(mine, waves);
        }
        // the next group's loads are in flight while the current one is reduced
        PairData<T> cur, nxt;
        if (t0 < tiles) pair_load<T, LEAF>(cur, t0, n, aligned, x0, x1, y0, y1);
        for (int p = 0; PL::TILES * p < per_wave; ++p) {
            const int64_t tile = t0 + PL::TILES * p;
            if (PL::TILES * (p + 1) < per_wave && tile + PL::TILES < tiles)
                pair_load<T, LEAF>(nxt, tile + PL::TILES, n, aligned, x0, x1, y0, y1);
            if (tile < tiles) {
                const Pair<T> v = pair_reduce<T, LEAF>(cur, lds);
#pragma unroll
                for (int q = 0; q < PL::TILES; ++q) {
                    const Pair<T> val{readlane_t(v.hi, q * PL::LANES), readlane_t(v.lo, q * PL::LANES)};
                    if (lane == PL::TILES * p + q && tile + q < tiles) mine = val;
                }
            }
            cur = nxt;
        }
        mine = butterfly_m<T, PLAIN>(mine, lane, per_wave);
        return join(mine, waves);
    }
#endif
    if (!PIPE && wave < waves) {
        const int64_t t0 = b * per_block + (int64_t)wave * per_wave;
        for (int t = 0; t < per_wave; ++t) {
            const int64_t tile = t0 + t;
            if (tile < tiles) {
                TileData<T> cur;
                tile_load<T, LEAF>(cur, tile, n, aligned, x0, x1, y0, y1);
                const Pair<T> v = tile_reduce<T, LEAF>(cur);
                if (lane == t) mine = v;
            }
        }
        mine = butterfly_m<T, PLAIN>(mine, lane, per_wave);
    } else if (wave < waves) {
        const int64_t t0 = b * per_block + (int64_t)wave * per_wave;
        // software pipeline: the next tile's loads are in flight while the
        // current tile is reduced
        TileData<T> cur, nxt;
        if (t0 < tiles) tile_load<T, LEAF>(cur, t0, n, aligned, x0, x1, y0, y1);
        for (int t = 0; t < per_wave; ++t) {
            const int64_t tile = t0 + t;
            if (t + 1 < per_wave && tile + 1 < tiles)
                tile_load<T, LEAF>(nxt, tile + 1, n, aligned, x0, x1, y0, y1);
            if (tile < tiles) {
                const Pair<T> v = tile_reduce<T, LEAF>(cur);
                if (lane == t) mine = v;
            }
            cur = nxt;
        }
        mine = butterfly_m<T, PLAIN>(mine, lane, per_wave);
    }
    return join(mine, waves);
}

// Join of the aligned group of `span` partials (a power of two, at most
// WAVES * 64 * 64) starting at b * span; partials at index >= count are
// (+0, +0).  Each of the block's WAVES waves takes span / WAVES consecutive
// partials (or one) and folds them in chunks of 64 K: lane l loads K
// consecutive partials of the chunk (K a power of two, at most KMAX) and
// forms their subtree in registers, a butterfly joins the 64 lanes, and lane
// j keeps chunk j until a last butterfly joins the chunks.  Every subtree is
// aligned, so the tree is the same for any WAVES and KMAX.  Valid in thread
// 0.  Call from every thread.
template <typename T, bool PLAIN, int WAVES = 4, int KMAX = 8>
__device__ __forceinline__ Pair<T> block_join(int64_t b, int64_t count, int64_t span, const Pair<T> *in) {
    const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
    const int64_t per_wave = span >= WAVES ? span / WAVES : 1;
    const int waves = (int)(span / per_wave);
    Pair<T> mine{T(0), T(0)};
    if (wave < waves && count > 0) {  // count == 0: every partial is zero (and `in` may be NULL)
        const int64_t first = b * span + (int64_t)wave * per_wave;
        const int64_t width = per_wave < 64 ? per_wave : 64;  // lanes per chunk
        const int64_t runs = per_wave / width;                 // partials per lane over the wave
        const int K = runs < KMAX ? (int)runs : KMAX;
        const int64_t chunk = width * K;
        const int64_t chunks = per_wave / chunk;
        for (int64_t j = 0; j < chunks; ++j) {
            const int64_t base = first + j * chunk + (int64_t)lane * K;
            // every load is issued (an absent partial reads partial 0 and is
            // replaced by zero), so all KMAX are in flight together
            Pair<T> v[KMAX];
#pragma unroll
            for (int q = 0; q < KMAX; ++q) {
                const int64_t i = base + q;
                const bool ok = q < K && lane < width && i < count;
                const Pair<T> p = in[ok ? i : 0];
                v[q] = ok ? p : Pair<T>{T(0), T(0)};
            }
#pragma unroll
            for (int w = KMAX; w > 1; w >>= 1) {
                if (w <= K) {
#pragma unroll
                    for (int q = 0; q < w / 2; ++q) v[q] = node<T, PLAIN>(v[2 * q], v[2 * q + 1]);
                }
            }
            const Pair<T> r = butterfly_m<T, PLAIN>(v[0], lane, (int)width);
            if (lane == j || chunks == 1) mine = r;
        }
        mine = butterfly_m<T, PLAIN>(mine, lane, (int)chunks);
    }
    return join_waves<T, PLAIN, WAVES>(mine, waves);
}

}  // namespace tf
