// Twofold sum and dot over the fixed pairwise tree.
//
// The tree is defined by element indices only (tiles of 256 leaves, complete
// adjacent pairing inside a tile, tile results paired the same way up to a
// power of two), so every launch geometry below evaluates the very same
// tree and the result is bitwise reproducible.
//
// Mapping onto gfx950:
//   * one wave reduces one tile, or a group of two (binary64) or four
//     (binary32) adjacent tiles at a time (tf_tree.hpp);
//   * one block of 4, 8 or 16 waves reduces an aligned group of
//     `per_block` tiles (a subtree): each wave takes per_block / waves
//     consecutive tiles, lane t keeps the value of the wave's tile t and a
//     butterfly finishes the wave's aligned group; the waves' results meet
//     in LDS and one more butterfly joins them, so every tree level above
//     the leaves stays in registers;
//   * the per-block partials are joined by the same pairing in one more
//     pass, one block of 16 waves (middle passes only past 65536 of them).
#include "tf_tree.hpp"


// First-pass waves keep the next tile group's loads in flight while the
// current one is reduced (1), or load each group when reached (0: 65
// instead of 100 VGPRs in binary64, so seven blocks per CU instead of four;
// 0-3 % faster on every leaf kind, measured on MI355X).
#ifndef TF_RED_PIPE
#define TF_RED_PIPE 0
#endif

namespace tf {

template <typename T>
__device__ __forceinline__ void write_out(T *out, const Pair<T> &v, bool plain) {
    out[0] = v.hi;
    if (!plain) out[1] = v.lo;
}

// Tiles -> one partial per block (or the final result when there is one),
// blocks of WAVES waves.
template <typename T, int LEAF, int WAVES, bool ONE_PASS>
__global__ __launch_bounds__(64 * WAVES) void reduce_tiles_kernel(int64_t n, int64_t tiles, int per_block,
                                                                  int aligned, const T *x0, const T *x1,
                                                                  const T *y0, const T *y1,
                                                                  Pair<T> *partial, T *out) {
    constexpr bool PLAIN = LeafTraits<LEAF>::plain;
    const Pair<T> r = block_subtree<T, LEAF, WAVES, ONE_PASS, TF_RED_PIPE>(blockIdx.x, per_block, n, tiles,
                                                                          aligned != 0,
                                                              x0, x1, y0, y1);
    if (threadIdx.x == 0) {
        if (out) write_out(out, r, PLAIN);
        else partial[blockIdx.x] = r;
    }
}

// Partials -> partials of the next level (see block_join).
template <typename T, bool PLAIN>
__global__ __launch_bounds__(kBlock) void reduce_partials_kernel(int64_t count, int64_t span,
                                                                 const Pair<T> *in, Pair<T> *partial,
                                                                 T *out) {
    const Pair<T> r = block_join<T, PLAIN>(blockIdx.x, count, span, in);
    if (threadIdx.x == 0) {
        if (out) write_out(out, r, PLAIN);
        else partial[blockIdx.x] = r;
    }
}

// The last level, one block: 16 waves share the join, each lane folding up
// to 16 consecutive partials in registers (a whole last level of 16384
// partials in one round of loads), same tree.
constexpr int kWideBlock = 1024;
template <typename T, bool PLAIN>
__global__ __launch_bounds__(kWideBlock) void reduce_last_kernel(int64_t count, int64_t span, const Pair<T> *in,
                                                                 T *out) {
    const Pair<T> r = block_join<T, PLAIN, kWideBlock / 64, 16>(0, count, span, in);
    if (threadIdx.x == 0) write_out(out, r, PLAIN);
}

constexpr int64_t kMaxSpan = 4 * 64 * 64;                   // partials a middle-level block joins
constexpr int64_t kLastSpan = (kWideBlock / 64) * 64 * 64;  // partials the last-level block joins

static int64_t pow2_ceil(int64_t v) {
    int64_t p = 1;
    while (p < v) p <<= 1;
    return p;
}

// First-pass geometry when none is configured: per element size and leaf
// kind, the fastest whole call (first pass plus the joins of its partials)
// of sweeps on MI355X at n = 2^26 over 8-256 tiles and 4, 8 or 16 waves per
// block, confirmed by alternating per-call runs after a streaming kernel
// (as in the benchmark step):
//   binary32 twofold sum, dot of dotted       32 tiles,  8 waves
//   vectors, plain dot
//   binary32 dotted sum, plain sum            128 tiles, 16 waves
//   binary32, leaves from three or four       32 tiles,  4 waves
//   binary64, leaves from one or two arrays   64 tiles,  16 waves
//   binary64, leaves from three or four       16 tiles,  4 waves
static int leaf_arrays(int leaf) {
    switch (leaf) {
    case LEAF_SUM_D: case LEAF_PSUM: return 1;
    case LEAF_SUM_T: case LEAF_DOT_DD: case LEAF_PDOT: return 2;
    case LEAF_DOT_TT: return 4;
    default: return 3;
    }
}

struct AutoShape {
    int64_t tiles;
    int waves;
};

static AutoShape auto_shape(int elem_size, int leaf) {
    if (leaf_arrays(leaf) > 2) return elem_size == 4 ? AutoShape{32, 4} : AutoShape{16, 4};
    if (elem_size == 4) {
        // (64 tiles x 16 waves is 1-2 us faster for the dots in isolated
        // runs but 8-10 us slower inside the benchmark step, measured twice)
        return leaf == LEAF_SUM_D || leaf == LEAF_PSUM ? AutoShape{128, 16} : AutoShape{32, 8};
    }
    return {64, 16};
}

RedShape reduce_shape(int64_t n, int64_t per_block) {
    RedShape s;
    s.tiles = (n + kTile - 1) / kTile;
    const int64_t P = pow2_ceil(s.tiles > 0 ? s.tiles : 1);
    int64_t pb = per_block;
    if (pb > P) pb = P;
    s.per_block = pb;
    s.blocks = (s.tiles + pb - 1) / pb;
    s.padded = P / pb;
    return s;
}

int64_t tiles_per_block(int elem_size, int leaf) {
    const int64_t c = config().red_tiles_per_block;
    return c > 0 ? c : auto_shape(elem_size, leaf).tiles;
}

// Waves per first-pass block: the configured 4, 8 or 16, else the tuned
// value; never more waves than tiles.
static int reduce_waves(int elem_size, int leaf, int64_t per_block) {
    int64_t w = config().red_waves;
    if (w == 0) w = auto_shape(elem_size, leaf).waves;
    while (w > 4 && w > per_block) w /= 2;
    return (int)w;
}

// The levels after the first pass: middle levels join kMaxSpan partials per
// block until at most kLastSpan remain, which one last-level block joins.
struct RedLevel {
    int64_t count, span, next_count;
    bool last;
};
template <typename F>
static void for_each_level(const RedShape &s, F f) {
    int64_t count = s.blocks, padded = s.padded;
    while (padded > 1) {
        const int64_t span = padded <= kLastSpan ? padded : kMaxSpan;
        const int64_t next_padded = padded / span;
        const int64_t next_count = (count + span - 1) / span;
        f(RedLevel{count, span, next_count, next_padded == 1});
        count = next_count;
        padded = next_padded;
    }
}

// Partials launch_reduce stores in the workspace: the first pass's
// per-block partials and every further level that is not the last.
int64_t reduce_work_pairs(int64_t n, int64_t per_block) {
    if (n <= 0) return 0;
    const RedShape s = reduce_shape(n, per_block);
    int64_t total = s.padded > 1 ? s.blocks : 0;
    for_each_level(s, [&](const RedLevel &l) {
        if (!l.last) total += l.next_count;
    });
    return total;
}

// The first pass with blocks of WAVES waves: the one-pass kernel when each
// wave takes exactly one group of tile pairs.
template <typename T, int LEAF, int WAVES>
static void launch_tiles(const Launch &L, int64_t n, const RedShape &s, const T *x0, const T *x1, const T *y0,
                         const T *y1, Pair<T> *work, T *out) {
    constexpr bool PAIRS = TF_RED_PAIRS && LeafTraits<LEAF>::arrays <= TF_RED_PAIR_ARRAYS;
    if (PAIRS && s.per_block == (int64_t)WAVES * PairLayout<T>::TILES)
        tf_launch((reduce_tiles_kernel<T, LEAF, WAVES, PAIRS>), dim3((unsigned)s.blocks), dim3(64 * WAVES), 0,
                  L.stream, n, s.tiles, (int)s.per_block, (int)L.aligned, x0, x1, y0, y1, work, out);
    else
        tf_launch((reduce_tiles_kernel<T, LEAF, WAVES, false>), dim3((unsigned)s.blocks), dim3(64 * WAVES), 0,
                  L.stream, n, s.tiles, (int)s.per_block, (int)L.aligned, x0, x1, y0, y1, work, out);
}

template <typename T, int LEAF>
static void launch_reduce(const Launch &L, int64_t n, int64_t per_block, const T *x0, const T *x1,
                          const T *y0, const T *y1, T *out, Pair<T> *work) {
    constexpr bool PLAIN = LeafTraits<LEAF>::plain;
    if (n == 0) {  // empty: the partial pass over zero partials writes (+0, +0)
        tf_launch((reduce_partials_kernel<T, PLAIN>), dim3(1), dim3(kBlock), 0, L.stream,
                  (int64_t)0, (int64_t)1, (const Pair<T> *)nullptr, (Pair<T> *)nullptr, out);
        return;
    }
    const RedShape s = reduce_shape(n, per_block);
    const bool single = s.padded == 1;
    const int waves = reduce_waves(sizeof(T), LEAF, s.per_block);
    if (waves == 16) launch_tiles<T, LEAF, 16>(L, n, s, x0, x1, y0, y1, work, single ? out : nullptr);
    else if (waves == 8) launch_tiles<T, LEAF, 8>(L, n, s, x0, x1, y0, y1, work, single ? out : nullptr);
    else launch_tiles<T, LEAF, 4>(L, n, s, x0, x1, y0, y1, work, single ? out : nullptr);
    Pair<T> *src = work;
    for_each_level(s, [&](const RedLevel &l) {
        Pair<T> *dst = src + l.count;
        if (l.last && l.span >= kWideBlock / 64)
            tf_launch((reduce_last_kernel<T, PLAIN>), dim3(1), dim3(kWideBlock), 0, L.stream, l.count, l.span,
                      (const Pair<T> *)src, out);
        else
            tf_launch((reduce_partials_kernel<T, PLAIN>), dim3((unsigned)l.next_count), dim3(kBlock), 0,
                      L.stream, l.count, l.span, (const Pair<T> *)src, dst, l.last ? out : (T *)nullptr);
        src = dst;
    });
}

template <typename T>
void run_reduce(const Launch &L, int leaf_kind, int64_t n, int64_t per_block, const void *x0, const void *x1,
                const void *y0, const void *y1, void *out, void *work) {
    const T *a0 = (const T *)x0, *a1 = (const T *)x1, *b0 = (const T *)y0, *b1 = (const T *)y1;
    T *o = (T *)out;
    Pair<T> *w = (Pair<T> *)work;
    switch (leaf_kind) {
    case LEAF_SUM_D: launch_reduce<T, LEAF_SUM_D>(L, n, per_block, a0, a1, b0, b1, o, w); break;
    case LEAF_SUM_T: launch_reduce<T, LEAF_SUM_T>(L, n, per_block, a0, a1, b0, b1, o, w); break;
    case LEAF_DOT_DD: launch_reduce<T, LEAF_DOT_DD>(L, n, per_block, a0, a1, b0, b1, o, w); break;
    case LEAF_DOT_TT: launch_reduce<T, LEAF_DOT_TT>(L, n, per_block, a0, a1, b0, b1, o, w); break;
    case LEAF_DOT_TD: launch_reduce<T, LEAF_DOT_TD>(L, n, per_block, a0, a1, b0, b1, o, w); break;
    case LEAF_DOT_DT: launch_reduce<T, LEAF_DOT_DT>(L, n, per_block, a0, a1, b0, b1, o, w); break;
    case LEAF_PSUM: launch_reduce<T, LEAF_PSUM>(L, n, per_block, a0, a1, b0, b1, o, w); break;
    default: launch_reduce<T, LEAF_PDOT>(L, n, per_block, a0, a1, b0, b1, o, w); break;
    }
}
template void run_reduce<double>(const Launch &, int, int64_t, int64_t, const void *, const void *,
                                 const void *, const void *, void *, void *);
template void run_reduce<float>(const Launch &, int, int64_t, int64_t, const void *, const void *,
                                const void *, const void *, void *, void *);

}  // namespace tf
