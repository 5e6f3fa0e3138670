// Twofold sum and dot over the fixed pairwise tree.
//
// The tree is defined by element indices only (tiles of 256 leaves, complete
// adjacent pairing inside a tile, tile results paired the same way up to a
// power of two), so every launch geometry below evaluates the very same
// tree and the result is bitwise reproducible.
//
// Mapping onto gfx950:
//   * one wave reduces one tile (tf_tree.hpp);
//   * one block of 4 waves reduces an aligned group of `per_block` tiles
//     (a subtree): each wave folds its consecutive tiles with a binary
//     counter (subtrees of 1, 2, 4, ... tiles merged as they complete), and
//     thread 0 joins the (at most 4) wave results;
//   * the per-block partials are joined by the same pairing in one more
//     pass (a second pass only when there are more than 16384 of them).
//   * within a block, lane t of a wave keeps the wave's t-th subtree value
//     and a butterfly finishes the wave's aligned group: every tree level
//     stays in registers.
#include "tf_tree.hpp"

namespace tf {

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
    const Pair<T> r = block_subtree<T, LEAF>(blockIdx.x, per_block, n, tiles, aligned != 0, x0, x1, y0, y1);
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

// The last level, one block: 16 waves share the join (a quarter of the
// chunks per wave that four waves would fold one after another), same tree.
constexpr int kWideBlock = 1024;
template <typename T, bool PLAIN>
__global__ __launch_bounds__(kWideBlock) void reduce_last_kernel(int64_t count, int64_t span, const Pair<T> *in,
                                                                 T *out) {
    const Pair<T> r = block_join<T, PLAIN, kWideBlock / 64>(0, count, span, in);
    if (threadIdx.x == 0) write_out(out, r, PLAIN);
}

constexpr int64_t kMaxSpan = 4 * 64 * 64;  // partials one block joins

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

// Partials launch_reduce stores in the workspace for n leaves: the first
// pass's per-block partials and every further level that is not the last.
int64_t reduce_work_pairs(int64_t n) {
    if (n <= 0) return 0;
    const RedShape s = reduce_shape(n);
    int64_t total = 0, count = s.blocks, padded = s.padded;
    if (padded > 1) total += count;
    while (padded > 1) {
        const int64_t span = padded < kMaxSpan ? padded : kMaxSpan;
        const int64_t next_padded = padded / span;
        const int64_t next_count = (count + span - 1) / span;
        if (next_padded > 1) total += next_count;
        count = next_count;
        padded = next_padded;
    }
    return total;
}

template <typename T, int LEAF>
static void launch_reduce(const Launch &L, int64_t n, const T *x0, const T *x1, const T *y0,
                          const T *y1, T *out, Pair<T> *work) {
    constexpr bool PLAIN = LeafTraits<LEAF>::plain;
    if (n == 0) {  // empty: the partial pass over zero partials writes (+0, +0)
        tf_launch((reduce_partials_kernel<T, PLAIN>), dim3(1), dim3(kBlock), 0, L.stream,
                  (int64_t)0, (int64_t)1, (const Pair<T> *)nullptr, (Pair<T> *)nullptr, out);
        return;
    }
    const RedShape s = reduce_shape(n);
    const bool single = s.padded == 1;
    tf_launch((reduce_tiles_kernel<T, LEAF>), dim3((unsigned)s.blocks), dim3(kBlock), 0, L.stream,
              n, s.tiles, (int)s.per_block, (int)L.aligned, x0, x1, y0, y1, work,
              single ? out : (T *)nullptr);
    int64_t count = s.blocks, padded = s.padded;
    Pair<T> *src = work;
    while (padded > 1) {
        const int64_t span = padded < kMaxSpan ? padded : kMaxSpan;
        const int64_t next_padded = padded / span;
        const int64_t next_count = (count + span - 1) / span;
        Pair<T> *dst = src + count;
        const bool last = next_padded == 1;
        if (last && span >= kWideBlock / 64)
            tf_launch((reduce_last_kernel<T, PLAIN>), dim3(1), dim3(kWideBlock), 0, L.stream, count, span,
                      (const Pair<T> *)src, out);
        else
            tf_launch((reduce_partials_kernel<T, PLAIN>), dim3((unsigned)next_count), dim3(kBlock), 0,
                      L.stream, count, span, (const Pair<T> *)src, dst, last ? out : (T *)nullptr);
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
