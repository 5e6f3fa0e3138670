// Serving: a persistent kernel over a device job table.
//
// Block 0 of the persistent grid is the dispatcher: one thread polls the
// host-coherent descriptor ring (system-scope acquire), copies each new
// descriptor into its device slot and opens the slot with a release store of
// the slot's control word.  Every other block is a worker: its first wave
// reads the 64 control words (one per lane), picks the job with the fewest
// unclaimed units (oldest first among equals) and claims a unit with a
// fetch-add on the control word (wait-free: the returned word says which
// units of which job the block owns, or that it came too late; a large job
// is claimed several consecutive units at a time); the whole block
// processes each unit (a 4096-leaf aligned subtree of a sum / dot, or 4096
// elements of an axpy / Horner), then adds their number to the job's done
// counter.
// A block keeps its LDS copy of the descriptor while it keeps claiming
// units of the same job.  The
// block that completes a job's last unit joins the per-unit partials and
// writes the job's completion record (generation last, system-scope
// release).  Workers never wait for each other, so the grid needs no
// co-residency; every wave leaves its loop once the dispatcher has raised
// the stop flag and no unit is left, and the dispatcher itself exits on the
// host's stop request or after 20 ms without work.
//
// Inputs of RANDOM / ILLCOND jobs are written by the workers themselves, in
// a generation phase of the job that precedes its compute units (the
// persistent kernel never waits for another kernel: streams share a few
// hardware queues, and a second kernel may be queued behind this one).
#include <hip/hip_runtime.h>

#include <mutex>
#include <new>
#include <vector>

#include "tf_serve_host.hpp"
#include "tf_tree.hpp"

namespace tf {

// Waves per worker block.  A unit is processed by the whole block, and the
// tree of a reduction unit does not depend on how many waves share it.
#ifndef TF_SERVE_WAVES
#define TF_SERVE_WAVES 8
#endif
static_assert(TF_SERVE_WAVES == 4 || TF_SERVE_WAVES == 8 || TF_SERVE_WAVES == 16, "4, 8 or 16 waves per worker");
constexpr int kServeWaves = TF_SERVE_WAVES;
constexpr int kServeBlock = 64 * kServeWaves;

// ---------------------------------------------------------------------------
// counter-based input generator (same recipe as the host test generator)
// ---------------------------------------------------------------------------

__device__ __forceinline__ uint64_t mix64(uint64_t z) {
    z = (z ^ (z >> 30)) * TFS_MIX1;
    z = (z ^ (z >> 27)) * TFS_MIX2;
    return z ^ (z >> 31);
}
__device__ __forceinline__ uint64_t draw(uint64_t seed, int64_t i, int a) {
    return mix64(seed + ((uint64_t)(4 * i + a) + 1) * TFS_GAMMA);
}

template <typename T>
__device__ __forceinline__ T gen_value(uint64_t r);
template <>
__device__ __forceinline__ double gen_value<double>(uint64_t r) {
    const int e = (int)((r >> 52) & 0x7ff) % 41 - 20;
    const uint64_t bits = (r & 0x8000000000000000ull) | ((uint64_t)(1023 + e) << 52) | (r & 0xfffffffffffffull);
    return __builtin_bit_cast(double, bits);
}
template <>
__device__ __forceinline__ float gen_value<float>(uint64_t r) {
    const int e = (int)((r >> 52) & 0x7ff) % 41 - 20;
    const uint32_t bits = (uint32_t)((r >> 32) & 0x80000000u) | ((uint32_t)(127 + e) << 23) | (uint32_t)(r & 0x7fffffu);
    return __builtin_bit_cast(float, bits);
}
// u in [-1, 1), exact
template <typename T>
__device__ __forceinline__ T gen_u(uint64_t r);
template <>
__device__ __forceinline__ double gen_u<double>(uint64_t r) { return (double)(r >> 11) * 0x1p-52 - 1.0; }
template <>
__device__ __forceinline__ float gen_u<float>(uint64_t r) { return (float)(uint32_t)(r >> 40) * 0x1p-23f - 1.0f; }
// u in [0, 1), exact
template <typename T>
__device__ __forceinline__ T gen_u01(uint64_t r);
template <>
__device__ __forceinline__ double gen_u01<double>(uint64_t r) { return (double)(r >> 11) * 0x1p-53; }
template <>
__device__ __forceinline__ float gen_u01<float>(uint64_t r) { return (float)(uint32_t)(r >> 40) * 0x1p-24f; }

template <typename T>
__device__ __forceinline__ T low_scale();  // 2^-p
template <>
__device__ __forceinline__ double low_scale<double>() { return 0x1p-53; }
template <>
__device__ __forceinline__ float low_scale<float>() { return 0x1p-24f; }
template <typename T>
__device__ __forceinline__ T cancel_scale();  // relative size left after cancellation
template <>
__device__ __forceinline__ double cancel_scale<double>() { return 0x1p-40; }
template <>
__device__ __forceinline__ float cancel_scale<float>() { return 0x1p-16f; }

// How a job's inputs are drawn: x by gen_value (sums, dots, axpy; their
// ill-conditioned kind cancels y against -a x instead), or in a narrow band
// around 1 for Horner (a tighter one for its ill-conditioned kind).
enum GenMode { GEN_VALUE = 0, GEN_AXPY_ILL = 1, GEN_HORNER = 2, GEN_HORNER_ILL = 3 };

// Element i of every input array the job generates.  The job's pattern is
// a template argument, so a unit's unrolled element loop has no branches
// and the independent elements' hash chains interleave.
template <typename T, int MODE, bool X1, bool Y0, bool Y1>
__device__ __forceinline__ void gen_elem(T *x0, T *x1, T *y0, T *y1, uint64_t s, int64_t i, T a0) {
    T a;
    if constexpr (MODE == GEN_HORNER_ILL) a = T(1) + gen_u<T>(draw(s, i, 0)) * T(0x1p-12);
    else if constexpr (MODE == GEN_HORNER) a = T(0.9) + T(0.2) * gen_u01<T>(draw(s, i, 0));
    else a = gen_value<T>(draw(s, i, 0));
    x0[i] = a;
    if constexpr (X1) x1[i] = a * (gen_u<T>(draw(s, i, 1)) * low_scale<T>());
    if constexpr (Y0) {
        T b;
        if constexpr (MODE == GEN_AXPY_ILL)  // axpy with y ~ -a x
            b = -(a0 * a) + a * (gen_u<T>(draw(s, i, 2)) * cancel_scale<T>());
        else
            b = gen_value<T>(draw(s, i, 2));
        y0[i] = b;
        if constexpr (Y1) y1[i] = b * (gen_u<T>(draw(s, i, 3)) * low_scale<T>());
    }
}

// One generation unit: elements [unit * TFS_CLAIM, (unit + 1) * TFS_CLAIM) of
// every input array the job generates, consecutive threads on consecutive
// elements; a full unit in a loop of fixed length, unrolled so that the
// independent elements' arithmetic and stores overlap.
template <typename T, int MODE, bool X1, bool Y0, bool Y1>
__device__ void gen_unit_as(const tfs_desc &d, int unit) {
    T *x0 = (T *)d.x0, *x1 = (T *)d.x1, *y0 = (T *)d.y0, *y1 = (T *)d.y1;
    const uint64_t s = d.seed;
    const T a0 = T(d.a0);
    const int64_t base = (int64_t)unit * TFS_CLAIM;
    const int64_t end = d.n < base + TFS_CLAIM ? d.n : base + TFS_CLAIM;
    if (end - base == TFS_CLAIM) {
#pragma unroll 4
        for (int k = 0; k < TFS_CLAIM / kServeBlock; ++k)
            gen_elem<T, MODE, X1, Y0, Y1>(x0, x1, y0, y1, s, base + k * kServeBlock + threadIdx.x, a0);
    } else {
        for (int64_t i = base + threadIdx.x; i < end; i += kServeBlock)
            gen_elem<T, MODE, X1, Y0, Y1>(x0, x1, y0, y1, s, i, a0);
    }
}

template <typename T, int MODE, bool X1>
__device__ __forceinline__ void gen_unit_y(const tfs_desc &d, int unit) {
    if constexpr (MODE == GEN_HORNER || MODE == GEN_HORNER_ILL) gen_unit_as<T, MODE, X1, false, false>(d, unit);
    else if (!d.y0) gen_unit_as<T, MODE, X1, false, false>(d, unit);
    else if (!d.y1) gen_unit_as<T, MODE, X1, true, false>(d, unit);
    else gen_unit_as<T, MODE, X1, true, true>(d, unit);
}

template <typename T, int MODE>
__device__ __forceinline__ void gen_unit_x(const tfs_desc &d, int unit) {
    if (d.x1) gen_unit_y<T, MODE, true>(d, unit);
    else gen_unit_y<T, MODE, false>(d, unit);
}

template <typename T>
__device__ void gen_unit(const tfs_desc &d, int unit) {
    const bool horner = d.op == TFS_OP_HORNER, ill = d.kind == TFS_KIND_ILLCOND;
    if (horner && ill) gen_unit_x<T, GEN_HORNER_ILL>(d, unit);
    else if (horner) gen_unit_x<T, GEN_HORNER>(d, unit);
    else if (ill) gen_unit_x<T, GEN_AXPY_ILL>(d, unit);
    else gen_unit_x<T, GEN_VALUE>(d, unit);
}

// ---------------------------------------------------------------------------
// persistent kernel
// ---------------------------------------------------------------------------

struct DevSlot {
    uint32_t done;  // units of the current phase finished
    uint32_t pad;
    uint64_t t_open;   // dispatcher's clock when it opened the slot
    uint64_t t_start;  // first unit claimed
    uint64_t t_ready;  // compute phase opened after generation (0: provided inputs)
    tfs_desc d;
};
struct DevState {
    // The control words sit together (four cache lines), apart from the
    // descriptors: an idle worker's scan reads them all in one load.
    uint64_t ctl[TFS_MAX_SLOTS];  // TFS_CTL(gen, phase, units, next); 0 = empty
    DevSlot slot[TFS_MAX_SLOTS];
    uint64_t stop;
};

__device__ __forceinline__ uint64_t ld_acq_sys(const uint64_t *p) {
    return __hip_atomic_load(p, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_SYSTEM);
}
__device__ __forceinline__ uint64_t ld_sys(const uint64_t *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
}
__device__ __forceinline__ void st_rel_sys(uint64_t *p, uint64_t v) {
    __hip_atomic_store(p, v, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
}

__device__ void dispatcher(tfs_shared *sh, DevState *st, uint64_t idle_ticks) {
    uint64_t consumed = ld_sys(&sh->consumed);  // resume after a relaunch
    uint64_t last = wall_clock64();
    uint64_t beats = 0;
    int how = 2;
    st_rel_sys(&sh->kernel_state, 1);
    while (true) {
        const uint64_t pub = ld_acq_sys(&sh->pub_count);
        const bool fresh = consumed < pub;
        while (consumed < pub) {
            // The whole entry into registers first, then into the slot: the
            // loads (plain, after the acquire above) are independent and
            // share one round trip over the host link.  Copied word by word
            // from memory to memory, each store could alias the next load
            // and every word would cost a round trip of its own.
            constexpr unsigned kWords = sizeof(tfs_desc) / 8;
            static_assert(sizeof(tfs_desc) % 8 == 0, "descriptor is copied in 8-byte words");
            const uint64_t *src = (const uint64_t *)&sh->ring[consumed % TFS_RING];
            uint64_t w[kWords];
#pragma unroll
            for (unsigned k = 0; k < kWords; ++k) w[k] = src[k];
            tfs_desc e;
            __builtin_memcpy(&e, w, sizeof e);
            const int slot = e.slot;
            const uint64_t gen = e.gen;
            const int nclaims = e.nclaims;
            ++consumed;
            if (slot >= 0 && slot < TFS_MAX_SLOTS) {  // a malformed entry is skipped
                DevSlot *s = &st->slot[slot];
                uint64_t *dst = (uint64_t *)&s->d;
#pragma unroll
                for (unsigned k = 0; k < kWords; ++k) dst[k] = w[k];
                s->done = 0;
                s->t_start = 0;
                s->t_ready = 0;
                s->t_open = wall_clock64();
                const uint64_t open = e.ngen > 0 ? TFS_CTL(gen, TFS_PHASE_GEN, e.ngen, 0)
                                                 : TFS_CTL(gen, TFS_PHASE_COMPUTE, nclaims, 0);
                __hip_atomic_store(&st->ctl[slot], open, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
            }
            st_rel_sys(&sh->consumed, consumed);
        }
        if (fresh) last = wall_clock64();
        if (ld_acq_sys(&sh->stop)) break;
        if (wall_clock64() - last > idle_ticks) {
            bool busy = false;
            for (int k = 0; k < TFS_MAX_SLOTS; ++k)
                busy |= __hip_atomic_load(&st->ctl[k], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0;
            if (!busy) {
                how = 3;
                break;
            }
            last = wall_clock64();
        }
        if ((++beats & 1023) == 0) st_rel_sys(&sh->heartbeat, beats);
        __builtin_amdgcn_s_sleep(16);
    }
    __hip_atomic_store(&st->stop, (uint64_t)1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    st_rel_sys(&sh->kernel_state, (uint64_t)how);
}

// Reduction units with the next tile group's loads in flight while the
// current one is reduced (1) or each loaded when reached (0, fewer
// registers).
#ifndef TF_SERVE_RED_PIPE
#define TF_SERVE_RED_PIPE 1
#endif

// Vectors per operand and thread in flight in a vector unit.
#ifndef TF_SERVE_VEC_GROUP
#define TF_SERVE_VEC_GROUP 4
#endif

// ---- one unit of a reduction job ---------------------------------------------

template <typename T, int LEAF>
__device__ void claim_reduce(const tfs_desc &d, int claim) {
    const T *x0 = (const T *)d.x0, *x1 = (const T *)d.x1, *y0 = (const T *)d.y0, *y1 = (const T *)d.y1;
    const bool aligned = ((d.x0 | d.x1 | d.y0 | d.y1) & 15u) == 0;
    const int64_t tiles = (d.n + kTile - 1) / kTile;
    const Pair<T> r = block_subtree<T, LEAF, kServeWaves, false, TF_SERVE_RED_PIPE>(
        claim, d.tiles_per_claim, d.n, tiles, aligned, x0, x1, y0, y1);
    if (threadIdx.x == 0) ((Pair<T> *)d.part)[claim] = r;
}

template <typename T>
__device__ __forceinline__ uint64_t bits_of(T v) {
    if constexpr (sizeof(T) == 8) return __builtin_bit_cast(uint64_t, v);
    else return (uint64_t)__builtin_bit_cast(uint32_t, v);
}

// Block-wide reduction of a vector unit's summary (max is exact and the
// sums are integers, so the order does not matter); result in thread 0.
__device__ tfs_vsum block_summary(tfs_vsum v) {
    __shared__ tfs_vsum s[kServeBlock];
    const int t = threadIdx.x;
    s[t] = v;
    __syncthreads();
    for (int w = kServeBlock / 2; w > 0; w >>= 1) {
        if (t < w) {
            s[t].max0 = fmax(s[t].max0, s[t + w].max0);
            s[t].max1 = fmax(s[t].max1, s[t + w].max1);
            s[t].n_flagged += s[t + w].n_flagged;
            s[t].nonfinite += s[t + w].nonfinite;
            s[t].hash0 += s[t + w].hash0;
            s[t].hash1 += s[t + w].hash1;
        }
        __syncthreads();
    }
    const tfs_vsum r = s[0];
    __syncthreads();
    return r;
}

template <typename T>
__device__ __forceinline__ void account(tfs_vsum &acc, T z0, T z1, double thr) {
    const double a0 = fabs((double)z0), a1 = fabs((double)z1);
    const bool finite = isfinite(z0) && isfinite(z1);
    acc.max0 = fmax(acc.max0, a0);
    acc.max1 = fmax(acc.max1, a1);
    acc.nonfinite += finite ? 0 : 1;
    acc.n_flagged += (!finite || a1 > thr * a0) ? 1 : 0;
    acc.hash0 += bits_of(z0);
    acc.hash1 += bits_of(z1);
}

// ---- one unit of an axpy / Horner job ----------------------------------------

// Horner element with the coefficients read from the block's copy of the
// descriptor (already rounded to T), the same steps as horner_one.
template <typename T, bool XT>
__device__ __forceinline__ Pair<T> horner_desc(const double *c, int degree, T x0, T x1) {
    Pair<T> r{(T)c[degree], T(0)};
    for (int k = degree - 1; k >= 0; --k) {
        const Pair<T> m = XT ? mul_tt(r.hi, r.lo, x0, x1) : mul_td(r.hi, r.lo, x0);
        r = add_td(m.hi, m.lo, (T)c[k]);
    }
    return r;
}

template <typename T, int OP, bool XT, bool YT>
__device__ __forceinline__ Pair<T> vector_elem(const tfs_desc &d, T a0, T a1, T x0, T x1, T y0, T y1) {
    if constexpr (OP == TFS_OP_AXPY) return axpy_one<T, XT, YT>(a0, a1, x0, x1, y0, y1);
    else return horner_desc<T, XT>(d.c, d.degree, x0, x1);
}


static_assert(TF_MAX_DEGREE < 64, "a wave's lanes hold the Horner coefficients");

// One round of a vector unit: U 16-byte vectors per operand and thread,
// consecutive threads on consecutive vectors.
template <typename T, int U>
struct VecRound {
    using V = typename Vec<T>::type;
    V p0[U], p1[U], q0[U], q1[U];
};

// Loads the round of U vectors per operand starting at vector j0 of the
// unit whose first vector is vb.
template <typename T, int OP, bool XT, bool YT, int U>
__device__ __forceinline__ void round_load(const tfs_desc &d, VecRound<T, U> &R, int64_t vb, int j0) {
    constexpr bool HAS_Y = OP == TFS_OP_AXPY;
    const T *x0 = (const T *)d.x0, *x1 = (const T *)d.x1, *y0 = (const T *)d.y0, *y1 = (const T *)d.y1;
#pragma unroll
    for (int u = 0; u < U; ++u) {
        const int64_t i = vb + (int64_t)(j0 + u) * kServeBlock + threadIdx.x;
        R.p0[u] = vload(x0, i);
        if constexpr (XT) R.p1[u] = vload(x1, i);
        if constexpr (HAS_Y) R.q0[u] = vload(y0, i);
        if constexpr (HAS_Y && YT) R.q1[u] = vload(y1, i);
    }
}

// Computes and stores a loaded round, adding its elements to the summary.
template <typename T, int OP, bool XT, bool YT, int U>
__device__ __forceinline__ void round_run(const tfs_desc &d, const VecRound<T, U> &R, int64_t vb, int j0,
                                          tfs_vsum &acc) {
    using V = typename Vec<T>::type;
    constexpr int W = Vec<T>::N;
    constexpr bool HAS_Y = OP == TFS_OP_AXPY;
    T *z0 = (T *)d.z0, *z1 = (T *)d.z1;
    Pair<T> z[U][W];
    if constexpr (OP == TFS_OP_HORNER) {
        // the U * W elements' Horner steps interleaved (degree loop outside),
        // each element's operations unchanged: a wave has that many
        // independent chains to issue.  Lane k holds coefficient k (degree
        // <= 32 < 64), and each step takes its coefficient with a readlane:
        // no LDS read and wait inside the degree loop.
        const int lane = threadIdx.x & 63;
        const T cl = (T)d.c[lane <= d.degree ? lane : 0];
        const T cd = readlane_t(cl, d.degree);
#pragma unroll
        for (int u = 0; u < U; ++u)
#pragma unroll
            for (int k = 0; k < W; ++k) z[u][k] = Pair<T>{cd, T(0)};
        for (int j = d.degree - 1; j >= 0; --j) {
            const T cj = readlane_t(cl, j);
#pragma unroll
            for (int u = 0; u < U; ++u)
#pragma unroll
                for (int k = 0; k < W; ++k) {
                    const Pair<T> m = XT ? mul_tt(z[u][k].hi, z[u][k].lo, R.p0[u][k], R.p1[u][k])
                                         : mul_td(z[u][k].hi, z[u][k].lo, R.p0[u][k]);
                    z[u][k] = add_td(m.hi, m.lo, cj);
                }
        }
    } else {
        const T a0 = (T)d.a0, a1 = (T)d.a1;
#pragma unroll
        for (int u = 0; u < U; ++u)
#pragma unroll
            for (int k = 0; k < W; ++k)
                z[u][k] = vector_elem<T, OP, XT, YT>(d, a0, a1, R.p0[u][k], XT ? R.p1[u][k] : T(0),
                                                     HAS_Y ? R.q0[u][k] : T(0), (HAS_Y && YT) ? R.q1[u][k] : T(0));
    }
#pragma unroll
    for (int u = 0; u < U; ++u) {
        V r0, r1;
#pragma unroll
        for (int k = 0; k < W; ++k) {
            r0[k] = z[u][k].hi;
            r1[k] = z[u][k].lo;
            account(acc, z[u][k].hi, z[u][k].lo, d.thr);
        }
        const int64_t i = vb + (int64_t)(j0 + u) * kServeBlock + threadIdx.x;
        vstore(z0, i, r0);
        vstore(z1, i, r1);
    }
}

// One unit of TFS_CLAIM elements, added to the summary: 16-byte vectors,
// TF_SERVE_VEC_GROUP per operand in flight, consecutive threads on
// consecutive vectors; a short or misaligned unit takes a scalar loop.
template <typename T, int OP, bool XT, bool YT>
__device__ __forceinline__ void claim_vector(const tfs_desc &d, int claim, tfs_vsum &acc) {
    constexpr int W = Vec<T>::N;
    constexpr int NV = TFS_CLAIM / kServeBlock / W;  // vectors per thread
    constexpr int U = NV < TF_SERVE_VEC_GROUP ? NV : TF_SERVE_VEC_GROUP;
    constexpr bool HAS_Y = OP == TFS_OP_AXPY;
    const T *x0 = (const T *)d.x0, *x1 = (const T *)d.x1, *y0 = (const T *)d.y0, *y1 = (const T *)d.y1;
    T *z0 = (T *)d.z0, *z1 = (T *)d.z1;
    const int64_t base = (int64_t)claim * TFS_CLAIM;
    const int64_t end = d.n < base + TFS_CLAIM ? d.n : base + TFS_CLAIM;
    const bool aligned = ((d.x0 | d.x1 | d.y0 | d.y1 | d.z0 | d.z1) & 15u) == 0;
    if (aligned && end == base + TFS_CLAIM) {
#pragma unroll
        for (int j0 = 0; j0 < NV; j0 += U) {
            VecRound<T, U> R;
            round_load<T, OP, XT, YT, U>(d, R, base / W, j0);
            round_run<T, OP, XT, YT, U>(d, R, base / W, j0, acc);
        }
    } else {
        const T a0 = (T)d.a0, a1 = (T)d.a1;
        for (int64_t i = base + threadIdx.x; i < end; i += kServeBlock) {
            const Pair<T> z = vector_elem<T, OP, XT, YT>(d, a0, a1, x0[i], XT ? x1[i] : T(0),
                                                        HAS_Y ? y0[i] : T(0), (HAS_Y && YT) ? y1[i] : T(0));
            z0[i] = z.hi;
            z1[i] = z.lo;
            account(acc, z.hi, z.lo, d.thr);
        }
    }
}

// The vector units [claim, claim + count) of a job with one block summary
// for the batch, written as the first unit's partial; the batch's other
// partials are zero.  A summary holds maxima of magnitudes and sums, for
// which zero is neutral, so the job's totals do not depend on the batching.
template <typename T, int OP, bool XT, bool YT>
__device__ void vector_units(const tfs_desc &d, int claim, int count) {
    tfs_vsum acc = {0.0, 0.0, 0, 0, 0, 0};
    for (int c = claim; c < claim + count; ++c) claim_vector<T, OP, XT, YT>(d, c, acc);
    const tfs_vsum r = block_summary(acc);
    if (threadIdx.x == 0) {
        tfs_vsum *part = (tfs_vsum *)d.part;
        part[claim] = r;
        for (int c = claim + 1; c < claim + count; ++c) part[c] = tfs_vsum{0.0, 0.0, 0, 0, 0, 0};
    }
}

// The compute units [claim, claim + count) of a job: reduction units one by
// one (one partial each), vector units as one batch.
template <typename T>
__device__ void run_units(const tfs_desc &d, int claim, int count) {
    const bool xt = d.x1 != 0, yt = d.y1 != 0;
    switch (d.op) {
    case TFS_OP_SUM:
        for (int c = claim; c < claim + count; ++c) {
            if (xt) claim_reduce<T, LEAF_SUM_T>(d, c);
            else claim_reduce<T, LEAF_SUM_D>(d, c);
        }
        break;
    case TFS_OP_DOT:
        for (int c = claim; c < claim + count; ++c) {
            if (xt && yt) claim_reduce<T, LEAF_DOT_TT>(d, c);
            else if (xt) claim_reduce<T, LEAF_DOT_TD>(d, c);
            else if (yt) claim_reduce<T, LEAF_DOT_DT>(d, c);
            else claim_reduce<T, LEAF_DOT_DD>(d, c);
        }
        break;
    case TFS_OP_AXPY:
        if (xt && yt) vector_units<T, TFS_OP_AXPY, true, true>(d, claim, count);
        else if (xt) vector_units<T, TFS_OP_AXPY, true, false>(d, claim, count);
        else if (yt) vector_units<T, TFS_OP_AXPY, false, true>(d, claim, count);
        else vector_units<T, TFS_OP_AXPY, false, false>(d, claim, count);
        break;
    default:
        if (xt) vector_units<T, TFS_OP_HORNER, true, false>(d, claim, count);
        else vector_units<T, TFS_OP_HORNER, false, false>(d, claim, count);
    }
}

// ---- completion ------------------------------------------------------------------

template <typename T>
__device__ void finalize(const tfs_desc &d, DevSlot *S, uint64_t *ctl, tfs_done *rec) {
    tfs_done out = {};
    if (d.op == TFS_OP_SUM || d.op == TFS_OP_DOT) {
        // four partials per lane in flight: the serving kernel's register budget is set
        // by its largest path, and two waves per SIMD must fit
        const Pair<T> r = block_join<T, false, kServeWaves, 4>(0, d.nclaims, d.padded, (const Pair<T> *)d.part);
        const double z0 = (double)r.hi, z1 = (double)r.lo;
        out.z0 = z0;
        out.z1 = z1;
        const bool finite = isfinite(z0) && isfinite(z1);
        out.nonfinite = finite ? 0 : 1;
        out.flag = (!finite || fabs(z1) > d.thr * fabs(z0)) ? 1 : 0;
    } else {
        tfs_vsum acc = {0.0, 0.0, 0, 0, 0, 0};
        const tfs_vsum *p = (const tfs_vsum *)d.part;
        for (int k = threadIdx.x; k < d.nclaims; k += kServeBlock) {
            acc.max0 = fmax(acc.max0, p[k].max0);
            acc.max1 = fmax(acc.max1, p[k].max1);
            acc.n_flagged += p[k].n_flagged;
            acc.nonfinite += p[k].nonfinite;
            acc.hash0 += p[k].hash0;
            acc.hash1 += p[k].hash1;
        }
        const tfs_vsum r = block_summary(acc);
        out.max0 = r.max0;
        out.max1 = r.max1;
        out.n_flagged = r.n_flagged;
        out.nonfinite = r.nonfinite;
        out.hash0 = r.hash0;
        out.hash1 = r.hash1;
        out.flag = (r.nonfinite > 0 || r.max1 > d.thr * r.max0) ? 1 : 0;
    }
    if (threadIdx.x == 0) {
        // empty the slot first: the host reuses it only after seeing the record
        __hip_atomic_store(ctl, (uint64_t)0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        out.t_open = S->t_open;
        out.t_start = S->t_start;
        out.t_ready = S->t_ready;
        out.t_end = wall_clock64();
        out.status = TF_OK;
        rec->status = out.status;
        rec->flag = out.flag;
        rec->z0 = out.z0;
        rec->z1 = out.z1;
        rec->max0 = out.max0;
        rec->max1 = out.max1;
        rec->n_flagged = out.n_flagged;
        rec->nonfinite = out.nonfinite;
        rec->hash0 = out.hash0;
        rec->hash1 = out.hash1;
        rec->t_open = out.t_open;
        rec->t_start = out.t_start;
        rec->t_ready = out.t_ready;
        rec->t_end = out.t_end;
        st_rel_sys(&rec->gen, d.gen);
    }
}

// Build-time knobs (results never depend on them): worker blocks per
// compute unit, and the split of a job's remaining units over the workers
// that sets the claim batch.
#ifndef TF_SERVE_WORKERS_PER_CU
#define TF_SERVE_WORKERS_PER_CU 1
#endif
#ifndef TF_SERVE_BATCH_SHARE
#define TF_SERVE_BATCH_SHARE 400  // percent of a fair share of the remaining units per claim
#endif
#ifndef TF_SERVE_IDLE_SLEEP
#define TF_SERVE_IDLE_SLEEP 127  // s_sleep units (64 cycles) between scans of an idle worker
#endif
static_assert(TF_SERVE_WORKERS_PER_CU >= 1 && TF_SERVE_WORKERS_PER_CU <= 4, "1 to 4 worker blocks per CU");

// Units per claim when `remaining` units of a job are left and `workers`
// blocks compete: TF_SERVE_BATCH_SHARE percent of remaining / workers,
// between 1 and TFS_MAX_BATCH.
__device__ __forceinline__ uint64_t batch_for(uint64_t remaining, uint64_t workers) {
    const uint64_t k = remaining * TF_SERVE_BATCH_SHARE / (100 * (workers ? workers : 1));
    return k < 1 ? 1 : k > TFS_MAX_BATCH ? TFS_MAX_BATCH : k;
}

__device__ void worker(tfs_shared *sh, DevState *st) {
    __shared__ int s_slot, s_claim, s_count, s_phase, s_last, s_have_slot, s_have_phase;
    __shared__ uint32_t s_gen, s_have_gen;
    __shared__ uint64_t s_desc[sizeof(tfs_desc) / 8];
    const int t = threadIdx.x;
    if (t == 0) {
        s_have_slot = -1;
        s_have_gen = 0;
        s_have_phase = -1;
    }
    while (true) {
        if (t < 64) {
            const uint64_t c = __hip_atomic_load(&st->ctl[t], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            const uint64_t gen = TFS_CTL_GEN(c), nt = TFS_CTL_NTILES(c), nx = TFS_CTL_NEXT(c);
            // shortest remaining job first (fewest unclaimed units), then oldest
            const uint64_t key = (gen != 0 && nx < nt) ? ((nt - nx) << 32) | gen : ~0ull;
            uint64_t m = key;
#pragma unroll
            for (int d = 1; d < 64; d <<= 1) {
                const uint64_t o = __shfl_xor(m, d);
                m = o < m ? o : m;
            }
            if (m == ~0ull) {
                if (t == 0) {
                    const bool stop = __hip_atomic_load(&st->stop, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) != 0;
                    s_slot = stop ? -3 : -1;
                }
            } else if (key == m) {  // the one lane holding the chosen job
                // Wait-free claim: the returned word names the units this
                // block owns and the phase they belong to.  The slot may have been emptied or reopened for a
                // newer job since the scan; an add past the last unit (or on
                // an empty word, which the next opening overwrites) claims
                // nothing, and a unit of a newer job is as good as any.
                // Relaxed: the claim publishes nothing, and the one thing it
                // must see, the descriptor, is acquired below (fence after
                // this read of the opening's release store) only when the
                // block's cached copy is for another job.  Each agent-scope
                // acquire or release costs an L2 invalidate or write-back
                // on this chip, so the per-unit path keeps a single release.
                // A large job is claimed a batch of consecutive units at a
                // time (one fetch-add and one count per batch: atomics on
                // one word serialise, at tens of nanoseconds each), sized as
                // a share of the remaining units per worker (batch_for).
                const uint64_t k = batch_for(nt - nx, gridDim.x - 1);
                const uint64_t old = __hip_atomic_fetch_add(&st->ctl[t], k, __ATOMIC_RELAXED,
                                                             __HIP_MEMORY_SCOPE_AGENT);
                const uint64_t g = TFS_CTL_GEN(old), first = TFS_CTL_NEXT(old), total = TFS_CTL_NTILES(old);
                const bool ok = g != 0 && first < total;
                s_slot = ok ? t : -2;
                s_claim = (int)first;
                s_count = ok ? (int)(first + k < total ? k : total - first) : 0;
                s_phase = (int)TFS_CTL_PHASE(old);
                s_gen = (uint32_t)g;
            }
        }
        __syncthreads();
        const int slot = s_slot, claim = s_claim, count = s_count, phase = s_phase;
        const uint32_t gen = s_gen;
        // A new job, or the compute phase of a job whose inputs other blocks
        // have just generated: acquire (descriptor, inputs) before use.
        const bool fresh = slot >= 0 && (slot != s_have_slot || gen != s_have_gen || phase != s_have_phase);
        __syncthreads();
        if (slot == -3) break;
        if (slot < 0) {
            if (slot == -1) __builtin_amdgcn_s_sleep(TF_SERVE_IDLE_SLEEP);
            continue;
        }
        DevSlot *S = &st->slot[slot];
        if (fresh) {  // the block's copy of the descriptor is for another job
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
            const uint64_t *src = (const uint64_t *)&S->d;
            for (unsigned k = t; k < sizeof(tfs_desc) / 8; k += kServeBlock) s_desc[k] = src[k];
            if (t == 0) {
                s_have_slot = slot;
                s_have_gen = gen;
                s_have_phase = phase;
            }
            __syncthreads();
        }
        const tfs_desc &d = *(const tfs_desc *)s_desc;
        const bool gen_phase = phase == TFS_PHASE_GEN;
        if (claim == 0 && t == 0 && (gen_phase || d.ngen == 0)) S->t_start = wall_clock64();
        if (gen_phase) {
            for (int c = claim; c < claim + count; ++c) {
                if (d.dtype == TF_F64) gen_unit<double>(d, c);
                else gen_unit<float>(d, c);
            }
        } else if (count > 0) {
            if (d.dtype == TF_F64) run_units<double>(d, claim, count);
            else run_units<float>(d, claim, count);
        }
        __syncthreads();
        if (t == 0) {
            // release fence + relaxed count: the block that counts the last
            // unit reads the end of every other block's release sequence and
            // acquires them all with the fence below
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
            const uint32_t done = __hip_atomic_fetch_add(&S->done, (uint32_t)count, __ATOMIC_RELAXED,
                                                         __HIP_MEMORY_SCOPE_AGENT);
            s_last = done + (uint32_t)count == (uint32_t)(gen_phase ? d.ngen : d.nclaims);
        }
        __syncthreads();
        if (s_last) {
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
            if (gen_phase) {
                // Every input is written: reopen the slot for the compute
                // units (a late add of the generation phase that lands after
                // this store is a valid claim of a compute unit; one before
                // it claimed nothing and is overwritten).
                if (t == 0) {
                    S->done = 0;
                    S->t_ready = wall_clock64();
                    __hip_atomic_store(&st->ctl[slot], TFS_CTL(d.gen, TFS_PHASE_COMPUTE, d.nclaims, 0),
                                       __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
                }
            } else if (d.dtype == TF_F64) {
                finalize<double>(d, S, &st->ctl[slot], &sh->done[slot]);
            } else {
                finalize<float>(d, S, &st->ctl[slot], &sh->done[slot]);
            }
        }
        __syncthreads();
    }
}

// Every worker block must be resident: with k worker blocks of w waves per
// CU each SIMD holds k w / 4 waves, so the registers are capped for that.
__global__ __launch_bounds__(kServeBlock)
__attribute__((amdgpu_waves_per_eu(TF_SERVE_WORKERS_PER_CU * TF_SERVE_WAVES / 4)))
void serve_kernel(tfs_shared *sh, DevState *st, uint64_t idle_ticks) {
    if (blockIdx.x == 0) {
        if (threadIdx.x == 0) dispatcher(sh, st, idle_ticks);
        return;
    }
    worker(sh, st);
}

// ---------------------------------------------------------------------------
// HIP implementation of the server's device interface
// ---------------------------------------------------------------------------

class HipDevice : public tfs::DeviceOps {
  public:
    int init(int device, uint64_t budget) {
        device_ = device;
        if (hipSetDevice(device) != hipSuccess) return TF_EDEVICE;
        if (budget && hipMalloc(&pool_, budget) != hipSuccess) return TF_ENOMEM;
        if (hipHostMalloc((void **)&shared_, sizeof(tfs_shared), hipHostMallocCoherent | hipHostMallocMapped) !=
            hipSuccess)
            return TF_ENOMEM;
        memset(shared_, 0, sizeof(tfs_shared));
        if (hipMalloc(&state_, sizeof(DevState)) != hipSuccess) return TF_ENOMEM;
        if (hipMemset(state_, 0, sizeof(DevState)) != hipSuccess) return TF_EDEVICE;
        if (hipStreamCreateWithFlags(&work_, hipStreamNonBlocking) != hipSuccess) return TF_EDEVICE;
        int rate_khz = 100000, cus = 256;
        (void)hipDeviceGetAttribute(&rate_khz, hipDeviceAttributeWallClockRate, device);
        (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, device);
        tick_hz_ = (double)rate_khz * 1000.0;
        // The grid (dispatcher + workers) is exactly TF_SERVE_WORKERS_PER_CU
        // blocks per CU, so every block is resident whatever the kernel's
        // register count (a block left waiting for a CU would never run
        // beside the persistent ones); at most 1024 workers: the claim
        // counter's overshoot bound.
        workers_ = cus * TF_SERVE_WORKERS_PER_CU - 1;
        if (workers_ < 1) workers_ = 1;
        if (workers_ > 1024) workers_ = 1024;
        return TF_OK;
    }
    ~HipDevice() override {
        if (device_ >= 0) (void)hipSetDevice(device_);
        if (work_) (void)hipStreamSynchronize(work_);
        if (work_) (void)hipStreamDestroy(work_);
        if (state_) (void)hipFree(state_);
        if (shared_) (void)hipHostFree(shared_);
        if (pool_) (void)hipFree(pool_);
    }
    uint64_t pool_base() override { return (uint64_t)pool_; }
    tfs_shared *shared() override { return shared_; }
    double tick_hz() const { return tick_hz_; }
    int start() override {
        (void)hipSetDevice(device_);
        __atomic_store_n(&shared_->stop, 0, __ATOMIC_RELEASE);
        const uint64_t zero = 0;
        if (hipMemcpy(&state_->stop, &zero, sizeof zero, hipMemcpyHostToDevice) != hipSuccess) return TF_EDEVICE;
        __atomic_store_n(&shared_->kernel_state, 1, __ATOMIC_RELEASE);  // launched: no second launch on publish
        // Drain after 20 ms without work: the kernel's hardware queue may be
        // shared with other streams of the process, whose work waits until
        // it exits; the host relaunches it with the next job.
        const uint64_t idle = (uint64_t)(0.02 * tick_hz_);
        return tf_launch(serve_kernel, dim3(1 + workers_), dim3(kServeBlock), 0, work_, shared_, state_, idle) == hipSuccess
                   ? TF_OK
                   : TF_EDEVICE;
    }
    bool running() override { return hipStreamQuery(work_) == hipErrorNotReady; }
    int stop() override {
        __atomic_store_n(&shared_->stop, 1, __ATOMIC_RELEASE);
        return hipStreamSynchronize(work_) == hipSuccess ? TF_OK : TF_EDEVICE;
    }

  private:
    int device_ = -1;
    void *pool_ = nullptr;
    tfs_shared *shared_ = nullptr;
    DevState *state_ = nullptr;
    hipStream_t work_ = nullptr;
    double tick_hz_ = 1e8;
    int workers_ = 256;
};

}  // namespace tf

struct tfs_server {
    tf::HipDevice dev;
    tfs::Server *server = nullptr;
};

extern "C" {

double tfs_clock(void) { return tfs::now_s(); }

tfs_server *tfs_create(int device, uint64_t budget_bytes, int max_slots) {
    if (max_slots < 1 || max_slots > TFS_MAX_SLOTS || budget_bytes < 4096) return nullptr;
    tfs_server *s = new (std::nothrow) tfs_server;
    if (!s) return nullptr;
    if (s->dev.init(device, budget_bytes) != TF_OK) {
        delete s;
        return nullptr;
    }
    s->server = new tfs::Server(&s->dev, budget_bytes, max_slots);
    s->server->set_tick_hz(s->dev.tick_hz());
    if (s->server->start() != TF_OK) {
        delete s->server;
        delete s;
        return nullptr;
    }
    return s;
}

int tfs_submit(tfs_server *s, const tfs_job *job, double t_arrive, uint64_t *id) {
    if (!s || !job) return TF_EINVAL;
    return s->server->submit(*job, t_arrive, id);
}

int tfs_poll(tfs_server *s, tfs_result *out, int max) {
    if (!s || !out || max < 0) return TF_EINVAL;
    return s->server->poll(out, max);
}

int tfs_get_stats(tfs_server *s, tfs_stats *out) {
    if (!s || !out) return TF_EINVAL;
    s->server->stats(out);
    return TF_OK;
}

int tfs_destroy(tfs_server *s) {
    if (!s) return TF_EINVAL;
    s->server->shutdown();
    delete s->server;
    delete s;
    return TF_OK;
}

}  // extern "C"
