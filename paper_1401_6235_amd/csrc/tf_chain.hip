// Chains: one operation applied `reps` times to a value held in registers,
// the compute-bound regime of the paper's performance criteria (data already
// next to the arithmetic units, so the cost is the arithmetic alone).
//
// Each thread carries C independent chains (elements base + c * 256 of its
// block's slice, so loads and stores stay coalesced); the C chains give the
// scheduler independent instructions to interleave while one step waits on
// the previous one.  Inputs are read once and outputs written once, so HBM
// traffic is negligible next to the reps * n operations.
#include "tf_internal.hpp"

// Independent chains per thread (tuned on MI355X: enough to cover the
// latency of dependent VALU steps without spilling).
#ifndef TF_CHAIN_C
#define TF_CHAIN_C 4
#endif
#ifndef TF_PLAIN_CHAIN_C
#define TF_PLAIN_CHAIN_C 4
#endif
// Steps per loop iteration (the step count is a run-time value; a
// remainder loop takes the rest).
#ifndef TF_CHAIN_UNROLL
#define TF_CHAIN_UNROLL 4
#endif
#ifndef TF_PLAIN_CHAIN_UNROLL
#define TF_PLAIN_CHAIN_UNROLL 4
#endif

namespace tf {

template <typename T, int OP, bool YT, int C>
__global__ __launch_bounds__(kBlock) void chain_kernel(int64_t n, int64_t reps, const T *x0, const T *x1,
                                                       const T *y0, const T *y1, T *z0, T *z1) {
    constexpr bool HAS_Y = !op_unary(OP);
    const int64_t base = (int64_t)blockIdx.x * kBlock * C + threadIdx.x;
    T a0[C], a1[C], b0[C], b1[C];
#pragma unroll
    for (int c = 0; c < C; ++c) {
        const int64_t i = base + (int64_t)c * kBlock;
        const bool in = i < n;
        a0[c] = in ? x0[i] : T(1);
        a1[c] = in && x1 ? x1[i] : T(0);
        b0[c] = in && HAS_Y ? y0[i] : T(1);
        b1[c] = in && YT ? y1[i] : T(0);
    }
#pragma unroll TF_CHAIN_UNROLL
    for (int64_t k = 0; k < reps; ++k) {
#pragma unroll
        for (int c = 0; c < C; ++c) {
            const Pair<T> z = apply<T, OP, true, YT>(a0[c], a1[c], b0[c], b1[c]);
            a0[c] = z.hi;
            a1[c] = z.lo;
        }
    }
#pragma unroll
    for (int c = 0; c < C; ++c) {
        const int64_t i = base + (int64_t)c * kBlock;
        if (i < n) {
            z0[i] = a0[c];
            z1[i] = a1[c];
        }
    }
}

template <typename T, int OP, int C>
__global__ __launch_bounds__(kBlock) void plain_chain_kernel(int64_t n, int64_t reps, const T *x, const T *y,
                                                             T *z) {
    constexpr bool HAS_Y = OP != OP_SQRT;
    const int64_t base = (int64_t)blockIdx.x * kBlock * C + threadIdx.x;
    T a[C], b[C];
#pragma unroll
    for (int c = 0; c < C; ++c) {
        const int64_t i = base + (int64_t)c * kBlock;
        a[c] = i < n ? x[i] : T(1);
        b[c] = i < n && HAS_Y ? y[i] : T(1);
    }
#pragma unroll TF_PLAIN_CHAIN_UNROLL
    for (int64_t k = 0; k < reps; ++k) {
#pragma unroll
        for (int c = 0; c < C; ++c) a[c] = apply_plain<T, OP>(a[c], b[c]);
    }
#pragma unroll
    for (int c = 0; c < C; ++c) {
        const int64_t i = base + (int64_t)c * kBlock;
        if (i < n) z[i] = a[c];
    }
}

template <typename T, int OP>
static void launch_chain(const Launch &L, int64_t n, int64_t reps, const T *x0, const T *x1, const T *y0,
                         const T *y1, T *z0, T *z1) {
    constexpr int C = TF_CHAIN_C;
    const unsigned g = grid_for(n, (int64_t)kBlock * C, 0);
    if (y1 && !op_unary(OP))
        tf_launch((chain_kernel<T, OP, true, C>), dim3(g), dim3(kBlock), 0, L.stream, n, reps, x0, x1,
                  y0, y1, z0, z1);
    else
        tf_launch((chain_kernel<T, OP, false, C>), dim3(g), dim3(kBlock), 0, L.stream, n, reps, x0,
                  x1, y0, nullptr, z0, z1);
}

// Operation code of one chain step: mode 0 twofold, 1 coupled, 2 Dekker.
int chain_code(int op, int mode) {
    static const int coupled[5] = {OP_ADD, OP_SUB, OP_MUL_P, OP_DIV_P, OP_SQRT_P};
    if (mode == TF_MODE_TWOFOLD) return op;
    return coupled[op] + (mode == TF_MODE_DEKKER ? OP_RENORM : 0);
}

template <typename T>
void run_chain(const Launch &L, int code, int64_t n, int64_t reps, const void *x0, const void *x1,
               const void *y0, const void *y1, void *z0, void *z1) {
    const T *a0 = (const T *)x0, *a1 = (const T *)x1, *b0 = (const T *)y0, *b1 = (const T *)y1;
    T *c0 = (T *)z0, *c1 = (T *)z1;
    switch (code) {
#define TF_CHAIN_CASE(K)                                                                           \
    case K: launch_chain<T, K>(L, n, reps, a0, a1, b0, b1, c0, c1); break;
        TF_CHAIN_CASE(OP_ADD)
        TF_CHAIN_CASE(OP_SUB)
        TF_CHAIN_CASE(OP_MUL)
        TF_CHAIN_CASE(OP_DIV)
        TF_CHAIN_CASE(OP_SQRT)
        TF_CHAIN_CASE(OP_MUL_P)
        TF_CHAIN_CASE(OP_DIV_P)
        TF_CHAIN_CASE(OP_SQRT_P)
        TF_CHAIN_CASE(OP_RENORM + OP_ADD)
        TF_CHAIN_CASE(OP_RENORM + OP_SUB)
        TF_CHAIN_CASE(OP_RENORM + OP_MUL_P)
        TF_CHAIN_CASE(OP_RENORM + OP_DIV_P)
        TF_CHAIN_CASE(OP_RENORM + OP_SQRT_P)
#undef TF_CHAIN_CASE
    default: break;  // codes come from chain_code
    }
}
template void run_chain<double>(const Launch &, int, int64_t, int64_t, const void *, const void *,
                                const void *, const void *, void *, void *);
template void run_chain<float>(const Launch &, int, int64_t, int64_t, const void *, const void *,
                               const void *, const void *, void *, void *);

template <typename T>
void run_plain_chain(const Launch &L, int op, int64_t n, int64_t reps, const void *x, const void *y, void *z) {
    constexpr int C = TF_PLAIN_CHAIN_C;
    const unsigned g = grid_for(n, (int64_t)kBlock * C, 0);
    const T *a = (const T *)x, *b = (const T *)y;
    T *c = (T *)z;
    switch (op) {
#define TF_PCHAIN_CASE(K)                                                                          \
    case K:                                                                                        \
        tf_launch((plain_chain_kernel<T, K, C>), dim3(g), dim3(kBlock), 0, L.stream, n, reps, a, b, c); \
        break;
        TF_PCHAIN_CASE(OP_ADD)
        TF_PCHAIN_CASE(OP_SUB)
        TF_PCHAIN_CASE(OP_MUL)
        TF_PCHAIN_CASE(OP_DIV)
        TF_PCHAIN_CASE(OP_SQRT)
#undef TF_PCHAIN_CASE
    default: break;
    }
}
template void run_plain_chain<double>(const Launch &, int, int64_t, int64_t, const void *, const void *, void *);
template void run_plain_chain<float>(const Launch &, int, int64_t, int64_t, const void *, const void *, void *);

}  // namespace tf
