// Elementwise twofold operations, their plain counterparts, axpy, Horner and
// the memory probe.  All are streaming kernels bound by HBM bandwidth: each
// thread moves 16-byte vectors (2 doubles / 4 floats) with non-temporal
// loads and stores, UNROLL independent vectors in flight, consecutive
// threads on consecutive vectors so every wave touches contiguous 1 KiB
// lines.  A ragged tail (n not a multiple of the vector width) is finished
// by the first threads of block 0; misaligned arrays take a scalar kernel.
#include "tf_internal.hpp"

// Vectors in flight per thread, tuned on MI355X at n = 2^28: binary64
// kernels run best with one 16-byte vector per operand per thread, binary32
// binary operations with four (the square root, with half the streams,
// with one).
#ifndef TF_EW_UNROLL_F64
#define TF_EW_UNROLL_F64 1
#endif
#ifndef TF_EW_UNROLL_F32
#define TF_EW_UNROLL_F32 4
#endif
#ifndef TF_EW_UNROLL_F32_UNARY
#define TF_EW_UNROLL_F32_UNARY 1
#endif
#ifndef TF_PLAIN_UNROLL
#define TF_PLAIN_UNROLL 4
#endif
// Threads per block and consecutive block-sized groups of vectors one block
// walks through (1: one-shot grid).
#ifndef TF_EW_BLOCK
#define TF_EW_BLOCK 256
#endif
#ifndef TF_EW_CHUNK
#define TF_EW_CHUNK 1
#endif

namespace tf {

constexpr int kEwBlock = TF_EW_BLOCK;

// ---------------------------------------------------------------------------
// twofold binary / unary operations
// ---------------------------------------------------------------------------

template <typename T, int OP, bool XT, bool YT, int UNROLL>
__global__ __launch_bounds__(kEwBlock) void ew_vec_kernel(int64_t n, const T *x0, const T *x1,
                                                        const T *y0, const T *y1, T *z0, T *z1) {
    using V = typename Vec<T>::type;
    constexpr int W = Vec<T>::N;
    constexpr bool HAS_Y = !op_unary(OP);
    const int64_t nvec = n / W;
    for (int64_t grp = (int64_t)blockIdx.x * TF_EW_CHUNK; grp * kEwBlock * UNROLL < nvec;
         grp += (int64_t)gridDim.x * TF_EW_CHUNK)
    for (int64_t c = 0, base = grp * kEwBlock * UNROLL + threadIdx.x; c < TF_EW_CHUNK && base < nvec;
         ++c, base += (int64_t)kEwBlock * UNROLL) {
        V a0[UNROLL], a1[UNROLL], b0[UNROLL], b1[UNROLL];
#pragma unroll
        for (int u = 0; u < UNROLL; ++u) {
            const int64_t i = base + (int64_t)u * kEwBlock;
            if (i < nvec) {
                a0[u] = vload(x0, i);
                if constexpr (XT) a1[u] = vload(x1, i);
                if constexpr (HAS_Y) b0[u] = vload(y0, i);
                if constexpr (HAS_Y && YT) b1[u] = vload(y1, i);
            }
        }
#pragma unroll
        for (int u = 0; u < UNROLL; ++u) {
            const int64_t i = base + (int64_t)u * kEwBlock;
            if (i < nvec) {
                V r0, r1;
#pragma unroll
                for (int k = 0; k < W; ++k) {
                    const Pair<T> z = apply<T, OP, XT, YT>(a0[u][k], XT ? a1[u][k] : T(0),
                                                          HAS_Y ? b0[u][k] : T(0),
                                                          (HAS_Y && YT) ? b1[u][k] : T(0));
                    r0[k] = z.hi;
                    r1[k] = z.lo;
                }
                vstore(z0, i, r0);
                vstore(z1, i, r1);
            }
        }
    }
    if (blockIdx.x == 0) {
        const int64_t i = nvec * W + threadIdx.x;
        if (i < n) {
            const Pair<T> z = apply<T, OP, XT, YT>(x0[i], XT ? x1[i] : T(0), HAS_Y ? y0[i] : T(0),
                                                  (HAS_Y && YT) ? y1[i] : T(0));
            z0[i] = z.hi;
            z1[i] = z.lo;
        }
    }
}

template <typename T, int OP, bool XT, bool YT>
__global__ __launch_bounds__(kBlock) void ew_scalar_kernel(int64_t n, const T *x0, const T *x1,
                                                           const T *y0, const T *y1, T *z0, T *z1) {
    constexpr bool HAS_Y = !op_unary(OP);
    const int64_t step = (int64_t)gridDim.x * kBlock;
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += step) {
        const Pair<T> z = apply<T, OP, XT, YT>(x0[i], XT ? x1[i] : T(0), HAS_Y ? y0[i] : T(0),
                                              (HAS_Y && YT) ? y1[i] : T(0));
        z0[i] = z.hi;
        z1[i] = z.lo;
    }
}

template <typename T, int OP, bool XT, bool YT>
static void launch_ew(const Launch &L, int64_t n, const T *x0, const T *x1, const T *y0, const T *y1,
                      T *z0, T *z1) {
    constexpr int UNROLL = sizeof(T) == 8 ? TF_EW_UNROLL_F64
                           : op_unary(OP) ? TF_EW_UNROLL_F32_UNARY
                                          : TF_EW_UNROLL_F32;
    if (L.aligned) {
        const int64_t nvec = n / Vec<T>::N;
        const unsigned g = grid_for(nvec, (int64_t)kEwBlock * UNROLL * TF_EW_CHUNK, L.cap);
        tf_launch((ew_vec_kernel<T, OP, XT, YT, UNROLL>), dim3(g), dim3(kEwBlock), 0, L.stream,
                  n, x0, x1, y0, y1, z0, z1);
    } else {
        const unsigned g = grid_for(n, kBlock, L.cap);
        tf_launch((ew_scalar_kernel<T, OP, XT, YT>), dim3(g), dim3(kBlock), 0, L.stream, n,
                  x0, x1, y0, y1, z0, z1);
    }
}

template <typename T, int OP>
static void dispatch_ew(const Launch &L, int64_t n, const T *x0, const T *x1, const T *y0,
                        const T *y1, T *z0, T *z1) {
    const bool xt = x1 != nullptr, yt = y1 != nullptr;
    if (xt && yt) launch_ew<T, OP, true, true>(L, n, x0, x1, y0, y1, z0, z1);
    else if (xt) launch_ew<T, OP, true, false>(L, n, x0, x1, y0, y1, z0, z1);
    else if (yt) launch_ew<T, OP, false, true>(L, n, x0, x1, y0, y1, z0, z1);
    else launch_ew<T, OP, false, false>(L, n, x0, x1, y0, y1, z0, z1);
}

template <typename T, int OP>
static void dispatch_unary(const Launch &L, int64_t n, const T *x0, const T *x1, T *z0, T *z1) {
    if (x1) launch_ew<T, OP, true, false>(L, n, x0, x1, nullptr, nullptr, z0, z1);
    else launch_ew<T, OP, false, false>(L, n, x0, nullptr, nullptr, nullptr, z0, z1);
}

template <typename T>
void run_elementwise(const Launch &L, int op, int64_t n, const void *x0, const void *x1,
                     const void *y0, const void *y1, void *z0, void *z1) {
    const T *a0 = (const T *)x0, *a1 = (const T *)x1, *b0 = (const T *)y0, *b1 = (const T *)y1;
    T *c0 = (T *)z0, *c1 = (T *)z1;
    switch (op) {
    case OP_ADD: dispatch_ew<T, OP_ADD>(L, n, a0, a1, b0, b1, c0, c1); break;
    case OP_SUB: dispatch_ew<T, OP_SUB>(L, n, a0, a1, b0, b1, c0, c1); break;
    case OP_MUL: dispatch_ew<T, OP_MUL>(L, n, a0, a1, b0, b1, c0, c1); break;
    case OP_DIV: dispatch_ew<T, OP_DIV>(L, n, a0, a1, b0, b1, c0, c1); break;
    case OP_SQRT: dispatch_unary<T, OP_SQRT>(L, n, a0, a1, c0, c1); break;
    case OP_MUL_P: dispatch_ew<T, OP_MUL_P>(L, n, a0, a1, b0, b1, c0, c1); break;
    case OP_DIV_P: dispatch_ew<T, OP_DIV_P>(L, n, a0, a1, b0, b1, c0, c1); break;
    case OP_SQRT_P: dispatch_unary<T, OP_SQRT_P>(L, n, a0, a1, c0, c1); break;
    case OP_RENORM + OP_ADD: dispatch_ew<T, OP_RENORM + OP_ADD>(L, n, a0, a1, b0, b1, c0, c1); break;
    case OP_RENORM + OP_SUB: dispatch_ew<T, OP_RENORM + OP_SUB>(L, n, a0, a1, b0, b1, c0, c1); break;
    case OP_RENORM + OP_MUL_P: dispatch_ew<T, OP_RENORM + OP_MUL_P>(L, n, a0, a1, b0, b1, c0, c1); break;
    case OP_RENORM + OP_DIV_P: dispatch_ew<T, OP_RENORM + OP_DIV_P>(L, n, a0, a1, b0, b1, c0, c1); break;
    case OP_RENORM + OP_SQRT_P: dispatch_unary<T, OP_RENORM + OP_SQRT_P>(L, n, a0, a1, c0, c1); break;
    case OP_FAST_TWO_SUM:
        launch_ew<T, OP_FAST_TWO_SUM, true, false>(L, n, a0, a1, nullptr, nullptr, c0, c1);
        break;
    default: break;  // codes are checked by the caller
    }
}
template void run_elementwise<double>(const Launch &, int, int64_t, const void *, const void *,
                                      const void *, const void *, void *, void *);
template void run_elementwise<float>(const Launch &, int, int64_t, const void *, const void *,
                                     const void *, const void *, void *, void *);

// ---------------------------------------------------------------------------
// plain counterparts and the memory probe
// ---------------------------------------------------------------------------

// OP_COPY (vmem): z = x, with y read and discarded through a dependency the
// compiler cannot drop (the select never fires for finite or NaN data).
constexpr int OP_COPY = 99;

template <typename T, int OP, int UNROLL>
__global__ __launch_bounds__(kEwBlock) void plain_vec_kernel(int64_t n, const T *x, const T *y, T *z) {
    using V = typename Vec<T>::type;
    constexpr int W = Vec<T>::N;
    constexpr bool HAS_Y = OP != OP_SQRT;
    const int64_t nvec = n / W;
    for (int64_t grp = (int64_t)blockIdx.x * TF_EW_CHUNK; grp * kEwBlock * UNROLL < nvec;
         grp += (int64_t)gridDim.x * TF_EW_CHUNK)
    for (int64_t c = 0, base = grp * kEwBlock * UNROLL + threadIdx.x; c < TF_EW_CHUNK && base < nvec;
         ++c, base += (int64_t)kEwBlock * UNROLL) {
        V a[UNROLL], b[UNROLL];
#pragma unroll
        for (int u = 0; u < UNROLL; ++u) {
            const int64_t i = base + (int64_t)u * kEwBlock;
            if (i < nvec) {
                a[u] = vload(x, i);
                if constexpr (HAS_Y) b[u] = vload(y, i);
            }
        }
#pragma unroll
        for (int u = 0; u < UNROLL; ++u) {
            const int64_t i = base + (int64_t)u * kEwBlock;
            if (i < nvec) {
                V r;
#pragma unroll
                for (int k = 0; k < W; ++k) {
                    if constexpr (OP == OP_COPY) {
                        // keep the load of y live without arithmetic on the
                        // copied value: y is never exactly this bit pattern
                        r[k] = b[u][k] == T(-1.2345e-30) ? b[u][k] : a[u][k];
                    } else {
                        r[k] = apply_plain<T, OP>(a[u][k], HAS_Y ? b[u][k] : T(0));
                    }
                }
                vstore(z, i, r);
            }
        }
    }
    if (blockIdx.x == 0) {
        const int64_t i = nvec * W + threadIdx.x;
        if (i < n) {
            if constexpr (OP == OP_COPY) z[i] = x[i];
            else z[i] = apply_plain<T, OP>(x[i], HAS_Y ? y[i] : T(0));
        }
    }
}

template <typename T, int OP>
__global__ __launch_bounds__(kBlock) void plain_scalar_kernel(int64_t n, const T *x, const T *y, T *z) {
    constexpr bool HAS_Y = OP != OP_SQRT;
    const int64_t step = (int64_t)gridDim.x * kBlock;
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += step) {
        if constexpr (OP == OP_COPY) z[i] = y[i] == T(-1.2345e-30) ? y[i] : x[i];
        else z[i] = apply_plain<T, OP>(x[i], HAS_Y ? y[i] : T(0));
    }
}

template <typename T, int OP>
static void launch_plain(const Launch &L, int64_t n, const T *x, const T *y, T *z) {
    constexpr int UNROLL = TF_PLAIN_UNROLL;
    if (L.aligned) {
        const unsigned g = grid_for(n / Vec<T>::N, (int64_t)kEwBlock * UNROLL * TF_EW_CHUNK, L.cap);
        tf_launch((plain_vec_kernel<T, OP, UNROLL>), dim3(g), dim3(kEwBlock), 0, L.stream, n, x,
                  y, z);
    } else {
        const unsigned g = grid_for(n, kBlock, L.cap);
        tf_launch((plain_scalar_kernel<T, OP>), dim3(g), dim3(kBlock), 0, L.stream, n, x, y, z);
    }
}

template <typename T>
void run_plain(const Launch &L, int op, int64_t n, const void *x, const void *y, void *z) {
    const T *a = (const T *)x, *b = (const T *)y;
    T *c = (T *)z;
    switch (op) {
    case OP_ADD: launch_plain<T, OP_ADD>(L, n, a, b, c); break;
    case OP_SUB: launch_plain<T, OP_SUB>(L, n, a, b, c); break;
    case OP_MUL: launch_plain<T, OP_MUL>(L, n, a, b, c); break;
    case OP_DIV: launch_plain<T, OP_DIV>(L, n, a, b, c); break;
    case OP_SQRT: launch_plain<T, OP_SQRT>(L, n, a, b, c); break;
    default: launch_plain<T, OP_COPY>(L, n, a, b, c); break;
    }
}
template void run_plain<double>(const Launch &, int, int64_t, const void *, const void *, void *);
template void run_plain<float>(const Launch &, int, int64_t, const void *, const void *, void *);

// ---------------------------------------------------------------------------
// axpy: z = a x + y, a a twofold scalar
// ---------------------------------------------------------------------------

template <typename T, bool XT, bool YT, int UNROLL>
__global__ __launch_bounds__(kEwBlock) void axpy_vec_kernel(int64_t n, T a0, T a1, const T *x0,
                                                          const T *x1, const T *y0, const T *y1,
                                                          T *z0, T *z1) {
    using V = typename Vec<T>::type;
    constexpr int W = Vec<T>::N;
    const int64_t nvec = n / W;
    for (int64_t grp = (int64_t)blockIdx.x * TF_EW_CHUNK; grp * kEwBlock * UNROLL < nvec;
         grp += (int64_t)gridDim.x * TF_EW_CHUNK)
    for (int64_t c = 0, base = grp * kEwBlock * UNROLL + threadIdx.x; c < TF_EW_CHUNK && base < nvec;
         ++c, base += (int64_t)kEwBlock * UNROLL) {
        V p0[UNROLL], p1[UNROLL], q0[UNROLL], q1[UNROLL];
#pragma unroll
        for (int u = 0; u < UNROLL; ++u) {
            const int64_t i = base + (int64_t)u * kEwBlock;
            if (i < nvec) {
                p0[u] = vload(x0, i);
                if constexpr (XT) p1[u] = vload(x1, i);
                q0[u] = vload(y0, i);
                if constexpr (YT) q1[u] = vload(y1, i);
            }
        }
#pragma unroll
        for (int u = 0; u < UNROLL; ++u) {
            const int64_t i = base + (int64_t)u * kEwBlock;
            if (i < nvec) {
                V r0, r1;
#pragma unroll
                for (int k = 0; k < W; ++k) {
                    const Pair<T> z = axpy_one<T, XT, YT>(a0, a1, p0[u][k], XT ? p1[u][k] : T(0),
                                                         q0[u][k], YT ? q1[u][k] : T(0));
                    r0[k] = z.hi;
                    r1[k] = z.lo;
                }
                vstore(z0, i, r0);
                vstore(z1, i, r1);
            }
        }
    }
    if (blockIdx.x == 0) {
        const int64_t i = nvec * W + threadIdx.x;
        if (i < n) {
            const Pair<T> z = axpy_one<T, XT, YT>(a0, a1, x0[i], XT ? x1[i] : T(0), y0[i],
                                                 YT ? y1[i] : T(0));
            z0[i] = z.hi;
            z1[i] = z.lo;
        }
    }
}

template <typename T, bool XT, bool YT>
__global__ __launch_bounds__(kBlock) void axpy_scalar_kernel(int64_t n, T a0, T a1, const T *x0,
                                                             const T *x1, const T *y0, const T *y1,
                                                             T *z0, T *z1) {
    const int64_t step = (int64_t)gridDim.x * kBlock;
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += step) {
        const Pair<T> z =
            axpy_one<T, XT, YT>(a0, a1, x0[i], XT ? x1[i] : T(0), y0[i], YT ? y1[i] : T(0));
        z0[i] = z.hi;
        z1[i] = z.lo;
    }
}

template <typename T, bool XT, bool YT>
static void launch_axpy(const Launch &L, int64_t n, T a0, T a1, const T *x0, const T *x1,
                        const T *y0, const T *y1, T *z0, T *z1) {
    constexpr int UNROLL = sizeof(T) == 8 ? TF_EW_UNROLL_F64 : TF_EW_UNROLL_F32;
    if (L.aligned) {
        const unsigned g = grid_for(n / Vec<T>::N, (int64_t)kEwBlock * UNROLL * TF_EW_CHUNK, L.cap);
        tf_launch((axpy_vec_kernel<T, XT, YT, UNROLL>), dim3(g), dim3(kEwBlock), 0, L.stream, n,
                  a0, a1, x0, x1, y0, y1, z0, z1);
    } else {
        const unsigned g = grid_for(n, kBlock, L.cap);
        tf_launch((axpy_scalar_kernel<T, XT, YT>), dim3(g), dim3(kBlock), 0, L.stream, n, a0,
                  a1, x0, x1, y0, y1, z0, z1);
    }
}

template <typename T>
void run_axpy(const Launch &L, int64_t n, const void *a, const void *x0, const void *x1,
              const void *y0, const void *y1, void *z0, void *z1) {
    const T a0 = ((const T *)a)[0], a1 = ((const T *)a)[1];
    const T *p0 = (const T *)x0, *p1 = (const T *)x1, *q0 = (const T *)y0, *q1 = (const T *)y1;
    T *r0 = (T *)z0, *r1 = (T *)z1;
    if (p1 && q1) launch_axpy<T, true, true>(L, n, a0, a1, p0, p1, q0, q1, r0, r1);
    else if (p1) launch_axpy<T, true, false>(L, n, a0, a1, p0, p1, q0, q1, r0, r1);
    else if (q1) launch_axpy<T, false, true>(L, n, a0, a1, p0, p1, q0, q1, r0, r1);
    else launch_axpy<T, false, false>(L, n, a0, a1, p0, p1, q0, q1, r0, r1);
}
template void run_axpy<double>(const Launch &, int64_t, const void *, const void *, const void *,
                               const void *, const void *, void *, void *);
template void run_axpy<float>(const Launch &, int64_t, const void *, const void *, const void *,
                              const void *, const void *, void *, void *);

template <typename T>
__global__ __launch_bounds__(kBlock) void plain_axpy_kernel(int64_t n, T a, const T *x, const T *y, T *z,
                                                            int aligned) {
    using V = typename Vec<T>::type;
    constexpr int W = Vec<T>::N;
    const int64_t nvec = aligned ? n / W : 0;
    const int64_t step = (int64_t)gridDim.x * kBlock;
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < nvec; i += step) {
        const V p = vload(x, i), q = vload(y, i);
        V r;
#pragma unroll
        for (int k = 0; k < W; ++k) r[k] = a * p[k] + q[k];
        vstore(z, i, r);
    }
    for (int64_t i = nvec * W + (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += step)
        z[i] = a * x[i] + y[i];
}

template <typename T>
void run_plain_axpy(const Launch &L, int64_t n, const void *a, const void *x, const void *y, void *z) {
    const unsigned g = grid_for(L.aligned ? n / Vec<T>::N : n, kBlock, L.cap);
    tf_launch((plain_axpy_kernel<T>), dim3(g), dim3(kBlock), 0, L.stream, n, ((const T *)a)[0],
              (const T *)x, (const T *)y, (T *)z, (int)L.aligned);
}
template void run_plain_axpy<double>(const Launch &, int64_t, const void *, const void *, const void *,
                                     void *);
template void run_plain_axpy<float>(const Launch &, int64_t, const void *, const void *, const void *,
                                    void *);

// ---------------------------------------------------------------------------
// Horner: coefficients travel by value in the kernel arguments
// ---------------------------------------------------------------------------

template <typename T, bool XT>
__global__ __launch_bounds__(kBlock) void horner_kernel(int64_t n, int degree, Coeffs<T> C, const T *x0,
                                                        const T *x1, T *z0, T *z1, int aligned) {
    using V = typename Vec<T>::type;
    constexpr int W = Vec<T>::N;
    const int64_t nvec = aligned ? n / W : 0;
    const int64_t step = (int64_t)gridDim.x * kBlock;
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < nvec; i += step) {
        const V p0 = vload(x0, i);
        V p1;
        if constexpr (XT) p1 = vload(x1, i);
        V r0, r1;
#pragma unroll
        for (int k = 0; k < W; ++k) {
            const Pair<T> z = horner_one<T, XT>(C, degree, p0[k], XT ? p1[k] : T(0));
            r0[k] = z.hi;
            r1[k] = z.lo;
        }
        vstore(z0, i, r0);
        vstore(z1, i, r1);
    }
    for (int64_t i = nvec * W + (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += step) {
        const Pair<T> z = horner_one<T, XT>(C, degree, x0[i], XT ? x1[i] : T(0));
        z0[i] = z.hi;
        z1[i] = z.lo;
    }
}

template <typename T>
void run_horner(const Launch &L, int64_t n, int degree, const void *c, const void *x0, const void *x1,
                void *z0, void *z1) {
    Coeffs<T> C{};
    for (int k = 0; k <= degree; ++k) C.c[k] = ((const T *)c)[k];
    const unsigned g = grid_for(L.aligned ? n / Vec<T>::N : n, kBlock, L.cap);
    if (x1)
        tf_launch((horner_kernel<T, true>), dim3(g), dim3(kBlock), 0, L.stream, n, degree, C,
                  (const T *)x0, (const T *)x1, (T *)z0, (T *)z1, (int)L.aligned);
    else
        tf_launch((horner_kernel<T, false>), dim3(g), dim3(kBlock), 0, L.stream, n, degree, C,
                  (const T *)x0, (const T *)nullptr, (T *)z0, (T *)z1, (int)L.aligned);
}
template void run_horner<double>(const Launch &, int64_t, int, const void *, const void *, const void *,
                                 void *, void *);
template void run_horner<float>(const Launch &, int64_t, int, const void *, const void *, const void *,
                                void *, void *);

template <typename T>
__global__ __launch_bounds__(kBlock) void plain_horner_kernel(int64_t n, int degree, Coeffs<T> C,
                                                              const T *x, T *z, int aligned) {
    using V = typename Vec<T>::type;
    constexpr int W = Vec<T>::N;
    const int64_t nvec = aligned ? n / W : 0;
    const int64_t step = (int64_t)gridDim.x * kBlock;
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < nvec; i += step) {
        const V p = vload(x, i);
        V r;
#pragma unroll
        for (int k = 0; k < W; ++k) {
            T acc = C.c[degree];
            for (int j = degree - 1; j >= 0; --j) acc = acc * p[k] + C.c[j];
            r[k] = acc;
        }
        vstore(z, i, r);
    }
    for (int64_t i = nvec * W + (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += step) {
        T acc = C.c[degree];
        for (int j = degree - 1; j >= 0; --j) acc = acc * x[i] + C.c[j];
        z[i] = acc;
    }
}

template <typename T>
void run_plain_horner(const Launch &L, int64_t n, int degree, const void *c, const void *x, void *z) {
    Coeffs<T> C{};
    for (int k = 0; k <= degree; ++k) C.c[k] = ((const T *)c)[k];
    const unsigned g = grid_for(L.aligned ? n / Vec<T>::N : n, kBlock, L.cap);
    tf_launch((plain_horner_kernel<T>), dim3(g), dim3(kBlock), 0, L.stream, n, degree, C,
              (const T *)x, (T *)z, (int)L.aligned);
}
template void run_plain_horner<double>(const Launch &, int64_t, int, const void *, const void *, void *);
template void run_plain_horner<float>(const Launch &, int64_t, int, const void *, const void *, void *);

}  // namespace tf
