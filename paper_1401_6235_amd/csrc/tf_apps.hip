// Batched applications of the paper (Applications section) and the twofold
// fma: many independent small problems, one per thread, each solved with
// the twofold operations in the order its formula gives.
//
//  * Back-substitution for upper-triangular m x m systems (the Jordan-block
//    solve is the bidiagonal case).  Systems are interleaved in memory, so
//    one index runs over systems and every load of a wave is coalesced.  For
//    m <= 16 the order is a template constant and the solution stays in
//    registers; larger orders read the entries a thread has already
//    produced back from the output, where they are still cached.  Bound by
//    reading the matrices.
//  * Both roots of a quadratic by the school formula, NaN flowing through a
//    negative discriminant.  Elementwise, bound by HBM.
//  * z = x y + w with a twofold result.  Elementwise, bound by HBM.
#include "tf_internal.hpp"

namespace tf {

// ---- back-substitution ----------------------------------------------------------

template <typename T, bool UT, bool FT>
__global__ __launch_bounds__(kBlock) void trsv_kernel(int64_t nsys, int m, const T *U0, const T *U1,
                                                      const T *f0, const T *f1, T *x0, T *x1) {
    const int64_t step = (int64_t)gridDim.x * kBlock;
    for (int64_t k = (int64_t)blockIdx.x * kBlock + threadIdx.x; k < nsys; k += step) {
        for (int i = m - 1; i >= 0; --i) {
            const int64_t fi = (int64_t)i * nsys + k;
            Pair<T> s{f0[fi], FT ? f1[fi] : T(0)};
            for (int j = i + 1; j < m; ++j) {
                const int64_t a = ((int64_t)i * m + j) * nsys + k, b = (int64_t)j * nsys + k;
                const Pair<T> p = UT ? mul_tt(U0[a], U1[a], x0[b], x1[b]) : mul_dt(U0[a], x0[b], x1[b]);
                s = sub_tt(s.hi, s.lo, p.hi, p.lo);
            }
            const int64_t d = ((int64_t)i * m + i) * nsys + k;
            const Pair<T> x = UT ? div_tt(s.hi, s.lo, U0[d], U1[d]) : div_td(s.hi, s.lo, U0[d]);
            x0[fi] = x.hi;
            x1[fi] = x.lo;
        }
    }
}

// Orders up to kTrsvFixed: m is a compile-time constant, every loop is
// unrolled and the solution stays in registers.  Each row's operands (its
// part of U and of f) are read into registers before the row is computed,
// and with TF_TRSV_PREFETCH the next row's are read before the current row
// is computed: left to the compiler, the loads were interleaved with the
// dependent arithmetic and the wave waited for memory about 116 times per
// system batch instead of once per row.
constexpr int kTrsvFixed = 16;
#ifndef TF_TRSV_PREFETCH
#define TF_TRSV_PREFETCH 1
#endif

// Row i of system k: U[i][j] for j = i .. M-1 (twofold or dotted) and f_i.
template <typename T, int M, bool UT, bool FT>
struct TrsvRow {
    T u0[M], u1[M], f0, f1;
    __device__ __forceinline__ void load(int i, int64_t nsys, int64_t k, const T *U0, const T *U1, const T *F0,
                                         const T *F1) {
        f0 = F0[(int64_t)i * nsys + k];
        f1 = FT ? F1[(int64_t)i * nsys + k] : T(0);
#pragma unroll
        for (int j = 0; j < M; ++j) {
            if (j >= i) {
                const int64_t a = (int64_t)(i * M + j) * nsys + k;
                u0[j] = U0[a];
                u1[j] = UT ? U1[a] : T(0);
            }
        }
    }
};

template <typename T, int M, bool UT, bool FT>
__global__ __launch_bounds__(kBlock) void trsv_fixed_kernel(int64_t nsys, const T *U0, const T *U1, const T *f0,
                                                            const T *f1, T *x0, T *x1) {
    const int64_t step = (int64_t)gridDim.x * kBlock;
    for (int64_t k = (int64_t)blockIdx.x * kBlock + threadIdx.x; k < nsys; k += step) {
        T r0[M], r1[M];
        TrsvRow<T, M, UT, FT> row;
        row.load(M - 1, nsys, k, U0, U1, f0, f1);
#pragma unroll
        for (int i = M - 1; i >= 0; --i) {
            TrsvRow<T, M, UT, FT> next;
            if (TF_TRSV_PREFETCH && i > 0) next.load(i - 1, nsys, k, U0, U1, f0, f1);
            // keep the scheduler from sinking those loads into the row's
            // arithmetic: they stay in flight while the row is computed
            __builtin_amdgcn_sched_barrier(0);
            Pair<T> s{row.f0, row.f1};
#pragma unroll
            for (int j = i + 1; j < M; ++j) {
                const Pair<T> p = UT ? mul_tt(row.u0[j], row.u1[j], r0[j], r1[j]) : mul_dt(row.u0[j], r0[j], r1[j]);
                s = sub_tt(s.hi, s.lo, p.hi, p.lo);
            }
            const Pair<T> x = UT ? div_tt(s.hi, s.lo, row.u0[i], row.u1[i]) : div_td(s.hi, s.lo, row.u0[i]);
            r0[i] = x.hi;
            r1[i] = x.lo;
            if (i > 0) {
                if (TF_TRSV_PREFETCH) row = next;
                else row.load(i - 1, nsys, k, U0, U1, f0, f1);
            }
        }
#pragma unroll
        for (int i = 0; i < M; ++i) {
            x0[(int64_t)i * nsys + k] = r0[i];
            x1[(int64_t)i * nsys + k] = r1[i];
        }
    }
}

template <typename T, int M>
__global__ __launch_bounds__(kBlock) void plain_trsv_fixed_kernel(int64_t nsys, const T *U, const T *f, T *x) {
    const int64_t step = (int64_t)gridDim.x * kBlock;
    for (int64_t k = (int64_t)blockIdx.x * kBlock + threadIdx.x; k < nsys; k += step) {
        T r[M];
        TrsvRow<T, M, false, false> row;  // the same row staging as the twofold kernel
        row.load(M - 1, nsys, k, U, nullptr, f, nullptr);
#pragma unroll
        for (int i = M - 1; i >= 0; --i) {
            TrsvRow<T, M, false, false> next;
            if (TF_TRSV_PREFETCH && i > 0) next.load(i - 1, nsys, k, U, nullptr, f, nullptr);
            __builtin_amdgcn_sched_barrier(0);
            T s = row.f0;
#pragma unroll
            for (int j = i + 1; j < M; ++j) s = s - row.u0[j] * r[j];
            r[i] = s / row.u0[i];
            if (i > 0) {
                if (TF_TRSV_PREFETCH) row = next;
                else row.load(i - 1, nsys, k, U, nullptr, f, nullptr);
            }
        }
#pragma unroll
        for (int i = 0; i < M; ++i) x[(int64_t)i * nsys + k] = r[i];
    }
}

template <typename T, int M>
static void launch_trsv_fixed(const Launch &L, int64_t nsys, const T *a0, const T *a1, const T *b0, const T *b1,
                              T *c0, T *c1) {
    const dim3 g(grid_for(nsys, kBlock, 0)), b(kBlock);
    if (a1 && b1) tf_launch((trsv_fixed_kernel<T, M, true, true>), g, b, 0, L.stream, nsys, a0, a1, b0, b1, c0, c1);
    else if (a1) tf_launch((trsv_fixed_kernel<T, M, true, false>), g, b, 0, L.stream, nsys, a0, a1, b0, b1, c0, c1);
    else if (b1) tf_launch((trsv_fixed_kernel<T, M, false, true>), g, b, 0, L.stream, nsys, a0, a1, b0, b1, c0, c1);
    else tf_launch((trsv_fixed_kernel<T, M, false, false>), g, b, 0, L.stream, nsys, a0, a1, b0, b1, c0, c1);
}

template <typename T, int M = 1>
static bool dispatch_trsv_fixed(const Launch &L, int m, int64_t nsys, const T *a0, const T *a1, const T *b0,
                                const T *b1, T *c0, T *c1, const T *pu, const T *pf, T *px, bool plain) {
    if constexpr (M > kTrsvFixed) {
        return false;
    } else {
        if (m != M)
            return dispatch_trsv_fixed<T, M + 1>(L, m, nsys, a0, a1, b0, b1, c0, c1, pu, pf, px, plain);
        if (plain)
            tf_launch((plain_trsv_fixed_kernel<T, M>), dim3(grid_for(nsys, kBlock, 0)), dim3(kBlock), 0,
                      L.stream, nsys, pu, pf, px);
        else
            launch_trsv_fixed<T, M>(L, nsys, a0, a1, b0, b1, c0, c1);
        return true;
    }
}

template <typename T>
__global__ __launch_bounds__(kBlock) void plain_trsv_kernel(int64_t nsys, int m, const T *U, const T *f, T *x) {
    const int64_t step = (int64_t)gridDim.x * kBlock;
    for (int64_t k = (int64_t)blockIdx.x * kBlock + threadIdx.x; k < nsys; k += step) {
        for (int i = m - 1; i >= 0; --i) {
            T s = f[(int64_t)i * nsys + k];
            for (int j = i + 1; j < m; ++j) s = s - U[((int64_t)i * m + j) * nsys + k] * x[(int64_t)j * nsys + k];
            x[(int64_t)i * nsys + k] = s / U[((int64_t)i * m + i) * nsys + k];
        }
    }
}

template <typename T>
void run_trsv(const Launch &L, int64_t nsys, int m, const void *U0, const void *U1, const void *f0,
              const void *f1, void *x0, void *x1) {
    const unsigned g = grid_for(nsys, kBlock, 0);
    const T *a0 = (const T *)U0, *a1 = (const T *)U1, *b0 = (const T *)f0, *b1 = (const T *)f1;
    T *c0 = (T *)x0, *c1 = (T *)x1;
    if (dispatch_trsv_fixed<T>(L, m, nsys, a0, a1, b0, b1, c0, c1, nullptr, nullptr, nullptr, false)) return;
    if (U1 && f1)
        tf_launch((trsv_kernel<T, true, true>), dim3(g), dim3(kBlock), 0, L.stream, nsys, m, a0, a1, b0,
                  b1, c0, c1);
    else if (U1)
        tf_launch((trsv_kernel<T, true, false>), dim3(g), dim3(kBlock), 0, L.stream, nsys, m, a0, a1,
                  b0, nullptr, c0, c1);
    else if (f1)
        tf_launch((trsv_kernel<T, false, true>), dim3(g), dim3(kBlock), 0, L.stream, nsys, m, a0,
                  nullptr, b0, b1, c0, c1);
    else
        tf_launch((trsv_kernel<T, false, false>), dim3(g), dim3(kBlock), 0, L.stream, nsys, m, a0,
                  nullptr, b0, nullptr, c0, c1);
}
template void run_trsv<double>(const Launch &, int64_t, int, const void *, const void *, const void *,
                               const void *, void *, void *);
template void run_trsv<float>(const Launch &, int64_t, int, const void *, const void *, const void *,
                              const void *, void *, void *);

template <typename T>
void run_plain_trsv(const Launch &L, int64_t nsys, int m, const void *U, const void *f, void *x) {
    if (dispatch_trsv_fixed<T>(L, m, nsys, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, (const T *)U,
                               (const T *)f, (T *)x, true))
        return;
    tf_launch((plain_trsv_kernel<T>), dim3(grid_for(nsys, kBlock, 0)), dim3(kBlock), 0, L.stream, nsys,
              m, (const T *)U, (const T *)f, (T *)x);
}
template void run_plain_trsv<double>(const Launch &, int64_t, int, const void *, const void *, void *);
template void run_plain_trsv<float>(const Launch &, int64_t, int, const void *, const void *, void *);

// ---- quadratic -------------------------------------------------------------------

// q = b b - (4 a) c; d = RTF1(q); e = 2 a; r = (-b - d) / e; s = (-b + d) / e.
template <typename T>
__device__ __forceinline__ void quadratic_one(T a0, T a1, T b0, T b1, T c0, T c1, Pair<T> &r, Pair<T> &s) {
    const Pair<T> bb = mul_tt(b0, b1, b0, b1);
    const Pair<T> a4 = mul_tt(T(4), T(0), a0, a1);
    const Pair<T> ac = mul_tt(a4.hi, a4.lo, c0, c1);
    const Pair<T> q = sub_tt(bb.hi, bb.lo, ac.hi, ac.lo);
    const Pair<T> d = sqrt_t(q.hi, q.lo);
    const Pair<T> e = mul_tt(T(2), T(0), a0, a1);
    const Pair<T> u = sub_tt(-b0, -b1, d.hi, d.lo);
    const Pair<T> v = add_tt(-b0, -b1, d.hi, d.lo);
    r = div_tt(u.hi, u.lo, e.hi, e.lo);
    s = div_tt(v.hi, v.lo, e.hi, e.lo);
}

template <typename T>
__global__ __launch_bounds__(kBlock) void quadratic_kernel(int64_t n, const T *a0, const T *a1, const T *b0,
                                                           const T *b1, const T *c0, const T *c1, T *r0, T *r1,
                                                           T *s0, T *s1) {
    const int64_t step = (int64_t)gridDim.x * kBlock;
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += step) {
        Pair<T> r, s;
        quadratic_one(a0[i], a1[i], b0[i], b1[i], c0[i], c1[i], r, s);
        r0[i] = r.hi;
        r1[i] = r.lo;
        s0[i] = s.hi;
        s1[i] = s.lo;
    }
}

template <typename T>
__global__ __launch_bounds__(kBlock) void plain_quadratic_kernel(int64_t n, const T *a, const T *b, const T *c,
                                                                 T *r, T *s) {
    const int64_t step = (int64_t)gridDim.x * kBlock;
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += step) {
        const T q = b[i] * b[i] - (T(4) * a[i]) * c[i];
        const T d = sqrt_rn(q);
        const T e = T(2) * a[i];
        r[i] = (-b[i] - d) / e;
        s[i] = (-b[i] + d) / e;
    }
}

// 16-byte vectors of every array, one per thread; the ragged tail by block 0.
template <typename T>
__global__ __launch_bounds__(kBlock) void quadratic_vec_kernel(int64_t n, const T *a0, const T *a1, const T *b0,
                                                               const T *b1, const T *c0, const T *c1, T *r0,
                                                               T *r1, T *s0, T *s1) {
    using V = typename Vec<T>::type;
    constexpr int W = Vec<T>::N;
    const int64_t nvec = n / W;
    const int64_t step = (int64_t)gridDim.x * kBlock;
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < nvec; i += step) {
        const V pa0 = vload(a0, i), pa1 = vload(a1, i), pb0 = vload(b0, i), pb1 = vload(b1, i);
        const V pc0 = vload(c0, i), pc1 = vload(c1, i);
        V qr0, qr1, qs0, qs1;
#pragma unroll
        for (int k = 0; k < W; ++k) {
            Pair<T> r, s;
            quadratic_one(pa0[k], pa1[k], pb0[k], pb1[k], pc0[k], pc1[k], r, s);
            qr0[k] = r.hi;
            qr1[k] = r.lo;
            qs0[k] = s.hi;
            qs1[k] = s.lo;
        }
        vstore(r0, i, qr0);
        vstore(r1, i, qr1);
        vstore(s0, i, qs0);
        vstore(s1, i, qs1);
    }
    if (blockIdx.x == 0) {
        const int64_t i = nvec * W + threadIdx.x;
        if (i < n) {
            Pair<T> r, s;
            quadratic_one(a0[i], a1[i], b0[i], b1[i], c0[i], c1[i], r, s);
            r0[i] = r.hi;
            r1[i] = r.lo;
            s0[i] = s.hi;
            s1[i] = s.lo;
        }
    }
}

template <typename T>
void run_quadratic(const Launch &L, int64_t n, const void *const *in, void *const *out) {
    const T *a0 = (const T *)in[0], *a1 = (const T *)in[1], *b0 = (const T *)in[2], *b1 = (const T *)in[3];
    const T *c0 = (const T *)in[4], *c1 = (const T *)in[5];
    T *r0 = (T *)out[0], *r1 = (T *)out[1], *s0 = (T *)out[2], *s1 = (T *)out[3];
    if (L.aligned)
        tf_launch((quadratic_vec_kernel<T>), dim3(grid_for(n / Vec<T>::N, kBlock, L.cap)), dim3(kBlock), 0,
                  L.stream, n, a0, a1, b0, b1, c0, c1, r0, r1, s0, s1);
    else
        tf_launch((quadratic_kernel<T>), dim3(grid_for(n, kBlock, L.cap)), dim3(kBlock), 0, L.stream, n,
                  a0, a1, b0, b1, c0, c1, r0, r1, s0, s1);
}
template void run_quadratic<double>(const Launch &, int64_t, const void *const *, void *const *);
template void run_quadratic<float>(const Launch &, int64_t, const void *const *, void *const *);

template <typename T>
void run_plain_quadratic(const Launch &L, int64_t n, const void *a, const void *b, const void *c, void *r,
                         void *s) {
    tf_launch((plain_quadratic_kernel<T>), dim3(grid_for(n, kBlock, L.cap)), dim3(kBlock), 0, L.stream,
              n, (const T *)a, (const T *)b, (const T *)c, (T *)r, (T *)s);
}
template void run_plain_quadratic<double>(const Launch &, int64_t, const void *, const void *, const void *,
                                          void *, void *);
template void run_plain_quadratic<float>(const Launch &, int64_t, const void *, const void *, const void *,
                                         void *, void *);

// ---- fma ------------------------------------------------------------------------

#ifndef TF_FMA_UNROLL_F64
#define TF_FMA_UNROLL_F64 4
#endif
#ifndef TF_FMA_UNROLL_F32
#define TF_FMA_UNROLL_F32 4
#endif
template <typename T>
struct FmaUnroll {
    static constexpr int U = sizeof(T) == 8 ? TF_FMA_UNROLL_F64 : TF_FMA_UNROLL_F32;
};

// U 16-byte vectors per operand and thread, consecutive threads on
// consecutive vectors within each of the U strips of the block.
template <typename T, bool XT, bool YT, bool WT>
__global__ __launch_bounds__(kBlock) void fma_vec_kernel(int64_t n, const T *x0, const T *x1, const T *y0,
                                                         const T *y1, const T *w0, const T *w1, T *z0, T *z1) {
    using V = typename Vec<T>::type;
    constexpr int W = Vec<T>::N;
    constexpr int U = FmaUnroll<T>::U;
    const int64_t nvec = n / W;
    const int64_t step = (int64_t)gridDim.x * kBlock * U;
    for (int64_t base = (int64_t)blockIdx.x * kBlock * U + threadIdx.x; base < nvec; base += step) {
        V p0[U], q0[U], s0[U], p1[U], q1[U], s1[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t i = base + (int64_t)u * kBlock;
            if (i < nvec) {
                p0[u] = vload(x0, i);
                q0[u] = vload(y0, i);
                s0[u] = vload(w0, i);
                if constexpr (XT) p1[u] = vload(x1, i);
                if constexpr (YT) q1[u] = vload(y1, i);
                if constexpr (WT) s1[u] = vload(w1, i);
            }
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t i = base + (int64_t)u * kBlock;
            if (i < nvec) {
                V r0, r1;
#pragma unroll
                for (int k = 0; k < W; ++k) {
                    const Pair<T> z = fma_t<T, XT, YT, WT>(p0[u][k], XT ? p1[u][k] : T(0), q0[u][k],
                                                           YT ? q1[u][k] : T(0), s0[u][k], WT ? s1[u][k] : T(0));
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
            const Pair<T> z = fma_t<T, XT, YT, WT>(x0[i], XT ? x1[i] : T(0), y0[i], YT ? y1[i] : T(0), w0[i],
                                                   WT ? w1[i] : T(0));
            z0[i] = z.hi;
            z1[i] = z.lo;
        }
    }
}

template <typename T, bool XT, bool YT, bool WT>
__global__ __launch_bounds__(kBlock) void fma_scalar_kernel(int64_t n, const T *x0, const T *x1, const T *y0,
                                                            const T *y1, const T *w0, const T *w1, T *z0,
                                                            T *z1) {
    const int64_t step = (int64_t)gridDim.x * kBlock;
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += step) {
        const Pair<T> z = fma_t<T, XT, YT, WT>(x0[i], XT ? x1[i] : T(0), y0[i], YT ? y1[i] : T(0), w0[i],
                                               WT ? w1[i] : T(0));
        z0[i] = z.hi;
        z1[i] = z.lo;
    }
}

template <typename T, bool XT, bool YT, bool WT>
static void launch_fma(const Launch &L, int64_t n, const T *const *p, T *z0, T *z1) {
    if (L.aligned)
        tf_launch((fma_vec_kernel<T, XT, YT, WT>),
                  dim3(grid_for((n / Vec<T>::N + FmaUnroll<T>::U - 1) / FmaUnroll<T>::U, kBlock, L.cap)),
                  dim3(kBlock), 0, L.stream, n, p[0], p[1], p[2], p[3], p[4], p[5], z0, z1);
    else
        tf_launch((fma_scalar_kernel<T, XT, YT, WT>), dim3(grid_for(n, kBlock, L.cap)), dim3(kBlock), 0,
                  L.stream, n, p[0], p[1], p[2], p[3], p[4], p[5], z0, z1);
}

template <typename T>
void run_fma(const Launch &L, int64_t n, const void *const *in, void *z0, void *z1) {
    const T *p[6];
    for (int k = 0; k < 6; ++k) p[k] = (const T *)in[k];
    T *a = (T *)z0, *b = (T *)z1;
    const int form = (p[1] ? 4 : 0) | (p[3] ? 2 : 0) | (p[5] ? 1 : 0);
    switch (form) {
    case 7: launch_fma<T, true, true, true>(L, n, p, a, b); break;
    case 6: launch_fma<T, true, true, false>(L, n, p, a, b); break;
    case 5: launch_fma<T, true, false, true>(L, n, p, a, b); break;
    case 4: launch_fma<T, true, false, false>(L, n, p, a, b); break;
    case 3: launch_fma<T, false, true, true>(L, n, p, a, b); break;
    case 2: launch_fma<T, false, true, false>(L, n, p, a, b); break;
    case 1: launch_fma<T, false, false, true>(L, n, p, a, b); break;
    default: launch_fma<T, false, false, false>(L, n, p, a, b); break;
    }
}
template void run_fma<double>(const Launch &, int64_t, const void *const *, void *, void *);
template void run_fma<float>(const Launch &, int64_t, const void *const *, void *, void *);

template <typename T>
__global__ __launch_bounds__(kBlock) void plain_fma_kernel(int64_t n, const T *x, const T *y, const T *w, T *z) {
    const int64_t step = (int64_t)gridDim.x * kBlock;
    for (int64_t i = (int64_t)blockIdx.x * kBlock + threadIdx.x; i < n; i += step) z[i] = fma_rn(x[i], y[i], w[i]);
}

template <typename T>
void run_plain_fma(const Launch &L, int64_t n, const void *x, const void *y, const void *w, void *z) {
    tf_launch((plain_fma_kernel<T>), dim3(grid_for(n, kBlock, L.cap)), dim3(kBlock), 0, L.stream, n,
              (const T *)x, (const T *)y, (const T *)w, (T *)z);
}
template void run_plain_fma<double>(const Launch &, int64_t, const void *, const void *, const void *, void *);
template void run_plain_fma<float>(const Launch &, int64_t, const void *, const void *, const void *, void *);

}  // namespace tf
