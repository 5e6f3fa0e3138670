// C-ABI entry points: argument checks, variant and type dispatch, launch.
#include <stdint.h>

#include "tf_internal.hpp"

namespace tf {

Config &config() {
    static Config c;
    return c;
}

int num_cus() {
    static int cus = [] {
        int dev = 0, v = 0;
        if (hipGetDevice(&dev) != hipSuccess) return 256;
        if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || v <= 0)
            return 256;
        return v;
    }();
    return cus;
}

static bool aligned16(const void *p) { return p == nullptr || ((uintptr_t)p & 15u) == 0; }

// Every entry point makes its Launch before its first kernel launch, which
// starts the call's own launch status afresh.
static Launch make_launch(hipStream_t stream, std::initializer_list<const void *> ptrs) {
    call_status() = hipSuccess;
    Launch L;
    L.stream = stream;
    L.aligned = true;
    for (const void *p : ptrs) L.aligned = L.aligned && aligned16(p);
    const int64_t bpc = config().ew_blocks_per_cu;
    L.cap = bpc > 0 ? bpc * num_cus() : 0;
    return L;
}

static int size_of(int dtype) { return dtype == TF_F64 ? 8 : dtype == TF_F32 ? 4 : 0; }

// The status of this call's launches only: an error that other code left
// in the thread's HIP state is neither returned nor cleared.
static int finish() { return call_status() == hipSuccess ? TF_OK : TF_EDEVICE; }

}  // namespace tf

using namespace tf;

#define TF_CHECK(cond)                                                                             \
    do {                                                                                           \
        if (!(cond)) return TF_EINVAL;                                                             \
    } while (0)

extern "C" {

const char *tf_strerror(int status) {
    switch (status) {
    case TF_OK: return "success";
    case TF_EINVAL: return "invalid argument";
    case TF_EDEVICE: return "HIP call or kernel launch failed";
    case TF_ENOMEM: return "workspace too small or out of memory";
    case TF_EBUSY: return "resource temporarily exhausted";
    case TF_ESTATE: return "call not valid in the current state";
    default: return "unknown status";
    }
}

int tf_version(void) { return 10000; }

int64_t tf_config(int key, int64_t value) {
    Config &c = config();
    if (key == TF_CFG_EW_BLOCKS_PER_CU) {
        if (value < 0) return TF_EINVAL;
        const int64_t old = c.ew_blocks_per_cu;
        c.ew_blocks_per_cu = value;
        return old;
    }
    if (key == TF_CFG_RED_TILES_PER_BLOCK) {
        if (value < 0 || value > 256 || (value & (value - 1))) return TF_EINVAL;
        const int64_t old = c.red_tiles_per_block;
        c.red_tiles_per_block = value;
        return old;
    }
    if (key == TF_CFG_RED_WAVES) {
        if (value != 0 && value != 4 && value != 8 && value != 16) return TF_EINVAL;
        const int64_t old = c.red_waves;
        c.red_waves = value;
        return old;
    }
    return TF_EINVAL;
}

static int binary(int op, int dtype, int64_t n, const void *x0, const void *x1, const void *y0,
                  const void *y1, void *z0, void *z1, hipStream_t stream) {
    TF_CHECK(size_of(dtype) && n >= 0);
    if (n == 0) return TF_OK;
    TF_CHECK(x0 && y0 && z0 && z1);
    const Launch L = make_launch(stream, {x0, x1, y0, y1, z0, z1});
    if (dtype == TF_F64) run_elementwise<double>(L, op, n, x0, x1, y0, y1, z0, z1);
    else run_elementwise<float>(L, op, n, x0, x1, y0, y1, z0, z1);
    return finish();
}

int tf_add(int dtype, int64_t n, const void *x0, const void *x1, const void *y0, const void *y1,
           void *z0, void *z1, hipStream_t stream) {
    return binary(OP_ADD, dtype, n, x0, x1, y0, y1, z0, z1, stream);
}
int tf_sub(int dtype, int64_t n, const void *x0, const void *x1, const void *y0, const void *y1,
           void *z0, void *z1, hipStream_t stream) {
    return binary(OP_SUB, dtype, n, x0, x1, y0, y1, z0, z1, stream);
}
int tf_mul(int dtype, int64_t n, const void *x0, const void *x1, const void *y0, const void *y1,
           void *z0, void *z1, hipStream_t stream) {
    return binary(OP_MUL, dtype, n, x0, x1, y0, y1, z0, z1, stream);
}
int tf_div(int dtype, int64_t n, const void *x0, const void *x1, const void *y0, const void *y1,
           void *z0, void *z1, hipStream_t stream) {
    return binary(OP_DIV, dtype, n, x0, x1, y0, y1, z0, z1, stream);
}

int tf_sqrt(int dtype, int64_t n, const void *x0, const void *x1, void *z0, void *z1,
            hipStream_t stream) {
    TF_CHECK(size_of(dtype) && n >= 0);
    if (n == 0) return TF_OK;
    TF_CHECK(x0 && z0 && z1);
    const Launch L = make_launch(stream, {x0, x1, z0, z1});
    if (dtype == TF_F64) run_elementwise<double>(L, OP_SQRT, n, x0, x1, nullptr, nullptr, z0, z1);
    else run_elementwise<float>(L, OP_SQRT, n, x0, x1, nullptr, nullptr, z0, z1);
    return finish();
}

int tf_axpy(int dtype, int64_t n, const void *a, const void *x0, const void *x1, const void *y0,
            const void *y1, void *z0, void *z1, hipStream_t stream) {
    TF_CHECK(size_of(dtype) && n >= 0 && a);
    if (n == 0) return TF_OK;
    TF_CHECK(x0 && y0 && z0 && z1);
    const Launch L = make_launch(stream, {x0, x1, y0, y1, z0, z1});
    if (dtype == TF_F64) run_axpy<double>(L, n, a, x0, x1, y0, y1, z0, z1);
    else run_axpy<float>(L, n, a, x0, x1, y0, y1, z0, z1);
    return finish();
}

int tf_horner(int dtype, int64_t n, int degree, const void *c, const void *x0, const void *x1,
              void *z0, void *z1, hipStream_t stream) {
    TF_CHECK(size_of(dtype) && n >= 0 && c && degree >= 0 && degree <= TF_MAX_DEGREE);
    if (n == 0) return TF_OK;
    TF_CHECK(x0 && z0 && z1);
    const Launch L = make_launch(stream, {x0, x1, z0, z1});
    if (dtype == TF_F64) run_horner<double>(L, n, degree, c, x0, x1, z0, z1);
    else run_horner<float>(L, n, degree, c, x0, x1, z0, z1);
    return finish();
}

size_t tf_reduce_workspace_bytes(int dtype, int64_t n) {
    const int s = size_of(dtype);
    if (!s || n <= 0) return 0;
    const int64_t tiles = (n + 255) / 256;
    // one partial per tile at most (one tile per block), plus the next level
    return (size_t)(tiles + tiles / 256 + 4) * 2 * (size_t)s;
}

static int reduce(int leaf, int dtype, int64_t n, const void *x0, const void *x1, const void *y0,
                  const void *y1, void *out, void *work, size_t work_bytes, hipStream_t stream) {
    TF_CHECK(size_of(dtype) && n >= 0 && out);
    const size_t need = tf_reduce_workspace_bytes(dtype, n);
    if (n > 0) TF_CHECK(x0);
    if (need > 0 && (work == nullptr || work_bytes < need)) return TF_ENOMEM;
    const Launch L = make_launch(stream, {x0, x1, y0, y1});
    const int64_t pb = tiles_per_block(size_of(dtype), leaf);
    if (dtype == TF_F64) run_reduce<double>(L, leaf, n, pb, x0, x1, y0, y1, out, work);
    else run_reduce<float>(L, leaf, n, pb, x0, x1, y0, y1, out, work);
    return finish();
}

int tf_sum(int dtype, int64_t n, const void *x0, const void *x1, void *out, void *work,
           size_t work_bytes, hipStream_t stream) {
    return reduce(x1 ? LEAF_SUM_T : LEAF_SUM_D, dtype, n, x0, x1, nullptr, nullptr, out, work,
                  work_bytes, stream);
}

int tf_dot(int dtype, int64_t n, const void *x0, const void *x1, const void *y0, const void *y1,
           void *out, void *work, size_t work_bytes, hipStream_t stream) {
    if (n > 0) TF_CHECK(y0);
    const int leaf = x1 && y1 ? LEAF_DOT_TT : x1 ? LEAF_DOT_TD : y1 ? LEAF_DOT_DT : LEAF_DOT_DD;
    return reduce(leaf, dtype, n, x0, x1, y0, y1, out, work, work_bytes, stream);
}

static int plain_binary(int op, int dtype, int64_t n, const void *x, const void *y, void *z,
                        hipStream_t stream) {
    TF_CHECK(size_of(dtype) && n >= 0);
    if (n == 0) return TF_OK;
    TF_CHECK(x && z && (y || op == OP_SQRT));
    const Launch L = make_launch(stream, {x, y, z});
    if (dtype == TF_F64) run_plain<double>(L, op, n, x, y, z);
    else run_plain<float>(L, op, n, x, y, z);
    return finish();
}

int tf_plain_add(int dtype, int64_t n, const void *x, const void *y, void *z, hipStream_t stream) {
    return plain_binary(OP_ADD, dtype, n, x, y, z, stream);
}
int tf_plain_sub(int dtype, int64_t n, const void *x, const void *y, void *z, hipStream_t stream) {
    return plain_binary(OP_SUB, dtype, n, x, y, z, stream);
}
int tf_plain_mul(int dtype, int64_t n, const void *x, const void *y, void *z, hipStream_t stream) {
    return plain_binary(OP_MUL, dtype, n, x, y, z, stream);
}
int tf_plain_div(int dtype, int64_t n, const void *x, const void *y, void *z, hipStream_t stream) {
    return plain_binary(OP_DIV, dtype, n, x, y, z, stream);
}
int tf_plain_sqrt(int dtype, int64_t n, const void *x, void *z, hipStream_t stream) {
    return plain_binary(OP_SQRT, dtype, n, x, nullptr, z, stream);
}
int tf_vmem(int dtype, int64_t n, const void *x, const void *y, void *z, hipStream_t stream) {
    return plain_binary(-1, dtype, n, x, y, z, stream);
}

int tf_plain_axpy(int dtype, int64_t n, const void *a, const void *x, const void *y, void *z,
                  hipStream_t stream) {
    TF_CHECK(size_of(dtype) && n >= 0 && a);
    if (n == 0) return TF_OK;
    TF_CHECK(x && y && z);
    const Launch L = make_launch(stream, {x, y, z});
    if (dtype == TF_F64) run_plain_axpy<double>(L, n, a, x, y, z);
    else run_plain_axpy<float>(L, n, a, x, y, z);
    return finish();
}

int tf_plain_horner(int dtype, int64_t n, int degree, const void *c, const void *x, void *z,
                    hipStream_t stream) {
    TF_CHECK(size_of(dtype) && n >= 0 && c && degree >= 0 && degree <= TF_MAX_DEGREE);
    if (n == 0) return TF_OK;
    TF_CHECK(x && z);
    const Launch L = make_launch(stream, {x, z});
    if (dtype == TF_F64) run_plain_horner<double>(L, n, degree, c, x, z);
    else run_plain_horner<float>(L, n, degree, c, x, z);
    return finish();
}

int tf_plain_sum(int dtype, int64_t n, const void *x, void *out, void *work, size_t work_bytes,
                 hipStream_t stream) {
    return reduce(LEAF_PSUM, dtype, n, x, nullptr, nullptr, nullptr, out, work, work_bytes, stream);
}

int tf_plain_dot(int dtype, int64_t n, const void *x, const void *y, void *out, void *work,
                 size_t work_bytes, hipStream_t stream) {
    if (n > 0) TF_CHECK(y);
    return reduce(LEAF_PDOT, dtype, n, x, nullptr, y, nullptr, out, work, work_bytes, stream);
}

// ---- coupled algorithms, renormalisation ----------------------------------------

static int unary(int op, int dtype, int64_t n, const void *x0, const void *x1, void *z0, void *z1,
                 hipStream_t stream) {
    TF_CHECK(size_of(dtype) && n >= 0);
    if (n == 0) return TF_OK;
    TF_CHECK(x0 && z0 && z1);
    const Launch L = make_launch(stream, {x0, x1, z0, z1});
    if (dtype == TF_F64) run_elementwise<double>(L, op, n, x0, x1, nullptr, nullptr, z0, z1);
    else run_elementwise<float>(L, op, n, x0, x1, nullptr, nullptr, z0, z1);
    return finish();
}

int tf_coupled(int dtype, int op, int renorm, int64_t n, const void *x0, const void *x1, const void *y0,
               const void *y1, void *z0, void *z1, hipStream_t stream) {
    TF_CHECK(op >= TF_OP_ADD && op <= TF_OP_SQRT);
    const int code = chain_code(op, renorm ? TF_MODE_DEKKER : TF_MODE_COUPLED);
    if (op == TF_OP_SQRT) return unary(code, dtype, n, x0, x1, z0, z1, stream);
    return binary(code, dtype, n, x0, x1, y0, y1, z0, z1, stream);
}

int tf_renorm(int dtype, int64_t n, const void *z0, const void *z1, void *s, void *t, hipStream_t stream) {
    if (n > 0) TF_CHECK(z1);
    return unary(OP_FAST_TWO_SUM, dtype, n, z0, z1, s, t, stream);
}

// ---- chains --------------------------------------------------------------------------

int tf_chain(int dtype, int op, int mode, int64_t n, int64_t reps, const void *x0, const void *x1,
             const void *y0, const void *y1, void *z0, void *z1, hipStream_t stream) {
    TF_CHECK(size_of(dtype) && n >= 0 && reps >= 0 && op >= TF_OP_ADD && op <= TF_OP_SQRT);
    TF_CHECK(mode == TF_MODE_TWOFOLD || mode == TF_MODE_COUPLED || mode == TF_MODE_DEKKER);
    if (n == 0) return TF_OK;
    TF_CHECK(x0 && z0 && z1 && (y0 || op == TF_OP_SQRT));
    const Launch L = make_launch(stream, {});
    const int code = chain_code(op, mode);
    if (dtype == TF_F64) run_chain<double>(L, code, n, reps, x0, x1, y0, y1, z0, z1);
    else run_chain<float>(L, code, n, reps, x0, x1, y0, y1, z0, z1);
    return finish();
}

int tf_plain_chain(int dtype, int op, int64_t n, int64_t reps, const void *x, const void *y, void *z,
                   hipStream_t stream) {
    TF_CHECK(size_of(dtype) && n >= 0 && reps >= 0 && op >= TF_OP_ADD && op <= TF_OP_SQRT);
    if (n == 0) return TF_OK;
    TF_CHECK(x && z && (y || op == TF_OP_SQRT));
    const Launch L = make_launch(stream, {});
    if (dtype == TF_F64) run_plain_chain<double>(L, op, n, reps, x, y, z);
    else run_plain_chain<float>(L, op, n, reps, x, y, z);
    return finish();
}

// ---- applications ----------------------------------------------------------------------

int tf_trsv_upper(int dtype, int64_t nsys, int m, const void *U0, const void *U1, const void *f0,
                  const void *f1, void *x0, void *x1, hipStream_t stream) {
    TF_CHECK(size_of(dtype) && nsys >= 0 && m >= 1 && m <= TF_MAX_TRSV);
    if (nsys == 0) return TF_OK;
    TF_CHECK(U0 && f0 && x0 && x1);
    const Launch L = make_launch(stream, {});
    if (dtype == TF_F64) run_trsv<double>(L, nsys, m, U0, U1, f0, f1, x0, x1);
    else run_trsv<float>(L, nsys, m, U0, U1, f0, f1, x0, x1);
    return finish();
}

int tf_plain_trsv_upper(int dtype, int64_t nsys, int m, const void *U, const void *f, void *x,
                        hipStream_t stream) {
    TF_CHECK(size_of(dtype) && nsys >= 0 && m >= 1 && m <= TF_MAX_TRSV);
    if (nsys == 0) return TF_OK;
    TF_CHECK(U && f && x);
    const Launch L = make_launch(stream, {});
    if (dtype == TF_F64) run_plain_trsv<double>(L, nsys, m, U, f, x);
    else run_plain_trsv<float>(L, nsys, m, U, f, x);
    return finish();
}

int tf_quadratic(int dtype, int64_t n, const void *a0, const void *a1, const void *b0, const void *b1,
                 const void *c0, const void *c1, void *r0, void *r1, void *s0, void *s1, hipStream_t stream) {
    TF_CHECK(size_of(dtype) && n >= 0);
    if (n == 0) return TF_OK;
    TF_CHECK(a0 && a1 && b0 && b1 && c0 && c1 && r0 && r1 && s0 && s1);
    const void *in[6] = {a0, a1, b0, b1, c0, c1};
    void *out[4] = {r0, r1, s0, s1};
    const Launch L = make_launch(stream, {a0, a1, b0, b1, c0, c1, r0, r1, s0, s1});
    if (dtype == TF_F64) run_quadratic<double>(L, n, in, out);
    else run_quadratic<float>(L, n, in, out);
    return finish();
}

int tf_plain_quadratic(int dtype, int64_t n, const void *a, const void *b, const void *c, void *r, void *s,
                       hipStream_t stream) {
    TF_CHECK(size_of(dtype) && n >= 0);
    if (n == 0) return TF_OK;
    TF_CHECK(a && b && c && r && s);
    const Launch L = make_launch(stream, {});
    if (dtype == TF_F64) run_plain_quadratic<double>(L, n, a, b, c, r, s);
    else run_plain_quadratic<float>(L, n, a, b, c, r, s);
    return finish();
}

// ---- fma -------------------------------------------------------------------------------

int tf_fma(int dtype, int64_t n, const void *x0, const void *x1, const void *y0, const void *y1,
           const void *w0, const void *w1, void *z0, void *z1, hipStream_t stream) {
    TF_CHECK(size_of(dtype) && n >= 0);
    if (n == 0) return TF_OK;
    TF_CHECK(x0 && y0 && w0 && z0 && z1);
    const void *in[6] = {x0, x1, y0, y1, w0, w1};
    const Launch L = make_launch(stream, {x0, x1, y0, y1, w0, w1, z0, z1});
    if (dtype == TF_F64) run_fma<double>(L, n, in, z0, z1);
    else run_fma<float>(L, n, in, z0, z1);
    return finish();
}

int tf_plain_fma(int dtype, int64_t n, const void *x, const void *y, const void *w, void *z,
                 hipStream_t stream) {
    TF_CHECK(size_of(dtype) && n >= 0);
    if (n == 0) return TF_OK;
    TF_CHECK(x && y && w && z);
    const Launch L = make_launch(stream, {});
    if (dtype == TF_F64) run_plain_fma<double>(L, n, x, y, w, z);
    else run_plain_fma<float>(L, n, x, y, w, z);
    return finish();
}

}  // extern "C\"
