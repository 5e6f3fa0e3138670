// A C++ consumer of the C ABI: plain device pointers from hipMalloc, the
// functions declared in tf.h, no Python and no torch.  Test code: it also
// links the CPU oracle and checks every result bit for bit (NaN by class).
// Prints one line per check; exit status 0 when all pass.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <vector>

#include "tf.h"

extern "C" {  // the oracle's exports (tests only)
void orc_add_f64(int64_t, const double *, const double *, const double *, const double *, double *, double *);
void orc_div_f32(int64_t, const float *, const float *, const float *, const float *, float *, float *);
void orc_sum_f64(int64_t, const double *, const double *, double *);
void orc_dot_f32(int64_t, const float *, const float *, const float *, const float *, float *);
void orc_coupled_f64(int, int, int64_t, const double *, const double *, const double *, const double *,
                     double *, double *);
void orc_chain_f32(int, int, int64_t, int64_t, const float *, const float *, const float *, const float *,
                   float *, float *);
void orc_fma_f64(int64_t, const double *, const double *, const double *, const double *, const double *,
                 const double *, double *, double *);
}

static int failures = 0;

static void report(const char *what, bool ok) {
    std::printf("%-34s %s\n", what, ok ? "ok" : "MISMATCH");
    if (!ok) ++failures;
}

template <typename T>
static bool same_bits(const std::vector<T> &a, const std::vector<T> &b) {
    for (size_t i = 0; i < a.size(); ++i) {
        if (std::isnan(a[i]) && std::isnan(b[i])) continue;
        if (std::memcmp(&a[i], &b[i], sizeof(T)) != 0) return false;
    }
    return true;
}

// Inputs: a splitmix64 stream mapped to values of both signs over a few
// binades, low parts about one unit in the last place of the high parts.
static uint64_t mix(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}
template <typename T>
static std::vector<T> draw(size_t n, uint64_t seed, double scale, bool positive = false) {
    std::vector<T> v(n);
    for (size_t i = 0; i < n; ++i) {
        const uint64_t r = mix(seed + (i + 1) * 0x9E3779B97F4A7C15ull);
        const double u = (double)(r >> 11) * 0x1.0p-53;                 // [0, 1)
        const double s = positive || (r & 1) == 0 ? 1.0 : -1.0;
        v[i] = (T)(s * (0.5 + u) * std::ldexp(scale, (int)((r >> 1) % 9) - 4));
    }
    return v;
}

template <typename T>
static T *dev(const std::vector<T> &h) {
    T *p = nullptr;
    if (hipMalloc(&p, h.size() * sizeof(T) + 16) != hipSuccess) { std::puts("hipMalloc failed"); std::exit(2); }
    if (hipMemcpy(p, h.data(), h.size() * sizeof(T), hipMemcpyHostToDevice) != hipSuccess) std::exit(2);
    return p;
}
template <typename T>
static std::vector<T> host(const T *p, size_t n) {
    std::vector<T> h(n);
    if (hipDeviceSynchronize() != hipSuccess) { std::puts("kernel failed"); std::exit(2); }
    if (hipMemcpy(h.data(), p, n * sizeof(T), hipMemcpyDeviceToHost) != hipSuccess) std::exit(2);
    return h;
}

int main() {
    const int64_t n = 100003;
    std::printf("tf_version %d\n", tf_version());

    {  // binary64 add, twofold operands
        auto x0 = draw<double>(n, 1, 1.0), y0 = draw<double>(n, 2, 1.0);
        auto x1 = draw<double>(n, 3, 0x1.0p-53), y1 = draw<double>(n, 4, 0x1.0p-53);
        double *d[6] = {dev(x0), dev(x1), dev(y0), dev(y1), dev(x0), dev(x0)};
        const int st = tf_add(TF_F64, n, d[0], d[1], d[2], d[3], d[4], d[5], nullptr);
        std::vector<double> z0(n), z1(n);
        orc_add_f64(n, x0.data(), x1.data(), y0.data(), y1.data(), z0.data(), z1.data());
        report("tf_add f64", st == TF_OK && same_bits(host(d[4], n), z0) && same_bits(host(d[5], n), z1));

        // twofold sum of (x0, x1) with a caller workspace
        const size_t wb = tf_reduce_workspace_bytes(TF_F64, n);
        void *work = nullptr;
        double *out = nullptr;
        (void)hipMalloc(&work, wb);
        (void)hipMalloc(&out, 2 * sizeof(double));
        const int st2 = tf_sum(TF_F64, n, d[0], d[1], out, work, wb, nullptr);
        std::vector<double> s(2);
        orc_sum_f64(n, x0.data(), x1.data(), s.data());
        report("tf_sum f64", st2 == TF_OK && same_bits(host(out, 2), s));
        report("tf_sum with a short workspace", tf_sum(TF_F64, n, d[0], d[1], out, work, wb / 2, nullptr) == TF_ENOMEM);

        // Dekker-mode multiply
        const int st3 = tf_coupled(TF_F64, TF_OP_MUL, 1, n, d[0], d[1], d[2], d[3], d[4], d[5], nullptr);
        orc_coupled_f64(2, 1, n, x0.data(), x1.data(), y0.data(), y1.data(), z0.data(), z1.data());
        report("tf_coupled mul renorm f64", st3 == TF_OK && same_bits(host(d[4], n), z0) && same_bits(host(d[5], n), z1));

        // fma with a dotted addend
        const int st4 = tf_fma(TF_F64, n, d[0], d[1], d[2], d[3], d[2], nullptr, d[4], d[5], nullptr);
        orc_fma_f64(n, x0.data(), x1.data(), y0.data(), y1.data(), y0.data(), nullptr, z0.data(), z1.data());
        report("tf_fma f64", st4 == TF_OK && same_bits(host(d[4], n), z0) && same_bits(host(d[5], n), z1));
        for (double *p : d) (void)hipFree(p);
        (void)hipFree(work);
        (void)hipFree(out);
    }
    {  // binary32 divide with a dotted divisor, dot of plain vectors, Dekker chain
        auto x0 = draw<float>(n, 5, 1.0), y0 = draw<float>(n, 6, 1.0);
        auto x1 = draw<float>(n, 7, 0x1.0p-24);
        float *d[5] = {dev(x0), dev(x1), dev(y0), dev(x0), dev(x0)};
        const int st = tf_div(TF_F32, n, d[0], d[1], d[2], nullptr, d[3], d[4], nullptr);
        std::vector<float> z0(n), z1(n);
        orc_div_f32(n, x0.data(), x1.data(), y0.data(), nullptr, z0.data(), z1.data());
        report("tf_div f32, dotted divisor", st == TF_OK && same_bits(host(d[3], n), z0) && same_bits(host(d[4], n), z1));

        const size_t wb = tf_reduce_workspace_bytes(TF_F32, n);
        void *work = nullptr;
        float *out = nullptr;
        (void)hipMalloc(&work, wb);
        (void)hipMalloc(&out, 2 * sizeof(float));
        const int st2 = tf_dot(TF_F32, n, d[0], nullptr, d[2], nullptr, out, work, wb, nullptr);
        std::vector<float> s(2);
        orc_dot_f32(n, x0.data(), nullptr, y0.data(), nullptr, s.data());
        report("tf_dot f32", st2 == TF_OK && same_bits(host(out, 2), s));

        auto m = draw<float>(n, 8, 1.0, true);
        for (auto &v : m) v = 1.0f + (v - 1.0f) * 0x1.0p-12f;  // operands near 1: long chains stay in range
        float *dm = dev(m);
        const int st3 = tf_chain(TF_F32, TF_OP_MUL, TF_MODE_DEKKER, n, 300, d[0], d[1], dm, nullptr, d[3], d[4], nullptr);
        orc_chain_f32(2, 2, n, 300, x0.data(), x1.data(), m.data(), nullptr, z0.data(), z1.data());
        report("tf_chain mul dekker f32", st3 == TF_OK && same_bits(host(d[3], n), z0) && same_bits(host(d[4], n), z1));
        for (float *p : d) (void)hipFree(p);
        (void)hipFree(dm);
        (void)hipFree(work);
        (void)hipFree(out);
    }
    // An error that other code left in the thread's HIP state is neither
    // returned by a tf_* call as its own nor cleared by it.
    {
        const int64_t m = 1000;
        std::vector<double> a = draw<double>(m, 31, 1.0), b = draw<double>(m, 32, 1.0);
        double *da = dev(a), *db = dev(b), *o0 = dev(a), *o1 = dev(a);
        (void)hipGetLastError();
        int ndev = 0;
        const hipError_t planted = hipSetDevice(-1);  // invalid ordinal: fails, sets nothing
        (void)hipGetDeviceCount(&ndev);                // a successful call in between
        const bool sticky = planted != hipSuccess && hipPeekAtLastError() == planted;
        const int st = tf_add(TF_F64, m, da, nullptr, db, nullptr, o0, o1, nullptr);
        report("foreign pending error not returned", st == TF_OK);
        if (sticky) report("foreign pending error not cleared", hipPeekAtLastError() == planted);
        else std::printf("%-34s %s\n", "foreign pending error not cleared", "skipped (runtime keeps no sticky error)");
        (void)hipGetLastError();
        std::vector<double> z0(m), z1(m);
        orc_add_f64(m, a.data(), nullptr, b.data(), nullptr, z0.data(), z1.data());
        report("tf_add after a foreign error", same_bits(host(o0, m), z0) && same_bits(host(o1, m), z1));
        for (double *p : {da, db, o0, o1}) (void)hipFree(p);
    }
    // misuse is reported, not run
    report("invalid dtype", tf_add(7, 10, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr) == TF_EINVAL);
    report("NULL output", tf_sqrt(TF_F64, 10, (void *)16, nullptr, nullptr, nullptr, nullptr) == TF_EINVAL);
    report("n = 0 is a no-op", tf_mul(TF_F32, 0, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr) == TF_OK);
    report("tf_strerror", std::strcmp(tf_strerror(TF_EINVAL), "invalid argument") == 0);
    std::printf("%s\n", failures ? "FAILED" : "all passed");
    return failures ? 1 : 0;
}
