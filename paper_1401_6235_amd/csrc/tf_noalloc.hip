// tf_dot_noalloc: the twofold dot product with its partials kept in a
// statically allocated device array instead of a caller workspace, for
// callers that cannot allocate device memory.
//
// The array lives in this translation unit's code object; every device the
// library runs on holds its own copy, at its own address, until the process
// ends.  In host code the array's name is only a stand-in for the symbol, so
// its device address is looked up once per device with hipGetSymbolAddress
// and that address, never the name, is what the kernels are given.
#include <mutex>

#include "tf_internal.hpp"

namespace {

static __device__ __align__(256) unsigned char scratch[TF_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;

// Device address of `scratch` on the current device (nullptr on failure).
void *scratch_address(hipError_t *err) {
    static std::mutex mu;
    static void *addr[kMaxDevices] = {};
    int dev = -1;
    *err = hipGetDevice(&dev);
    if (*err != hipSuccess) return nullptr;
    if (dev < 0 || dev >= kMaxDevices) {
        *err = hipErrorInvalidDevice;
        return nullptr;
    }
    std::lock_guard<std::mutex> lock(mu);
    if (addr[dev] == nullptr) {
        void *p = nullptr;
        *err = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (*err != hipSuccess) return nullptr;
        addr[dev] = p;
    }
    return addr[dev];
}

int size_of(int dtype) { return dtype == TF_F64 ? 8 : dtype == TF_F32 ? 4 : 0; }

}  // namespace

extern "C" int tf_dot_noalloc(int dtype, int64_t n, const void *x0, const void *x1, const void *y0,
                              const void *y1, void *out, hipStream_t stream) {
    using namespace tf;
    const int s = size_of(dtype);
    if (!s || n < 0 || out == nullptr) return TF_EINVAL;
    if (n > 0 && (x0 == nullptr || y0 == nullptr)) return TF_EINVAL;
    // every partial of every level is written before it is read, so the
    // array needs no clearing between calls
    const int leaf = x1 && y1 ? LEAF_DOT_TT : x1 ? LEAF_DOT_TD : y1 ? LEAF_DOT_DT : LEAF_DOT_DD;
    const int64_t cap = (int64_t)(TF_NOALLOC_SCRATCH_BYTES / (2 * (size_t)s));
    // more tiles per block when the partials would not fit: the tree does
    // not depend on it
    int64_t pb = tiles_per_block(s, leaf);
    while (reduce_work_pairs(n, pb) > cap && pb < kMaxTilesPerBlock) pb *= 2;
    if (reduce_work_pairs(n, pb) > cap) return TF_ENOMEM;
    hipError_t err = hipSuccess;
    void *work = scratch_address(&err);
    if (work == nullptr) return TF_EDEVICE;
    call_status() = hipSuccess;
    Launch L;
    L.stream = stream;
    L.aligned = true;
    for (const void *p : {x0, x1, y0, y1}) L.aligned = L.aligned && ((uintptr_t)p & 15u) == 0;
    L.cap = 0;
    if (dtype == TF_F64) run_reduce<double>(L, leaf, n, pb, x0, x1, y0, y1, out, work);
    else run_reduce<float>(L, leaf, n, pb, x0, x1, y0, y1, out, work);
    return call_status() == hipSuccess ? TF_OK : TF_EDEVICE;
}
