// Kernel launch with a status of its own.
//
// hipGetLastError() reports and clears the calling thread's sticky error,
// which any earlier HIP call of the application may have left there.  An
// entry point that ended with it would return that foreign error as its own
// and erase it for the code it belongs to.  Launches made here go through
// hipLaunchKernel, whose return value concerns that launch only; a failure
// is recorded in the thread's per-call status, which an entry point resets
// before its first launch and reads after its last.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <tuple>
#include <type_traits>
#include <utility>

namespace tf {

// Status of the launches made by the current entry point on this thread.
inline hipError_t &call_status() {
    static thread_local hipError_t s = hipSuccess;
    return s;
}

template <typename Kernel, typename Tuple, std::size_t... I>
inline hipError_t launch_tuple(Kernel kernel, dim3 grid, dim3 block, std::size_t shared, hipStream_t stream,
                               Tuple &vals, std::index_sequence<I...>) {
    void *ptrs[] = {(void *)&std::get<I>(vals)..., nullptr};
    const hipError_t e = hipLaunchKernel((const void *)kernel, grid, block, ptrs, shared, stream);
    if (e != hipSuccess) call_status() = e;
    return e;
}

// Launches `kernel` with `args` converted to its parameter types (in the
// order and with the meaning hipLaunchKernelGGL gives them).
template <typename... P, typename... A>
inline hipError_t tf_launch(void (*kernel)(P...), dim3 grid, dim3 block, std::size_t shared, hipStream_t stream,
                            A &&...args) {
    static_assert(sizeof...(P) == sizeof...(A), "kernel argument count");
    std::tuple<std::decay_t<P>...> vals(std::forward<A>(args)...);
    return launch_tuple(kernel, grid, block, shared, stream, vals, std::index_sequence_for<P...>{});
}

}  // namespace tf
