// Kernel launch helper shared by the pipelines.  Every kernel of the library
// goes through launch(): it converts the arguments to the kernel's parameter
// types and, while kernel timing is enabled, brackets the dispatch with HIP
// events taken by the launch itself (hipExtLaunchKernel), on the launch's own
// stream, so per-kernel durations can be read back (mesh_timing_read).
// Launches into a stream that is being captured into a graph run untimed.
#pragma once

#include <hip/hip_ext.h>
#include <hip/hip_runtime.h>

#include <tuple>
#include <utility>

namespace mnb {

// True when launches of kernel `name` are being timed (timing on, and the
// name selected, or no selection).
bool timing_enabled(const char* name);
// While an UntimedScope lives on the calling thread, its launches run untimed
// (no event is created or taken from the pool).
struct UntimedScope {
    UntimedScope();
    ~UntimedScope();
    UntimedScope(const UntimedScope&) = delete;
    UntimedScope& operator=(const UntimedScope&) = delete;
};
// Hands out an event pair for one timed launch; false when timing is off or
// the record is full (the launch then runs untimed).
bool timing_begin(hipEvent_t* start, hipEvent_t* stop);
// Records that the pair brackets one launch of kernel `name`.
void timing_commit(const char* name, hipEvent_t start, hipEvent_t stop);

// As launch(), with `shm` bytes of dynamic LDS.
template <typename... P, typename... A>
hipError_t launch_shm(const char* name, void (*kernel)(P...), dim3 grid, dim3 block, size_t shm, hipStream_t stream,
                      A&&... a);

template <typename... P, typename... A>
hipError_t launch(const char* name, void (*kernel)(P...), dim3 grid, dim3 block, hipStream_t stream, A&&... a) {
    return launch_shm(name, kernel, grid, block, 0, stream, std::forward<A>(a)...);
}

template <typename... P, typename... A>
hipError_t launch_shm(const char* name, void (*kernel)(P...), dim3 grid, dim3 block, size_t shm, hipStream_t stream,
                      A&&... a) {
    static_assert(sizeof...(P) == sizeof...(A), "argument count");
    std::tuple<P...> vals(static_cast<P>(std::forward<A>(a))...);
    void* args[sizeof...(P) > 0 ? sizeof...(P) : 1];
    std::apply(
        [&](auto&... x) {
            int i = 0;
            ((args[i++] = (void*)&x), ...);
        },
        vals);
    if (grid.x == 0 || grid.y == 0 || grid.z == 0) return hipSuccess;
    hipEvent_t e0, e1;
    hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
    // launches recorded into a graph run untimed
    if (timing_enabled(name) && hipStreamIsCapturing(stream, &cap) == hipSuccess && cap == hipStreamCaptureStatusNone &&
        timing_begin(&e0, &e1)) {
        hipError_t e = hipExtLaunchKernel((const void*)kernel, grid, block, args, shm, stream, e0, e1, 0);
        if (e == hipSuccess) timing_commit(name, e0, e1);
        return e;
    }
    return hipLaunchKernel((const void*)kernel, grid, block, args, shm, stream);
}

}  // namespace mnb
