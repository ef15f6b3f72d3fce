// spx_prof.h -- optional per-kernel timing with HIP events on the launch stream.
#pragma once
#include <hip/hip_runtime.h>

// True while spx_profile_enable(1) is in effect.
bool spx_prof_on();
// Records a start event on `s` (returns nullptr when profiling is off or an event is unavailable).
hipEvent_t spx_prof_begin(hipStream_t s);
// Records the stop event and files (name, start, stop) for spx_profile_collect.
void spx_prof_end(const char* name, hipStream_t s, hipEvent_t start);

// Launch `kernel` like hipLaunchKernelGGL, bracketed by events when profiling is on.
#define SPX_LAUNCH(name, kernel, grid, block, lds, stream, ...)                      \
    do {                                                                             \
        hipEvent_t spx_e0_ = spx_prof_on() ? spx_prof_begin(stream) : nullptr;       \
        hipLaunchKernelGGL(kernel, grid, block, lds, stream, __VA_ARGS__);           \
        if (spx_e0_) spx_prof_end(name, stream, spx_e0_);                            \
    } while (0)
