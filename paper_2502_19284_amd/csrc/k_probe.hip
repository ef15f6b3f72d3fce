// k_probe.hip -- memory-system probe (a measurement aid, not part of any product).
//
// n random 8-byte loads from the first `window` doubles of x: thread i of the grid-stride loop
// loads x[h(i) mod window], h a 64-bit mixing function, and the loaded values are summed per
// thread into out (so the loads cannot be dropped).  With a window far larger than the L2, every
// load misses and fills one 128-byte line: the kernel measures the random line-fill rate that
// bounds the x gathers of the products; with a window inside the L2 it measures the L2 request
// rate.
#include "dev_common.h"
#include "spx_internal.h"

#define PROBE_GRID 8192
#define PROBE_NT 256

__device__ __forceinline__ uint64_t probe_mix(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

__global__ __launch_bounds__(PROBE_NT) void k_probe_gather(const double* __restrict__ x,
                                                           uint64_t mask, int64_t n,
                                                           double* __restrict__ out) {
    double a = 0.0;
    const int64_t t = (int64_t)blockIdx.x * PROBE_NT + threadIdx.x;
    for (int64_t i = t; i < n; i += (int64_t)PROBE_GRID * PROBE_NT) a += x[probe_mix(i) & mask];
    out[t] = a;
}

int64_t probe_out_len() { return (int64_t)PROBE_GRID * PROBE_NT; }

hipError_t launch_probe_gather(const double* x, int64_t window, int64_t n, double* out,
                               hipStream_t s) {
    SPX_LAUNCH("probe_gather", k_probe_gather, dim3(PROBE_GRID), dim3(PROBE_NT), 0, s, x,
               (uint64_t)window - 1u, n, out);
    return hipGetLastError();
}
