// dev_common.h -- wave64 / workgroup helpers shared by the HIP kernels of libspx (gfx950).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#define SPX_WAVE 64

__device__ __forceinline__ uint64_t spx_lanemask_lt() {
    const unsigned lane = __lane_id();
    return lane == 0 ? 0ull : (~0ull >> (64 - lane));
}

// Inclusive prefix within a wave (Hillis-Steele over 6 rounds of lane shifts).
template <typename T, typename Op>
__device__ __forceinline__ T wave_incl_scan(T v) {
    const int lane = __lane_id();
#pragma unroll
    for (int o = 1; o < SPX_WAVE; o <<= 1) {
        T t = __shfl_up(v, o, SPX_WAVE);
        if (lane >= o) v = Op::op(t, v);
    }
    return v;
}

template <typename T, typename Op>
__device__ __forceinline__ T wave_reduce(T v) {
#pragma unroll
    for (int o = SPX_WAVE / 2; o > 0; o >>= 1) v = Op::op(v, __shfl_xor(v, o, SPX_WAVE));
    return v;
}

template <typename T>
struct OpSum {
    __device__ __forceinline__ static T id() { return T(0); }
    __device__ __forceinline__ static T op(T a, T b) { return a + b; }
};

template <typename T>
struct OpOr {
    __device__ __forceinline__ static T id() { return T(0); }
    __device__ __forceinline__ static T op(T a, T b) { return a | b; }
};

template <typename T>
struct OpAnd {
    __device__ __forceinline__ static T id() { return ~T(0); }
    __device__ __forceinline__ static T op(T a, T b) { return a & b; }
};

// Max for non-negative operands (identity 0).
template <typename T>
struct OpMax {
    __device__ __forceinline__ static T id() { return T(0); }
    __device__ __forceinline__ static T op(T a, T b) { return a > b ? a : b; }
};

// Exclusive scan of one value per thread over a workgroup of NT threads.  `s_tmp` holds NT/64
// elements of LDS.  Returns the exclusive prefix; *total receives the workgroup total.
// Contains two barriers; every thread of the workgroup must call it.
template <int NT, typename T, typename Op>
__device__ __forceinline__ T block_excl_scan(T v, T* s_tmp, T* total) {
    constexpr int NW = NT / SPX_WAVE;
    const int w = threadIdx.x / SPX_WAVE;
    const int lane = __lane_id();
    T inc = wave_incl_scan<T, Op>(v);
    if (lane == SPX_WAVE - 1) s_tmp[w] = inc;
    __syncthreads();
    T pre = Op::id(), tot = Op::id();
#pragma unroll
    for (int i = 0; i < NW; ++i) {
        T t = s_tmp[i];
        if (i < w) pre = Op::op(pre, t);
        tot = Op::op(tot, t);
    }
    __syncthreads();
    *total = tot;
    // exclusive within the wave: the inclusive value of the previous lane
    T ex = __shfl_up(inc, 1, SPX_WAVE);
    if (lane == 0) ex = Op::id();
    return Op::op(pre, ex);
}

template <int NT, typename T, typename Op>
__device__ __forceinline__ T block_reduce(T v, T* s_tmp) {
    constexpr int NW = NT / SPX_WAVE;
    v = wave_reduce<T, Op>(v);
    if (__lane_id() == 0) s_tmp[threadIdx.x / SPX_WAVE] = v;
    __syncthreads();
    T tot = Op::id();
#pragma unroll
    for (int i = 0; i < NW; ++i) tot = Op::op(tot, s_tmp[i]);
    __syncthreads();
    return tot;
}

// s[r] += v for every lane with r >= 0, by LDS float atomics.  When neighbouring lanes of the wave
// hold the same r (runs of one row in storage order), each run is first summed by a segmented
// scan across its lanes and only its last lane adds: atomics on one address are serialised, and
// a run of 64 would cost 64 times one.  Every lane of the wave must call it (wave-uniform path).
__device__ __forceinline__ void lds_add_runs(double* s, int r, double v) {
    const int lane = __lane_id();
    const int rp = __shfl_up(r, 1, SPX_WAVE);
    const uint64_t heads = __ballot(lane == 0 || rp != r);
    if (heads == ~0ull) {  // no two neighbours share a row
        if (r >= 0) atomicAdd(&s[r], v);
        return;
    }
    // first lane of this lane's run: the highest head at or below it ((2 << 63) - 1 = all lanes)
    const int start = 63 - __clzll(heads & ((2ull << lane) - 1ull));
#pragma unroll
    for (int o = 1; o < SPX_WAVE; o <<= 1) {
        const double t = __shfl_up(v, o, SPX_WAVE);
        if (lane - o >= start) v += t;
    }
    const bool last = lane == SPX_WAVE - 1 || ((heads >> (lane + 1)) & 1ull);
    if (last && r >= 0) atomicAdd(&s[r], v);
}

static inline unsigned spx_div_up(int64_t a, int64_t b) { return (unsigned)((a + b - 1) / b); }
