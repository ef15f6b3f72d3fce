// dev_scan.h -- three-phase device scan (reduce, scan of tile sums, apply) over n <= 2^31 items.
//
// The items are produced by a load functor `ld(i)` and consumed by a store functor
// `st(i, inclusive_prefix, item)`, so a scan can read flags computed on the fly and scatter its
// results without a materialised input or output array.
//   phase 1  scan_tile_reduce : one total per tile of SCAN_TILE items
//   phase 2  scan_tile_sums   : one workgroup scans the tile totals (exclusive, in place) and
//                               writes the grand total to device memory
//   phase 3  scan_tile_apply  : each tile scans its items and calls st() with global prefixes
// Between phase 2 and 3 the caller may read the total back to size the output.
#pragma once
#include "dev_common.h"
#include "spx_prof.h"

#define SCAN_NT 256
#define SCAN_IPT 16
#define SCAN_TILE (SCAN_NT * SCAN_IPT)

// skewed LDS index: item i of a tile lives at i + i/16 so that thread t's 16 consecutive items
// fall in distinct banks
__device__ __forceinline__ int scan_skew(int i) { return i + (i >> 4); }

template <typename T, typename Op, typename Load>
__global__ __launch_bounds__(SCAN_NT) void scan_tile_reduce(Load ld, int64_t n, T* tile_sums) {
    __shared__ T s_tmp[SCAN_NT / SPX_WAVE];
    const int64_t base = (int64_t)blockIdx.x * SCAN_TILE;
    T acc = Op::id();
#pragma unroll
    for (int i = 0; i < SCAN_IPT; ++i) {
        int64_t idx = base + i * SCAN_NT + threadIdx.x;
        if (idx < n) acc = Op::op(acc, ld(idx));
    }
    T tot = block_reduce<SCAN_NT, T, Op>(acc, s_tmp);
    if (threadIdx.x == 0) tile_sums[blockIdx.x] = tot;
}

// Single workgroup: exclusive scan of tile_sums[0..nt) in place; *total = sum of all.
template <typename T, typename Op>
__global__ __launch_bounds__(SCAN_NT) void scan_tile_sums(T* tile_sums, int64_t nt, T* total) {
    __shared__ T s_data[SCAN_TILE + SCAN_TILE / 16];
    __shared__ T s_tmp[SCAN_NT / SPX_WAVE];
    T carry = Op::id();
    for (int64_t base = 0; base < nt; base += SCAN_TILE) {
#pragma unroll
        for (int i = 0; i < SCAN_IPT; ++i) {
            int li = i * SCAN_NT + threadIdx.x;
            int64_t idx = base + li;
            s_data[scan_skew(li)] = idx < nt ? tile_sums[idx] : Op::id();
        }
        __syncthreads();
        T v[SCAN_IPT];
        T run = Op::id();
#pragma unroll
        for (int j = 0; j < SCAN_IPT; ++j) {
            v[j] = run;  // exclusive
            run = Op::op(run, s_data[scan_skew(threadIdx.x * SCAN_IPT + j)]);
        }
        T chunk_total;
        T pre = block_excl_scan<SCAN_NT, T, Op>(run, s_tmp, &chunk_total);
        pre = Op::op(carry, pre);
#pragma unroll
        for (int j = 0; j < SCAN_IPT; ++j)
            s_data[scan_skew(threadIdx.x * SCAN_IPT + j)] = Op::op(pre, v[j]);
        __syncthreads();
#pragma unroll
        for (int i = 0; i < SCAN_IPT; ++i) {
            int li = i * SCAN_NT + threadIdx.x;
            int64_t idx = base + li;
            if (idx < nt) tile_sums[idx] = s_data[scan_skew(li)];
        }
        carry = Op::op(carry, chunk_total);
        __syncthreads();
    }
    if (threadIdx.x == 0 && total) *total = carry;
}

// Each tile: local scan of its items plus the tile's exclusive offset; st(i, incl, item) for every
// item i < n, where incl is the inclusive prefix (exclusive prefix = incl minus item for sums).
template <typename T, typename Op, typename Load, typename Store>
__global__ __launch_bounds__(SCAN_NT) void scan_tile_apply(Load ld, Store st, int64_t n,
                                                           const T* tile_offsets) {
    __shared__ T s_data[SCAN_TILE + SCAN_TILE / 16];
    __shared__ T s_tmp[SCAN_NT / SPX_WAVE];
    const int64_t base = (int64_t)blockIdx.x * SCAN_TILE;
#pragma unroll
    for (int i = 0; i < SCAN_IPT; ++i) {
        int li = i * SCAN_NT + threadIdx.x;
        int64_t idx = base + li;
        s_data[scan_skew(li)] = idx < n ? ld(idx) : Op::id();
    }
    __syncthreads();
    T item[SCAN_IPT];
    T run = Op::id();
#pragma unroll
    for (int j = 0; j < SCAN_IPT; ++j) {
        item[j] = s_data[scan_skew(threadIdx.x * SCAN_IPT + j)];
        run = Op::op(run, item[j]);
    }
    T tile_total;
    T pre = block_excl_scan<SCAN_NT, T, Op>(run, s_tmp, &tile_total);
    pre = Op::op(tile_offsets[blockIdx.x], pre);
    const int64_t first = base + (int64_t)threadIdx.x * SCAN_IPT;
#pragma unroll
    for (int j = 0; j < SCAN_IPT; ++j) {
        pre = Op::op(pre, item[j]);
        if (first + j < n) st(first + j, pre, item[j]);
    }
}

// Host-side driver.  tile_sums must hold spx_div_up(n, SCAN_TILE) elements; total one element.
template <typename T, typename Op, typename Load>
static inline hipError_t scan_phase12(Load ld, int64_t n, T* tile_sums, T* total,
                                      hipStream_t s) {
    if (n <= 0) return hipSuccess;
    const unsigned nt = spx_div_up(n, SCAN_TILE);
    SPX_LAUNCH("scan_tile_reduce", (scan_tile_reduce<T, Op, Load>), dim3(nt), dim3(SCAN_NT), 0, s, ld, n,
                       tile_sums);
    SPX_LAUNCH("scan_tile_sums", (scan_tile_sums<T, Op>), dim3(1), dim3(SCAN_NT), 0, s, tile_sums,
                       (int64_t)nt, total);
    return hipGetLastError();
}

template <typename T, typename Op, typename Load, typename Store>
static inline hipError_t scan_phase3(Load ld, Store st, int64_t n, const T* tile_sums,
                                     hipStream_t s) {
    if (n <= 0) return hipSuccess;
    const unsigned nt = spx_div_up(n, SCAN_TILE);
    SPX_LAUNCH("scan_tile_apply", (scan_tile_apply<T, Op, Load, Store>), dim3(nt), dim3(SCAN_NT), 0, s, ld,
                       st, n, tile_sums);
    return hipGetLastError();
}
