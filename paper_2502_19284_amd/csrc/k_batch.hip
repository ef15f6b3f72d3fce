// k_batch.hip -- one launch for the products of many matrices (gfx950).
//
// The product launch has G workgroups; workgroup b processes work items b, b + G, ... of the
// batch's item list, where an item is one tile of one matrix.  Merge tiles follow the merge-path
// product of Section 3.3 with the matrix's own tile length (256 * ipt items): the tile stages its
// row ends and products in LDS, every thread walks ipt items, a segmented scan passes open
// values between threads, and the value the tile leaves open goes to carry[t].  Row tiles hand
// whole rows to lane groups sized to the tile's average row length.  A second, small launch adds
// every merge matrix's carries into y in tile order (a device-wide handshake inside the product
// launch would need a release/acquire pair per tile, which costs more than the launch).
//
// Values are FP32 or bfloat16, x and y FP32; sums inside a tile are FP32, carries FP64.
#include "dev_common.h"
#include "dev_merge.h"
#include "dev_values.h"
#include "spx_internal.h"

#define BT_NT 256

__device__ __forceinline__ float bt_val(const BatchMat& M, int64_t k) {
    return M.bf16 ? __uint_as_float((uint32_t)ntload((const uint16_t*)M.val + k) << 16)
                  : ntload((const float*)M.val + k);
}

__device__ __forceinline__ float bt_x(const float* __restrict__ x,
                                      const int32_t* __restrict__ hot, int32_t c) {
    return c >= 0 ? x[c] : x[hot[~c]];
}

template <int IPT>
__device__ void bt_merge(const BatchMat& M, int t, const float* __restrict__ x,
                         float* __restrict__ y, int32_t* s_end, float* s_prod, int* s_wf,
                         float* s_wv) {
    const int tid = threadIdx.x;
    const int2 c0 = M.coords[t];
    const int2 c1 = M.coords[t + 1];
    const int r0 = c0.x, k0 = c0.y;
    const int nrows = c1.x - r0, nnzt = c1.y - k0;
    for (int i = tid; i < nrows; i += BT_NT) s_end[i] = ntload(M.row_ptr + r0 + 1 + i);
#pragma unroll
    for (int q = 0; q < IPT; ++q) {
        const int i = q * BT_NT + tid;
        if (i < nnzt) s_prod[i] = bt_val(M, (int64_t)k0 + i) * bt_x(x, M.hot_cols, ntload(M.col + k0 + i));
    }
    __syncthreads();

    const float open = merge_tile_sums<BT_NT, IPT, float>(s_end, s_prod, nrows, nnzt, k0, s_wf,
                                                          s_wv);
    if (tid == BT_NT - 1) {
        M.carry_row[t] = c1.x;  // m when nothing is left open
        M.carry_val[t] = (double)open;
    }
    for (int q = tid; q < nrows; q += BT_NT) y[r0 + q] = s_prod[q];
}

__device__ void bt_rows(const BatchMat& M, int t, const float* __restrict__ x,
                        float* __restrict__ y) {
    const int r0 = t * M.rows_per_tile;
    const int r1 = min(M.m, r0 + M.rows_per_tile);
    const int rows = r1 - r0;
    const int base = M.row_ptr[r0];
    const int nz = M.row_ptr[r1] - base;
    const int avg = rows > 0 ? (nz + rows - 1) / rows : 0;
    int g = 1;
    while (g < SPX_WAVE && g < avg) g <<= 1;
    const int tid = threadIdx.x;
    const int grp = tid / g, gl = tid % g, ngrp = BT_NT / g;
    for (int r = grp; r < rows; r += ngrp) {
        const int a = M.row_ptr[r0 + r], b = M.row_ptr[r0 + r + 1];
        float acc = 0;
        for (int k = a + gl; k < b; k += g) acc += bt_val(M, k) * bt_x(x, M.hot_cols, ntload(M.col + k));
        for (int o = g >> 1; o > 0; o >>= 1) acc += __shfl_xor(acc, o, SPX_WAVE);
        if (gl == 0) y[r0 + r] = acc;
    }
}

__global__ __launch_bounds__(BT_NT) void k_batch_spmv(const BatchMat* __restrict__ mats,
                                                      const int2* __restrict__ items,
                                                      int32_t nitems, int32_t max_tile,
                                                      const float* const* __restrict__ xs,
                                                      float* const* __restrict__ ys) {
    extern __shared__ int32_t s_dyn[];  // max_tile row ends, then max_tile products
    __shared__ int s_wf[BT_NT / SPX_WAVE];
    __shared__ float s_wv[BT_NT / SPX_WAVE];
    int32_t* s_end = s_dyn;
    float* s_prod = (float*)(s_dyn + max_tile);
    for (int it = blockIdx.x; it < nitems; it += gridDim.x) {
        const int2 w = items[it];
        const BatchMat M = mats[w.x];
        const float* x = xs[w.x];
        float* y = ys[w.x];
        if (M.plan == SPX_PLAN_MERGE_4) bt_merge<4>(M, w.y, x, y, s_end, s_prod, s_wf, s_wv);
        else if (M.plan == SPX_PLAN_MERGE_8) bt_merge<8>(M, w.y, x, y, s_end, s_prod, s_wf, s_wv);
        else if (M.plan == SPX_PLAN_MERGE_16) bt_merge<16>(M, w.y, x, y, s_end, s_prod, s_wf, s_wv);
        else bt_rows(M, w.y, x, y);
        __syncthreads();
    }
}

// One thread per work item: the first merge tile of every run of tiles that left the same row
// open adds the run's carries (carry_run_sum: fixed order) into y.
__global__ void k_batch_fixup(const BatchMat* __restrict__ mats, const int2* __restrict__ items,
                              int32_t nitems, float* const* __restrict__ ys) {
    const int it = blockIdx.x * blockDim.x + threadIdx.x;
    if (it >= nitems) return;
    const int2 w = items[it];
    const BatchMat& M = mats[w.x];
    if (M.plan > SPX_PLAN_MERGE_16) return;
    const int t = w.y;
    const int r = M.carry_row[t];
    if (r >= M.m) return;
    if (t > 0 && M.carry_row[t - 1] == r) return;
    const double acc =
        carry_run_sum(M.carry_row, M.tiles, t, r, [&](int u) { return M.carry_val[u]; });
    float* y = ys[w.x];
    y[r] = (float)(acc + (double)y[r]);
}

hipError_t launch_batch_spmv(const BatchMat* mats, const int2* items, int32_t nitems,
                             int32_t grid, int32_t max_tile, const float* const* xs,
                             float* const* ys, hipStream_t s) {
    if (nitems <= 0) return hipSuccess;
    const size_t lds = (size_t)max_tile * 8;
    SPX_LAUNCH("batch_spmv", k_batch_spmv, dim3(grid), dim3(BT_NT), lds, s, mats, items, nitems,
               max_tile, xs, ys);
    SPX_LAUNCH("batch_fixup", k_batch_fixup, dim3(spx_div_up(nitems, 256)), dim3(256), 0, s, mats,
               items, nitems, ys);
    return hipGetLastError();
}

// longest row: *out = max over rows of row_ptr[i+1] - row_ptr[i] (out starts at 0)
__global__ void k_batch_maxlen(const int32_t* __restrict__ row_ptr, int32_t m,
                               uint32_t* __restrict__ out) {
    uint32_t best = 0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < m;
         i += (int64_t)gridDim.x * blockDim.x)
        best = max(best, (uint32_t)(row_ptr[i + 1] - row_ptr[i]));
    best = wave_reduce<uint32_t, OpMax<uint32_t>>(best);
    if (__lane_id() == 0) atomicMax(out, best);
}

hipError_t launch_batch_maxlen(const int32_t* row_ptr, int32_t m, uint32_t* out, hipStream_t s) {
    if (m <= 0) return hipSuccess;
    int64_t g = spx_div_up(m, 256);
    if (g > 1024) g = 1024;
    SPX_LAUNCH("batch_maxlen", k_batch_maxlen, dim3((unsigned)g), dim3(256), 0, s, row_ptr, m,
               out);
    return hipGetLastError();
}

__global__ void k_fill_u32(uint32_t* __restrict__ p, int64_t n, uint32_t v) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

hipError_t launch_fill_u32(uint32_t* p, int64_t n, uint32_t v, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    int64_t g = spx_div_up(n, 256);
    if (g > 4096) g = 4096;
    SPX_LAUNCH("fill_u32", k_fill_u32, dim3((unsigned)g), dim3(256), 0, s, p, n, v);
    return hipGetLastError();
}
