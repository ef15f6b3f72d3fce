// dev_merge.h -- the merge-path tile of Section 3.3 (Algorithm 1), shared by the CRS product
// (k_spmv_crs.hip), the batched product (k_batch.hip) and the multi-vector product (k_spmm.hip).
//
// A tile covers a range of diagonals of the merge of the row ends row_ptr[1..m] with the entry
// indices 0..nnz-1.  Its nrows row ends (absolute entry indices, s_end) and nnzt entries, the
// first of which is entry k0, are staged in LDS.  The merge takes row end i before entry j when
// s_end[i] <= k0 + j: a row end is consumed as soon as all of its row's entries are.
#pragma once
#include "dev_common.h"

// segmented-sum combine: (flag, value) of an earlier then a later segment
template <typename T>
__device__ __forceinline__ void seg_combine(int& f, T& v, int f_later, T v_later) {
    v = f_later ? v_later : v + v_later;
    f = f | f_later;
}

// Split point of diagonal d of the tile: the number of row ends among its first d items.
__device__ __forceinline__ int merge_split(const int32_t* s_end, int nrows, int nnzt, int k0,
                                           int d) {
    int lo = max(0, d - nnzt), hi = min(d, nrows);
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (s_end[mid] <= k0 + d - mid - 1) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

// Row sums of a staged tile, NT threads of IPT consecutive items each.  On entry s_prod[j] holds
// the product of the tile's entry j.  Each thread walks its items from its own split point (an
// entry adds its product to the running value, a row end emits it); the value a thread leaves
// open reaches later threads through a segmented scan (shuffles inside a wave, s_wf / s_wv of
// NT / 64 elements across waves).  On return s_prod[i] holds the tile's sum of its i-th row, for
// every row that ends in the tile, and thread NT - 1 returns the sum the tile leaves open (to be
// carried into the row its last item belongs to); other threads return 0.  Three barriers:
// every thread of the workgroup calls it.
template <int NT, int IPT, typename ACC>
__device__ __forceinline__ ACC merge_tile_sums(const int32_t* s_end, ACC* s_prod, int nrows,
                                               int nnzt, int k0, int* s_wf, ACC* s_wv) {
    const int tid = threadIdx.x;
    const int items = nrows + nnzt;
    const int d = min(tid * IPT, items);
    const int dend = min(d + IPT, items);
    const int i0 = merge_split(s_end, nrows, nnzt, k0, d);
    int i = i0, j = d - i0;
    ACC run = 0;
    ACC outv[IPT];
    uint32_t endmask = 0;
#pragma unroll
    for (int q = 0; q < IPT; ++q) {
        outv[q] = 0;
        if (d + q < dend) {
            if (i < nrows && (j >= nnzt || s_end[i] <= k0 + j)) {
                outv[q] = run;
                run = 0;
                endmask |= 1u << q;
                ++i;
            } else {
                run += s_prod[j];
                ++j;
            }
        }
    }

    // segmented exclusive scan of (has_end, open value) over the threads of the tile
    int f = endmask != 0;
    ACC v = run;
    const int lane = __lane_id();
#pragma unroll
    for (int o = 1; o < SPX_WAVE; o <<= 1) {
        const int fu = __shfl_up(f, o, SPX_WAVE);
        const ACC vu = __shfl_up(v, o, SPX_WAVE);
        if (lane >= o) {
            int fa = fu;
            ACC va = vu;
            seg_combine(fa, va, f, v);
            f = fa;
            v = va;
        }
    }
    const int w = tid / SPX_WAVE;
    if (lane == SPX_WAVE - 1) {
        s_wf[w] = f;
        s_wv[w] = v;
    }
    int fex = __shfl_up(f, 1, SPX_WAVE);
    ACC vex = __shfl_up(v, 1, SPX_WAVE);
    if (lane == 0) {
        fex = 0;
        vex = 0;
    }
    __syncthreads();
    int fp = 0;
    ACC vp = 0;
    for (int ww = 0; ww < w; ++ww) seg_combine(fp, vp, s_wf[ww], s_wv[ww]);
    seg_combine(fp, vp, fex, vex);
    const ACC carry_in = vp;
    ACC open = 0;
    if (tid == NT - 1) {
        int ft = fp;
        open = vp;
        seg_combine(ft, open, (int)(endmask != 0), run);
    }

    // rows that end in the thread's items, in order, into s_prod (free once every walk is done)
    __syncthreads();
    int r = i0;
    bool first = true;
#pragma unroll
    for (int q = 0; q < IPT; ++q) {
        if (endmask & (1u << q)) {
            ACC o = outv[q];
            if (first) {
                o = carry_in + o;
                first = false;
            }
            s_prod[r] = o;
            ++r;
        }
    }
    __syncthreads();
    return open;
}

// Sum, in FP64, of the open values of the run of tiles t, t + 1, ... that left row r open (the
// run can be long: up to nnz / tile length tiles for one row).  The run is read 8 tiles per step
// into 8 partial sums combined in a fixed order, so the result is deterministic.  carry(u) is
// the open value of tile u.
template <typename CarryAt>
__device__ __forceinline__ double carry_run_sum(const int32_t* __restrict__ carry_row,
                                                int32_t tiles, int t, int r, CarryAt carry) {
    double a[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    bool go = true;
    for (int u = t; go; u += 8) {
        int rr[8];
        double vv[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            rr[q] = u + q < tiles ? carry_row[u + q] : -1;
            vv[q] = u + q < tiles ? carry(u + q) : 0.0;
        }
#pragma unroll
        for (int q = 0; q < 8; ++q) {
            go = go && rr[q] == r;
            if (go) a[q] += vv[q];
        }
    }
    return ((a[0] + a[1]) + (a[2] + a[3])) + ((a[4] + a[5]) + (a[6] + a[7]));
}
