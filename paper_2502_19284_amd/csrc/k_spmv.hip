// k_spmv.hip -- y = A x kernels for the three formats (gfx950, FP64 values, int32 indices).
//
// All three are bound by HBM bandwidth (about 12 bytes of matrix per 2 flops), so the designs
// aim at fully used cache lines for the index/value streams, many independent x gathers in
// flight per thread, and a single writer per y element (partial sums go to scratch and are added
// by a second kernel in a fixed order, so results are deterministic except inside CSBH's LDS
// accumulation).
#include "dev_common.h"
#include "spx_internal.h"

// Streamed once per product: non-temporal loads/stores keep them from displacing x in L2.
template <typename T>
__device__ __forceinline__ T ntload(const T* p) {
    return __builtin_nontemporal_load(p);
}
template <typename T>
__device__ __forceinline__ void ntstore(T* p, T v) {
    __builtin_nontemporal_store(v, p);
}

// x value of a stored column index: negative indices address the compact hot copy
__device__ __forceinline__ double xval(const double* __restrict__ x,
                                       const double* __restrict__ x_hot, int32_t c) {
    return c < 0 ? x_hot[~c] : x[c];
}

// ================================================================== merge-path CRS (Section 3.3)
//
// Tile t of MP_TILE items covers diagonals [t*MP_TILE, (t+1)*MP_TILE) of the merge of
// A = row_ptr[1..m] (row ends) and B = 0..nnz-1 (entries).  The tile stages its row ends and the
// products data[k]*x[col[k]] of its entries in LDS (coalesced loads, independent gathers), then
// each thread walks MP_IPT items from its own split point: an entry adds its product to the
// running value, a row end emits it.  The running value a thread leaves open is passed to later
// threads by a segmented scan; the value the tile leaves open goes to carry[t] and is added into
// y by the fix-up kernel.

// segmented-sum combine: (flag, value) of an earlier then a later segment
__device__ __forceinline__ void seg_combine(int& f, double& v, int f_later, double v_later) {
    v = f_later ? v_later : v + v_later;
    f = f | f_later;
}

__global__ __launch_bounds__(MP_NT) void k_spmv_merge(const int32_t* __restrict__ row_ptr,
                                                      const int32_t* __restrict__ col,
                                                      const double* __restrict__ val,
                                                      const double* __restrict__ x,
                                                      const double* __restrict__ x_hot,
                                                      double* __restrict__ y,
                                                      const int2* __restrict__ coords,
                                                      int32_t* __restrict__ carry_row,
                                                      double* __restrict__ carry_val, int32_t m) {
    __shared__ int32_t s_end[MP_TILE];
    __shared__ double s_prod[MP_TILE];
    __shared__ int s_wf[MP_NT / SPX_WAVE];
    __shared__ double s_wv[MP_NT / SPX_WAVE];

    const int tid = threadIdx.x;
    const int t = blockIdx.x;
    const int2 c0 = coords[t];
    const int2 c1 = coords[t + 1];
    const int r0 = c0.x, k0 = c0.y;
    const int nrows = c1.x - r0, nnzt = c1.y - k0;

    for (int i = tid; i < nrows; i += MP_NT) s_end[i] = ntload(row_ptr + r0 + 1 + i);
#pragma unroll
    for (int q = 0; q < MP_IPT; ++q) {
        const int i = q * MP_NT + tid;
        if (i < nnzt) s_prod[i] = ntload(val + k0 + i) * xval(x, x_hot, ntload(col + k0 + i));
    }
    __syncthreads();

    const int items = nrows + nnzt;
    const int d = min(tid * MP_IPT, items);
    const int dend = min(d + MP_IPT, items);
    int lo = max(0, d - nnzt), hi = min(d, nrows);
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (s_end[mid] <= k0 + d - mid - 1) lo = mid + 1;
        else hi = mid;
    }
    const int i0 = lo;
    int i = lo, j = d - lo;
    double run = 0.0;
    double outv[MP_IPT];
    uint32_t endmask = 0;
#pragma unroll
    for (int q = 0; q < MP_IPT; ++q) {
        outv[q] = 0.0;
        if (d + q < dend) {
            if (i < nrows && (j >= nnzt || s_end[i] <= k0 + j)) {
                outv[q] = run;
                run = 0.0;
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
    double v = run;
    {
        const int lane = __lane_id();
#pragma unroll
        for (int o = 1; o < SPX_WAVE; o <<= 1) {
            const int fu = __shfl_up(f, o, SPX_WAVE);
            const double vu = __shfl_up(v, o, SPX_WAVE);
            if (lane >= o) {
                int fa = fu;
                double va = vu;
                seg_combine(fa, va, f, v);
                f = fa;
                v = va;
            }
        }
    }
    const int w = tid / SPX_WAVE;
    const int lane = __lane_id();
    if (lane == SPX_WAVE - 1) {
        s_wf[w] = f;
        s_wv[w] = v;
    }
    // exclusive value within the wave
    int fex = __shfl_up(f, 1, SPX_WAVE);
    double vex = __shfl_up(v, 1, SPX_WAVE);
    if (lane == 0) {
        fex = 0;
        vex = 0.0;
    }
    __syncthreads();
    int fp = 0;
    double vp = 0.0;
    for (int ww = 0; ww < w; ++ww) seg_combine(fp, vp, s_wf[ww], s_wv[ww]);
    seg_combine(fp, vp, fex, vex);
    const double carry_in = vp;

    // the tile's open value leaves through carry[t]
    if (tid == MP_NT - 1) {
        int ft = fp;
        double vt = vp;
        seg_combine(ft, vt, endmask != 0, run);
        carry_row[t] = c1.x;  // m when nothing is left open
        carry_val[t] = vt;
    }

    // emit rows: stage in LDS (reusing s_prod), then coalesced stores
    __syncthreads();
    int r = i0;
    bool first = true;
#pragma unroll
    for (int q = 0; q < MP_IPT; ++q) {
        if (endmask & (1u << q)) {
            double o = outv[q];
            if (first) {
                o = carry_in + o;
                first = false;
            }
            s_prod[r] = o;
            ++r;
        }
    }
    __syncthreads();
    for (int q = tid; q < nrows; q += MP_NT) ntstore(y + r0 + q, s_prod[q]);
}

// Adds each tile's open value into y, tiles in order.  The first tile of a run of tiles that
// left the same row open sums the whole run, so every row is updated by one thread.
__global__ void k_spmv_merge_fixup(const int32_t* __restrict__ carry_row,
                                   const double* __restrict__ carry_val, int32_t tiles,
                                   double* __restrict__ y, int32_t m) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= tiles) return;
    const int r = carry_row[t];
    if (r >= m) return;
    if (t > 0 && carry_row[t - 1] == r) return;
    double acc = carry_val[t];
    for (int u = t + 1; u < tiles && carry_row[u] == r; ++u) acc = acc + carry_val[u];
    y[r] = acc + y[r];
}

hipError_t spmv_merge(const spx_matrix_s* A, const double* x, double* y, hipStream_t s) {
    if (A->mp_tiles <= 0) return hipSuccess;
    hipError_t e = launch_hot_gather(A->hot_cols, A->nhot, x, A->x_hot, s);
    if (e != hipSuccess) return e;
    SPX_LAUNCH("spmv_merge", k_spmv_merge, dim3(A->mp_tiles), dim3(MP_NT), 0, s, A->row_ptr, A->col,
               A->val, x, A->x_hot, y, A->mp_coords, A->mp_carry_row, A->mp_carry_val, A->m);
    SPX_LAUNCH("spmv_merge_fixup", k_spmv_merge_fixup, dim3(spx_div_up(A->mp_tiles, 256)), dim3(256), 0, s,
                       A->mp_carry_row, A->mp_carry_val, A->mp_tiles, y, A->m);
    return hipGetLastError();
}

// ================================================================== row-split CRS
//
// Workgroup b owns the rows [blocks[b], blocks[b+1]).  A block of short rows (< RS_NNZ entries,
// <= RS_ROWS rows) stages its products in LDS with coalesced loads; then groups of g lanes
// (g = largest power of two <= 64 with rows*g <= RS_NT) each reduce one row at a time, with a
// shuffle tree inside the group.  Rows longer than RS_LONG are blocks on their own and are skipped
// here: their RS_CHUNK-entry chunks are summed by k_spmv_rowsplit_long and the chunk sums added in
// chunk order by k_spmv_rowsplit_finish.

__global__ __launch_bounds__(RS_NT) void k_spmv_rowsplit(const int32_t* __restrict__ row_ptr,
                                                         const int32_t* __restrict__ col,
                                                         const double* __restrict__ val,
                                                         const double* __restrict__ x,
                                                         const double* __restrict__ x_hot,
                                                         double* __restrict__ y,
                                                         const int32_t* __restrict__ blocks) {
    __shared__ double s_prod[RS_NNZ];
    __shared__ int32_t s_rp[RS_ROWS + 1];
    const int tid = threadIdx.x;
    const int rs = blocks[blockIdx.x], re = blocks[blockIdx.x + 1];
    const int rows = re - rs;
    const int base = row_ptr[rs];
    const int nnzb = row_ptr[re] - base;
    if (rows == 1 && nnzb > RS_LONG) return;  // long row: chunk kernels
    const bool staged = nnzb <= RS_NNZ && rows <= RS_ROWS;
    if (staged) {
        for (int i = tid; i <= rows; i += RS_NT) s_rp[i] = ntload(row_ptr + rs + i) - base;
#pragma unroll
        for (int q = 0; q < RS_NNZ / RS_NT; ++q) {
            const int i = q * RS_NT + tid;
            if (i < nnzb) s_prod[i] = ntload(val + base + i) * xval(x, x_hot, ntload(col + base + i));
        }
        __syncthreads();
    }
    int g = 64;
    while (g > 1 && rows * g > RS_NT) g >>= 1;
    const int grp = tid / g, gl = tid % g, ngrp = RS_NT / g;
    for (int r = grp; r < rows; r += ngrp) {
        double acc = 0.0;
        if (staged) {
            const int a = s_rp[r], b = s_rp[r + 1];
            for (int k = a + gl; k < b; k += g) acc += s_prod[k];
        } else {
            const int a = row_ptr[rs + r], b = row_ptr[rs + r + 1];
            for (int k = a + gl; k < b; k += g) acc += val[k] * xval(x, x_hot, col[k]);
        }
        for (int o = g >> 1; o > 0; o >>= 1) acc += __shfl_xor(acc, o, SPX_WAVE);
        if (gl == 0) y[rs + r] = acc;
    }
}

__global__ __launch_bounds__(RS_NT) void k_spmv_rowsplit_long(
    const int32_t* __restrict__ row_ptr, const int32_t* __restrict__ col,
    const double* __restrict__ val, const double* __restrict__ x,
    const double* __restrict__ x_hot, const int32_t* __restrict__ long_rows, const int32_t* __restrict__ chunk_ptr, int32_t nlong,
    double* __restrict__ partials) {
    __shared__ double s_tmp[RS_NT / SPX_WAVE];
    const int c = blockIdx.x;
    // the long row that owns chunk c: last j with chunk_ptr[j] <= c
    int lo = 0, hi = nlong - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (chunk_ptr[mid] <= c) lo = mid;
        else hi = mid - 1;
    }
    const int r = long_rows[lo];
    const int kb = row_ptr[r] + (c - chunk_ptr[lo]) * RS_CHUNK;
    const int ke = min(kb + RS_CHUNK, row_ptr[r + 1]);
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    int k = kb + threadIdx.x;
    for (; k + 3 * RS_NT < ke; k += 4 * RS_NT) {
#pragma unroll
        for (int q = 0; q < 4; ++q)
            acc[q] += ntload(val + k + q * RS_NT) * xval(x, x_hot, ntload(col + k + q * RS_NT));
    }
    for (; k < ke; k += RS_NT) acc[0] += ntload(val + k) * xval(x, x_hot, ntload(col + k));
    double sum = block_reduce<RS_NT, double, OpSum<double>>((acc[0] + acc[1]) + (acc[2] + acc[3]),
                                                             s_tmp);
    if (threadIdx.x == 0) partials[c] = sum;
}

__global__ void k_spmv_rowsplit_finish(const int32_t* __restrict__ long_rows,
                                       const int32_t* __restrict__ chunk_ptr, int32_t nlong,
                                       const double* __restrict__ partials,
                                       double* __restrict__ y) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= nlong) return;
    double acc = 0.0;
    for (int c = chunk_ptr[j]; c < chunk_ptr[j + 1]; ++c) acc = acc + partials[c];
    y[long_rows[j]] = acc;
}

hipError_t spmv_rowsplit(const spx_matrix_s* A, const double* x, double* y, hipStream_t s) {
    hipError_t e = launch_hot_gather(A->hot_cols, A->nhot, x, A->x_hot, s);
    if (e != hipSuccess) return e;
    if (A->rs_nb > 0)
        SPX_LAUNCH("spmv_rowsplit", k_spmv_rowsplit, dim3(A->rs_nb), dim3(RS_NT), 0, s, A->row_ptr,
                   A->col, A->val, x, A->x_hot, y, A->rs_blocks);
    if (A->rs_nlong > 0) {
        SPX_LAUNCH("spmv_rowsplit_long", k_spmv_rowsplit_long, dim3(A->rs_nchunks), dim3(RS_NT), 0, s,
                           A->row_ptr, A->col, A->val, x, A->x_hot, A->rs_long_rows, A->rs_chunk_ptr,
                           A->rs_nlong, A->rs_partials);
        SPX_LAUNCH("spmv_rowsplit_finish", k_spmv_rowsplit_finish, dim3(spx_div_up(A->rs_nlong, 256)), dim3(256),
                           0, s, A->rs_long_rows, A->rs_chunk_ptr, A->rs_nlong, A->rs_partials, y);
    }
    return hipGetLastError();
}

// ================================================================== CSBH (Sections 3.1, 4.1)
//
// Work unit u = entries [k0, k1) of block row br (at most the unit size).  The workgroup keeps
// the block row's beta-entry slice of y in LDS and adds every product into it (LDS float atomics;
// the Hilbert order keeps consecutive entries of a block in nearby rows and columns).  Each
// thread takes CB_IPT consecutive entries; it finds the block of its first entry by binary search
// over the block row's pointers (staged in LDS when they fit) and walks forward from there.
// A unit that covers its whole block row writes the slice to y; otherwise it writes a partial
// slice to scratch and k_spmv_csbh_reduce adds the partial slices of the block row in unit order.

__global__ __launch_bounds__(CB_NT) void k_spmv_csbh(const int32_t* __restrict__ blk_ptr,
                                                     const uint32_t* __restrict__ packed,
                                                     const double* __restrict__ val,
                                                     const double* __restrict__ x,
                                                     double* __restrict__ y,
                                                     double* __restrict__ partials,
                                                     const int4* __restrict__ units, int k,
                                                     int32_t nbc, int32_t m, int stage_bp) {
    extern __shared__ double s_dyn[];
    const int beta = 1 << k;
    double* s_y = s_dyn;
    int32_t* s_bp = (int32_t*)(s_dyn + beta);
    const int tid = threadIdx.x;
    const int4 U = units[blockIdx.x];
    const int br = U.x, kb = U.y, ke = U.z, slot = U.w;
    const int32_t* gbp = blk_ptr + (int64_t)br * nbc;
    for (int i = tid; i < beta; i += CB_NT) s_y[i] = 0.0;
    if (stage_bp)
        for (int i = tid; i <= nbc; i += CB_NT) s_bp[i] = gbp[i];
    __syncthreads();
    const int32_t* bp = stage_bp ? s_bp : gbp;
    const uint32_t lmask = (uint32_t)beta - 1u;

    for (int base = kb; base < ke; base += CB_NT * CB_IPT) {
        const int k_first = base + tid * CB_IPT;
        if (k_first < ke) {
            // block b with bp[b] <= k_first < bp[b+1]
            int lo = 0, hi = nbc - 1;
            while (lo < hi) {
                const int mid = (lo + hi + 1) >> 1;
                if (bp[mid] <= k_first) lo = mid;
                else hi = mid - 1;
            }
            int b = lo;
            int next = bp[b + 1];
#pragma unroll
            for (int q = 0; q < CB_IPT; ++q) {
                const int kk = k_first + q;
                if (kk < ke) {
                    while (next <= kk && b < nbc - 1) {
                        ++b;
                        next = bp[b + 1];
                    }
                    const uint32_t p = ntload(packed + kk);
                    const int c = (b << k) + (int)(p & lmask);
                    atomicAdd(&s_y[p >> 16], ntload(val + kk) * x[c]);
                }
            }
        }
    }
    __syncthreads();
    const int row0 = br << k;
    const int rows = min(beta, m - row0);
    if (slot < 0) {
        for (int i = tid; i < rows; i += CB_NT) ntstore(y + row0 + i, s_y[i]);
    } else {
        double* dst = partials + (int64_t)slot * beta;
        for (int i = tid; i < rows; i += CB_NT) dst[i] = s_y[i];
    }
}

__global__ __launch_bounds__(256) void k_spmv_csbh_reduce(const int4* __restrict__ split,
                                                          const double* __restrict__ partials,
                                                          double* __restrict__ y, int k,
                                                          int32_t m) {
    const int4 S = split[blockIdx.x];
    const int beta = 1 << k;
    const int row0 = S.x << k;
    const int rows = min(beta, m - row0);
    for (int i = threadIdx.x; i < rows; i += 256) {
        double acc = 0.0;
        for (int q = 0; q < S.z; ++q) acc = acc + partials[(int64_t)(S.y + q) * beta + i];
        y[row0 + i] = acc;
    }
}

hipError_t spmv_csbh(const spx_matrix_s* A, const double* x, double* y, hipStream_t s) {
    if (A->cb_nunits <= 0) return hipSuccess;
    const int beta = 1 << A->log2_beta;
    const int stage_bp = (A->nbc + 1 <= CB_BP_STAGE_MAX) ? 1 : 0;
    const size_t lds = (size_t)beta * sizeof(double) + (stage_bp ? (size_t)(A->nbc + 1) * 4 : 0);
    if (lds > 64 * 1024) {
        hipError_t e = hipFuncSetAttribute((const void*)k_spmv_csbh,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
    }
    SPX_LAUNCH("spmv_csbh", k_spmv_csbh, dim3(A->cb_nunits), dim3(CB_NT), lds, s, A->blk_ptr,
                       A->packed, A->val, x, y, A->cb_partials, A->cb_units, A->log2_beta,
                       (int32_t)A->nbc, A->m, stage_bp);
    if (A->cb_nsplit > 0)
        SPX_LAUNCH("spmv_csbh_reduce", k_spmv_csbh_reduce, dim3(A->cb_nsplit), dim3(256), 0, s, A->cb_split,
                           A->cb_partials, y, A->log2_beta, A->m);
    return hipGetLastError();
}
