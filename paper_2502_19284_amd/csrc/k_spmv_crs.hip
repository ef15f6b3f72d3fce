// k_spmv_crs.hip -- y = A x for the CRS formats (merge-path and row-split), gfx950.
//
// Templated on the stored value type V (double, float, or bfloat16 bits), the vector type X of
// x and y (double for FP64 matrices, float for reduced-precision ones) and the accumulator ACC
// used inside a tile or row block.  Sums that cross tiles (merge carries) and rows longer than a
// row block (row-split long-row chunks) are always accumulated in FP64.
//
// All kernels are bound by memory traffic (about 12 bytes of matrix per 2 flops in FP64), and
// within it by the x gathers (one cache request per entry).  Matrix streams and y use
// non-temporal loads/stores so they do not displace x from L2; hot columns read the compact copy
// x_hot (see k_hot.hip).  Every y element has a single writer; partial sums go to scratch and are
// added by a second kernel in a fixed order, so results are deterministic.
#include "dev_common.h"
#include "dev_merge.h"
#include "dev_values.h"
#include "spx_internal.h"

// x value of a stored column index: negative indices address the compact hot copy
template <typename X>
__device__ __forceinline__ X xval(const X* __restrict__ x, const X* __restrict__ x_hot,
                                  int32_t c) {
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

template <typename V, typename X, typename ACC>
__global__ __launch_bounds__(MP_NT) void k_spmv_merge(
    const int32_t* __restrict__ row_ptr, const int32_t* __restrict__ col,
    const V* __restrict__ val, const X* __restrict__ x, const X* __restrict__ x_hot,
    X* __restrict__ y, const int2* __restrict__ coords, int32_t* __restrict__ carry_row,
    double* __restrict__ carry_val) {
    __shared__ int32_t s_end[MP_TILE];
    __shared__ ACC s_prod[MP_TILE];
    __shared__ int s_wf[MP_NT / SPX_WAVE];
    __shared__ ACC s_wv[MP_NT / SPX_WAVE];

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
        if (i < nnzt)
            s_prod[i] = (ACC)vget(val + k0 + i) * (ACC)xval(x, x_hot, ntload(col + k0 + i));
    }
    __syncthreads();

    const ACC open = merge_tile_sums<MP_NT, MP_IPT, ACC>(s_end, s_prod, nrows, nnzt, k0, s_wf,
                                                          s_wv);
    // the tile's open value leaves through carry[t]
    if (tid == MP_NT - 1) {
        carry_row[t] = c1.x;  // m when nothing is left open
        carry_val[t] = (double)open;
    }
    for (int q = tid; q < nrows; q += MP_NT) ntstore(y + r0 + q, (X)s_prod[q]);
}

// Adds each tile's open value into y in FP64.  The first tile of a run of tiles that left the
// same row open sums the whole run (carry_run_sum: fixed order, deterministic), so every row is
// updated by one thread.
template <typename X>
__global__ void k_spmv_merge_fixup(const int32_t* __restrict__ carry_row,
                                   const double* __restrict__ carry_val, int32_t tiles,
                                   X* __restrict__ y, int32_t m) {
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= tiles) return;
    const int r = carry_row[t];
    if (r >= m) return;
    if (t > 0 && carry_row[t - 1] == r) return;
    const double acc =
        carry_run_sum(carry_row, tiles, t, r, [&](int u) { return carry_val[u]; });
    y[r] = (X)(acc + (double)y[r]);
}

template <typename X>
__global__ void k_hot_gather_t(const int32_t* __restrict__ hot_cols, int32_t nhot,
                               const X* __restrict__ x, X* __restrict__ x_hot) {
    const int h = blockIdx.x * blockDim.x + threadIdx.x;
    if (h < nhot) x_hot[h] = x[hot_cols[h]];
}

template <typename X>
static hipError_t hot_gather(const spx_matrix_s* A, const X* x, hipStream_t s) {
    if (A->nhot <= 0) return hipSuccess;
    SPX_LAUNCH("hot_gather", k_hot_gather_t<X>, dim3(spx_div_up(A->nhot, 256)), dim3(256), 0, s,
               A->hot_cols, A->nhot, x, (X*)A->x_hot);
    return hipGetLastError();
}

// The merge-path product on explicit tiles, carries and hot-x scratch (the handle's own for
// spmv, a caller's plan for the one-column product of spx_spmm).
template <typename V, typename X, typename ACC>
static hipError_t merge_run(const spx_matrix_s* A, const V* val, const X* x, X* y,
                            const int2* coords, int32_t tiles, int32_t* crow, double* cval,
                            X* x_hot, hipStream_t s) {
    if (tiles <= 0) return hipSuccess;
    if (A->nhot > 0)
        SPX_LAUNCH("hot_gather", k_hot_gather_t<X>, dim3(spx_div_up(A->nhot, 256)), dim3(256), 0,
                   s, A->hot_cols, A->nhot, x, x_hot);
    SPX_LAUNCH("spmv_merge", (k_spmv_merge<V, X, ACC>), dim3(tiles), dim3(MP_NT), 0, s,
               A->row_ptr, A->col, val, x, (const X*)x_hot, y, coords, crow, cval);
    SPX_LAUNCH("spmv_merge_fixup", k_spmv_merge_fixup<X>, dim3(spx_div_up(tiles, 256)),
               dim3(256), 0, s, crow, cval, tiles, y, A->m);
    return hipGetLastError();
}

template <typename V, typename X, typename ACC>
static hipError_t merge_t(const spx_matrix_s* A, const V* val, const X* x, X* y, hipStream_t s) {
    return merge_run<V, X, ACC>(A, val, x, y, A->mp_coords, A->mp_tiles, A->mp_carry_row,
                                A->mp_carry_val, (X*)A->x_hot, s);
}

hipError_t spmv_merge_on_plan(const spx_matrix_s* A, const SpmmPlan& P, const void* x, void* y,
                              hipStream_t s) {
    switch (A->value_type) {
        case SPX_F64:
            return merge_run<double, double, double>(A, A->val, (const double*)x, (double*)y,
                                                     P.coords, P.tiles, P.carry_row, P.carry_val,
                                                     (double*)P.h, s);
        case SPX_F32:
            return merge_run<float, float, float>(A, (const float*)A->val_lp, (const float*)x,
                                                  (float*)y, P.coords, P.tiles, P.carry_row,
                                                  P.carry_val, (float*)P.h, s);
        default:
            return merge_run<uint16_t, float, float>(A, (const uint16_t*)A->val_lp,
                                                     (const float*)x, (float*)y, P.coords,
                                                     P.tiles, P.carry_row, P.carry_val,
                                                     (float*)P.h, s);
    }
}

// ================================================================== row-split CRS
//
// Workgroup b owns the rows [blocks[b], blocks[b+1]).  A block of short rows (< RS_NNZ entries,
// <= RS_ROWS rows) stages its products in LDS with coalesced loads; then groups of g lanes
// (g = largest power of two <= 64 with rows*g <= RS_NT) each reduce one row at a time, with a
// shuffle tree inside the group.  Rows longer than RS_LONG are blocks on their own and are skipped
// there: their RS_CHUNK-entry chunks are summed (in FP64) by other workgroups of the same launch
// and the chunk sums added in chunk order by k_spmv_rowsplit_finish.

template <typename V, typename X, typename ACC>
__device__ __forceinline__ void rowsplit_block(const int32_t* __restrict__ row_ptr,
                                               const int32_t* __restrict__ col,
                                               const V* __restrict__ val,
                                               const X* __restrict__ x,
                                               const X* __restrict__ x_hot, X* __restrict__ y,
                                               const int32_t* __restrict__ blocks, int b,
                                               ACC* s_prod, int32_t* s_rp) {
    const int tid = threadIdx.x;
    const int rs = blocks[b], re = blocks[b + 1];
    const int rows = re - rs;
    const int base = row_ptr[rs];
    const int nnzb = row_ptr[re] - base;
    if (rows == 1 && nnzb > RS_LONG) return;  // long row: chunk path
    const bool staged = nnzb <= RS_NNZ && rows <= RS_ROWS;
    if (staged) {
        for (int i = tid; i <= rows; i += RS_NT) s_rp[i] = ntload(row_ptr + rs + i) - base;
#pragma unroll
        for (int q = 0; q < RS_NNZ / RS_NT; ++q) {
            const int i = q * RS_NT + tid;
            if (i < nnzb)
                s_prod[i] =
                    (ACC)vget(val + base + i) * (ACC)xval(x, x_hot, ntload(col + base + i));
        }
        __syncthreads();
    }
    int g = 64;
    while (g > 1 && rows * g > RS_NT) g >>= 1;
    const int grp = tid / g, gl = tid % g, ngrp = RS_NT / g;
    for (int r = grp; r < rows; r += ngrp) {
        ACC acc = 0;
        if (staged) {
            const int a = s_rp[r], b2 = s_rp[r + 1];
            for (int k = a + gl; k < b2; k += g) acc += s_prod[k];
        } else {
            const int a = row_ptr[rs + r], b2 = row_ptr[rs + r + 1];
            for (int k = a + gl; k < b2; k += g)
                acc += (ACC)vget_plain(val + k) * (ACC)xval(x, x_hot, col[k]);
        }
        for (int o = g >> 1; o > 0; o >>= 1) acc += __shfl_xor(acc, o, SPX_WAVE);
        if (gl == 0) y[rs + r] = (X)acc;
    }
}

template <typename V, typename X>
__device__ __forceinline__ void rowsplit_chunk(const int32_t* __restrict__ row_ptr,
                                               const int32_t* __restrict__ col,
                                               const V* __restrict__ val,
                                               const X* __restrict__ x,
                                               const X* __restrict__ x_hot,
                                               const int32_t* __restrict__ long_rows,
                                               const int32_t* __restrict__ chunk_ptr,
                                               int32_t nlong, double* __restrict__ partials,
                                               int c, double* s_tmp) {
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
            acc[q] += (double)vget(val + k + q * RS_NT) *
                      (double)xval(x, x_hot, ntload(col + k + q * RS_NT));
    }
    for (; k < ke; k += RS_NT) acc[0] += (double)vget(val + k) * (double)xval(x, x_hot, ntload(col + k));
    const double sum = block_reduce<RS_NT, double, OpSum<double>>((acc[0] + acc[1]) + (acc[2] + acc[3]),
                                                                   s_tmp);
    if (threadIdx.x == 0) partials[c] = sum;
}

// One launch for both kinds of work: workgroups [0, nchunks) sum the long rows' chunks (the
// heavier items first), the rest take the row blocks.
template <typename V, typename X, typename ACC>
__global__ __launch_bounds__(RS_NT) void k_spmv_rowsplit(
    const int32_t* __restrict__ row_ptr, const int32_t* __restrict__ col,
    const V* __restrict__ val, const X* __restrict__ x, const X* __restrict__ x_hot,
    X* __restrict__ y, const int32_t* __restrict__ blocks, const int32_t* __restrict__ long_rows,
    const int32_t* __restrict__ chunk_ptr, int32_t nlong, int32_t nchunks,
    double* __restrict__ partials) {
    __shared__ ACC s_prod[RS_NNZ];
    __shared__ int32_t s_rp[RS_ROWS + 1];
    __shared__ double s_tmp[RS_NT / SPX_WAVE];
    const int b = blockIdx.x;
    if (b < nchunks)
        rowsplit_chunk<V, X>(row_ptr, col, val, x, x_hot, long_rows, chunk_ptr, nlong, partials, b,
                             s_tmp);
    else
        rowsplit_block<V, X, ACC>(row_ptr, col, val, x, x_hot, y, blocks, b - nchunks, s_prod,
                                  s_rp);
}

template <typename X>
__global__ void k_spmv_rowsplit_finish(const int32_t* __restrict__ long_rows,
                                       const int32_t* __restrict__ chunk_ptr, int32_t nlong,
                                       const double* __restrict__ partials, X* __restrict__ y) {
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= nlong) return;
    double acc = 0.0;
    for (int c = chunk_ptr[j]; c < chunk_ptr[j + 1]; ++c) acc = acc + partials[c];
    y[long_rows[j]] = (X)acc;
}

template <typename V, typename X, typename ACC>
static hipError_t rowsplit_t(const spx_matrix_s* A, const V* val, const X* x, X* y,
                             hipStream_t s) {
    hipError_t e = hot_gather<X>(A, x, s);
    if (e != hipSuccess) return e;
    const int32_t nchunks = A->rs_nlong > 0 ? A->rs_nchunks : 0;
    if (A->rs_nb + nchunks > 0)
        SPX_LAUNCH("spmv_rowsplit", (k_spmv_rowsplit<V, X, ACC>), dim3(A->rs_nb + nchunks),
                   dim3(RS_NT), 0, s, A->row_ptr, A->col, val, x, (const X*)A->x_hot, y,
                   A->rs_blocks, A->rs_long_rows, A->rs_chunk_ptr, A->rs_nlong, nchunks,
                   A->rs_partials);
    if (A->rs_nlong > 0) {
        SPX_LAUNCH("spmv_rowsplit_finish", k_spmv_rowsplit_finish<X>,
                   dim3(spx_div_up(A->rs_nlong, 256)), dim3(256), 0, s, A->rs_long_rows,
                   A->rs_chunk_ptr, A->rs_nlong, A->rs_partials, y);
    }
    return hipGetLastError();
}

// ================================================================== dispatch

hipError_t spmv_merge(const spx_matrix_s* A, const double* x, double* y, hipStream_t s) {
    return merge_t<double, double, double>(A, A->val, x, y, s);
}

hipError_t spmv_rowsplit(const spx_matrix_s* A, const double* x, double* y, hipStream_t s) {
    return rowsplit_t<double, double, double>(A, A->val, x, y, s);
}

hipError_t spmv_crs_f32(const spx_matrix_s* A, const float* x, float* y, hipStream_t s) {
    if (A->value_type == SPX_F32) {
        const float* v = (const float*)A->val_lp;
        return A->fmt == SPX_CSR_MERGE ? merge_t<float, float, float>(A, v, x, y, s)
                                       : rowsplit_t<float, float, float>(A, v, x, y, s);
    }
    const uint16_t* v = (const uint16_t*)A->val_lp;
    return A->fmt == SPX_CSR_MERGE ? merge_t<uint16_t, float, float>(A, v, x, y, s)
                                   : rowsplit_t<uint16_t, float, float>(A, v, x, y, s);
}

// ================================================================== value rounding at conversion

// Round-to-nearest-even of a double to bfloat16, returned as its 16 bits (sign, 8-bit exponent
// with bias 127, 7 fraction bits), from the bit fields of the double: in the normal range the 52
// fraction bits are cut to 7 and the 45 cut bits decide the rounding (above half: up; exactly
// half: up only if the kept fraction is odd), a carry out of the fraction stepping the exponent
// (up to the infinity); below 2^-126 the value is counted in units of the subnormal spacing
// 2^-133 with the same rule.  NaN stays a (quiet) NaN, zeros and infinities keep their sign.
__device__ __forceinline__ uint16_t bf16_rne(double v) {
    const uint64_t bits = (uint64_t)__double_as_longlong(v);
    const uint16_t sign = (uint16_t)((bits >> 48) & 0x8000u);
    const int ex = (int)((bits >> 52) & 0x7FF);
    const uint64_t frac = bits & ((1ull << 52) - 1ull);
    if (ex == 0x7FF) return sign | (frac ? 0x7FC0u : 0x7F80u);  // NaN / infinity
    const int E = ex - 1023;                                     // v = 1.frac 2^E (ex > 0)
    if (ex == 0 || E < -134) return sign;  // below half the subnormal spacing (or a zero)
    uint64_t kept, cut, half;
    if (E >= -126) {  // normal: exponent field E + 127, 7 fraction bits
        kept = ((uint64_t)(E + 127) << 7) | (frac >> 45);
        cut = frac & ((1ull << 45) - 1ull);
        half = 1ull << 44;
    } else {  // subnormal: |v| / 2^-133 = (2^52 + frac) 2^(E + 81), shift = -(E + 81) in 46..53
        const uint64_t sig = (1ull << 52) | frac;
        const int sh = -(E + 81);
        kept = sig >> sh;
        cut = sig & ((1ull << sh) - 1ull);
        half = 1ull << (sh - 1);
    }
    const bool up = cut > half || (cut == half && (kept & 1ull));
    kept += up ? 1u : 0u;  // may carry into the exponent; 0x7F80 is the infinity
    return sign | (uint16_t)(kept > 0x7F80u ? 0x7F80u : kept);
}

__global__ void k_round_values(const double* __restrict__ in, int64_t n, int32_t vt,
                               void* __restrict__ out) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        if (vt == SPX_F32) ((float*)out)[i] = (float)in[i];
        else ((uint16_t*)out)[i] = bf16_rne(in[i]);
    }
}

hipError_t launch_round_values(const double* in, int64_t n, int32_t vt, void* out,
                               hipStream_t s) {
    if (n <= 0) return hipSuccess;
    int64_t g = (n + 255) / 256;
    if (g > 65536) g = 65536;
    SPX_LAUNCH("round_values", k_round_values, dim3((unsigned)g), dim3(256), 0, s, in, n, vt, out);
    return hipGetLastError();
}
