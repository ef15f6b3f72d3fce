// k_spmm.hip -- Y = A X for k right-hand sides on the CRS formats (gfx950).
//
// Each column of Y is the product of Section 2's definition with one column of X; the k columns
// share one pass over the matrix, so the matrix stream is read once per k products.
//
// X reaches the product kernel as rows: the kc values X[j, c0 .. c0+kc) of column chunk c0 sit
// next to each other, so the kc lanes that serve one entry read one contiguous run (kc = 32 FP32
// values = one 128-byte line) instead of kc scattered values.  A row-major X is read in place; a
// column-major X (column c at X + c*ldx, the BLAS layout) is first copied into that row-major form
// by an LDS-tiled transpose.  Hot columns (k_hot.hip) get their own compact rows.  Y leaves the
// same way: kc lanes store one row's kc results as one contiguous run, and a column-major Y is
// written from a row-major scratch by the reverse transpose (scattered 4-byte stores into kc
// columns cost several times the whole product).
//
// Work is split as in merge-path SpMV (Section 3.3): tile t covers MP_TILE items of the merge of
// row ends and entries.  Within a tile, groups of KP lanes (KP = kc rounded up to a power of two)
// each walk MP_TILE * KP / MP_NT consecutive items; lane c of a group accumulates column c.  A
// group's first finished row and its open value at the end are combined across the groups of the
// tile by a segmented scan in LDS; the value the tile leaves open goes to carry[t][c] (FP64) and
// the fix-up kernel adds those into Y in tile order, so results are deterministic.  Accumulation
// inside a tile is in ACC (FP64 for FP64 matrices, FP32 for FP32/bfloat16 values), across tiles in
// FP64, as in the single-vector kernels.
#include "dev_common.h"
#include "dev_merge.h"
#include "dev_values.h"
#include "spx_internal.h"

#define MM_KMAX 64     // columns per chunk (one wave of lanes)
#define MM_STAGE_ROWS 64

// Z[j*kc + c] = X[j + c*ldx] for j < n, c < kc: column-major chunk -> row-major copy
template <typename X>
__global__ __launch_bounds__(256) void k_spmm_stage(const X* __restrict__ x, int64_t ldx,
                                                    int32_t n, int32_t kc, X* __restrict__ z) {
    __shared__ X s[MM_STAGE_ROWS * (MM_KMAX + 1)];
    const int64_t j0 = (int64_t)blockIdx.x * MM_STAGE_ROWS;
    const int rows = (int)min((int64_t)MM_STAGE_ROWS, (int64_t)n - j0);
    for (int e = threadIdx.x; e < MM_STAGE_ROWS * kc; e += 256) {
        const int c = e / MM_STAGE_ROWS, r = e % MM_STAGE_ROWS;
        if (r < rows) s[r * (MM_KMAX + 1) + c] = ntload(x + j0 + r + (int64_t)c * ldx);
    }
    __syncthreads();
    for (int e = threadIdx.x; e < rows * kc; e += 256) {
        const int r = e / kc, c = e % kc;
        z[(j0 + r) * kc + c] = s[r * (MM_KMAX + 1) + c];
    }
}

// Y[i + c*ldy] = W[i*kc + c] for i < m, c < kc: row-major result chunk -> column-major Y
template <typename X>
__global__ __launch_bounds__(256) void k_spmm_unstage(const X* __restrict__ w, int32_t m,
                                                      int32_t kc, X* __restrict__ y, int64_t ldy) {
    __shared__ X s[MM_STAGE_ROWS * (MM_KMAX + 1)];
    const int64_t i0 = (int64_t)blockIdx.x * MM_STAGE_ROWS;
    const int rows = (int)min((int64_t)MM_STAGE_ROWS, (int64_t)m - i0);
    for (int e = threadIdx.x; e < rows * kc; e += 256) {
        const int r = e / kc, c = e % kc;
        s[r * (MM_KMAX + 1) + c] = w[(i0 + r) * kc + c];
    }
    __syncthreads();
    for (int e = threadIdx.x; e < MM_STAGE_ROWS * kc; e += 256) {
        const int c = e / MM_STAGE_ROWS, r = e % MM_STAGE_ROWS;
        if (r < rows) ntstore(y + i0 + r + (int64_t)c * ldy, s[r * (MM_KMAX + 1) + c]);
    }
}

// H[h*kc + c] = R[hot_cols[h]*ldr + c]: compact rows of the hot columns from row-major R
template <typename X>
__global__ void k_spmm_hot(const int32_t* __restrict__ hot_cols, int32_t nhot,
                           const X* __restrict__ r, int64_t ldr, int32_t kc,
                           X* __restrict__ h) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (int64_t)nhot * kc) return;
    const int64_t hh = e / kc;
    const int c = (int)(e - hh * kc);
    h[e] = r[(int64_t)hot_cols[hh] * ldr + c];
}

template <typename X>
__device__ __forceinline__ X* mm_yptr(X* y, int64_t ldy, int row_major, int64_t r, int c) {
    return row_major ? y + r * ldy + c : y + r + (int64_t)c * ldy;
}

template <typename V, typename X, typename ACC, int KP>
__global__ __launch_bounds__(MP_NT) void k_spmm_merge(
    const int32_t* __restrict__ row_ptr, const int32_t* __restrict__ col,
    const V* __restrict__ val, const X* __restrict__ xr, int64_t ldr, const X* __restrict__ xh,
    int32_t kc, X* __restrict__ y, int64_t ldy, int row_major, const int2* __restrict__ coords,
    int32_t* __restrict__ carry_row, double* __restrict__ carry_val) {
    constexpr int NG = MP_NT / KP;     // groups per tile
    constexpr int IPG = MP_TILE / NG;  // items per group
    constexpr int U = 8;               // gathers in flight per lane
    __shared__ int32_t s_end[MP_TILE];
    __shared__ int32_t s_col[MP_TILE];
    __shared__ ACC s_val[MP_TILE];
    __shared__ int s_f[MP_NT];
    __shared__ ACC s_v[MP_NT];

    const int tid = threadIdx.x;
    const int t = blockIdx.x;
    const int2 c0 = coords[t];
    const int2 c1 = coords[t + 1];
    const int r0 = c0.x, k0 = c0.y;
    const int nrows = c1.x - r0, nnzt = c1.y - k0;
    for (int i = tid; i < nrows; i += MP_NT) s_end[i] = ntload(row_ptr + r0 + 1 + i);
    for (int i = tid; i < nnzt; i += MP_NT) {
        s_col[i] = ntload(col + k0 + i);
        s_val[i] = (ACC)vget(val + k0 + i);
    }
    __syncthreads();

    const int g = tid / KP, lane = tid % KP;
    const bool act = lane < kc;
    const int items = nrows + nnzt;
    const int d = min(g * IPG, items);
    const int de = min(d + IPG, items);
    const int is = merge_split(s_end, nrows, nnzt, k0, d);
    const int ie = merge_split(s_end, nrows, nnzt, k0, de);
    const int js = d - is, je = de - ie;

    ACC acc = 0;
    int i = is;
    int frow = -1;
    ACC fval = 0;
    for (int jb = js; jb < je; jb += U) {
        X xv[U];
        ACC av[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int jj = jb + u;
            xv[u] = 0;
            av[u] = 0;
            if (jj < je) {
                const int c = s_col[jj];
                av[u] = s_val[jj];
                const X* rowp = c >= 0 ? xr + (int64_t)c * ldr : xh + (int64_t)(~c) * kc;
                if (act) xv[u] = rowp[lane];
            }
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int jj = jb + u;
            if (jj < je) {
                while (i < ie && s_end[i] <= k0 + jj) {
                    if (frow < 0) {
                        frow = i;
                        fval = acc;
                    } else if (act) {
                        ntstore(mm_yptr(y, ldy, row_major, (int64_t)r0 + i, lane), (X)acc);
                    }
                    acc = 0;
                    ++i;
                }
                acc += av[u] * (ACC)xv[u];
            }
        }
    }
    for (; i < ie; ++i) {
        if (frow < 0) {
            frow = i;
            fval = acc;
        } else if (act) {
            ntstore(mm_yptr(y, ldy, row_major, (int64_t)r0 + i, lane), (X)acc);
        }
        acc = 0;
    }

    // segmented inclusive scan of (finished a row, open value) over the groups, per lane
    int f = frow >= 0;
    ACC v = acc;
    s_f[tid] = f;
    s_v[tid] = v;
    __syncthreads();
    for (int o = 1; o < NG; o <<= 1) {
        int fo = 0;
        ACC vo = 0;
        const bool has = g >= o;
        if (has) {
            fo = s_f[tid - o * KP];
            vo = s_v[tid - o * KP];
        }
        __syncthreads();
        if (has) {
            seg_combine(fo, vo, f, v);
            f = fo;
            v = vo;
            s_f[tid] = f;
            s_v[tid] = v;
        }
        __syncthreads();
    }
    const ACC cin = g > 0 ? s_v[tid - KP] : (ACC)0;
    if (frow >= 0 && act)
        ntstore(mm_yptr(y, ldy, row_major, (int64_t)r0 + frow, lane), (X)(cin + fval));
    if (g == NG - 1) {
        if (act) carry_val[(int64_t)t * kc + lane] = (double)v;
        if (lane == 0) carry_row[t] = c1.x;  // m when nothing is left open
    }
}

// Adds each tile's open values into Y in FP64: one thread per run of tiles that left the same row
// open, and column (carry_run_sum: fixed order, deterministic).
template <typename X>
__global__ void k_spmm_fixup(const int32_t* __restrict__ carry_row,
                             const double* __restrict__ carry_val, int32_t tiles, int32_t kc,
                             X* __restrict__ y, int64_t ldy, int row_major, int32_t m) {
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (int64_t)tiles * kc) return;
    const int t = (int)(e / kc), c = (int)(e - (int64_t)t * kc);
    const int r = carry_row[t];
    if (r >= m) return;
    if (t > 0 && carry_row[t - 1] == r) return;
    const double acc = carry_run_sum(carry_row, tiles, t, r,
                                     [&](int u) { return carry_val[(int64_t)u * kc + c]; });
    X* p = mm_yptr(y, ldy, row_major, (int64_t)r, c);
    *p = (X)(acc + (double)*p);
}

template <typename V, typename X, typename ACC>
static hipError_t launch_spmm_merge(int kp, dim3 grid, hipStream_t s, const spx_matrix_s* A,
                                    const V* val, const X* xr, int64_t ldr, const X* xh,
                                    int32_t kc, X* y, int64_t ldy, int row_major,
                                    const int2* coords, int32_t* crow, double* cval) {
#define MM_CASE(K)                                                                              \
    case K:                                                                                     \
        SPX_LAUNCH("spmm_merge", (k_spmm_merge<V, X, ACC, K>), grid, dim3(MP_NT), 0, s,         \
                   A->row_ptr, A->col, val, xr, ldr, xh, kc, y, ldy, row_major, coords, crow, \
                   cval);                                                                       \
        break;
    switch (kp) {
        MM_CASE(1)
        MM_CASE(2)
        MM_CASE(4)
        MM_CASE(8)
        MM_CASE(16)
        MM_CASE(32)
        MM_CASE(64)
        default: return hipErrorInvalidValue;
    }
#undef MM_CASE
    return hipGetLastError();
}

template <typename V, typename X, typename ACC>
static hipError_t spmm_t(const spx_matrix_s* A, const SpmmPlan& P, const V* val, int32_t k,
                         const X* x, int64_t ldx, X* y, int64_t ldy, int row_major,
                         hipStream_t s) {
    for (int32_t c0 = 0; c0 < k; c0 += MM_KMAX) {
        const int32_t kc = min((int32_t)MM_KMAX, k - c0);
        int kp = 1;
        while (kp < kc) kp <<= 1;
        if (kc == 1) {
            // one column held contiguously in X and Y: the single-vector merge-path product on
            // the plan's tiles and scratch (its LDS-staged products keep more gathers in flight
            // than a one-lane group walk, and nothing needs staging)
            const X* x1 = row_major ? (ldx == 1 ? x + c0 : nullptr) : x + (int64_t)c0 * ldx;
            X* y1 = row_major ? (ldy == 1 ? y + c0 : nullptr) : y + (int64_t)c0 * ldy;
            if (x1 && y1) {
                const hipError_t e = spmv_merge_on_plan(A, P, x1, y1, s);
                if (e != hipSuccess) return e;
                continue;
            }
        }
        const X* xr;
        int64_t ldr;
        if (row_major) {
            xr = x + c0;
            ldr = ldx;
        } else {
            if (A->n > 0)
                SPX_LAUNCH("spmm_stage", k_spmm_stage<X>,
                           dim3((unsigned)spx_div_up(A->n, MM_STAGE_ROWS)), dim3(256), 0, s,
                           x + (int64_t)c0 * ldx, ldx, A->n, kc, (X*)P.z);
            xr = (const X*)P.z;
            ldr = kc;
        }
        if (A->nhot > 0)
            SPX_LAUNCH("spmm_hot", k_spmm_hot<X>,
                       dim3((unsigned)spx_div_up((int64_t)A->nhot * kc, 256)), dim3(256), 0, s,
                       A->hot_cols, A->nhot, xr, ldr, kc, (X*)P.h);
        // results are produced row-major (kc lanes write one contiguous run per row); a
        // column-major Y receives them through the scratch W and an LDS-tiled transpose
        X* yc = row_major ? y + c0 : (X*)P.w;
        const int64_t ldyc = row_major ? ldy : kc;
        if (P.tiles > 0) {
            hipError_t e = launch_spmm_merge<V, X, ACC>(kp, dim3(P.tiles), s, A, val, xr, ldr,
                                                        (const X*)P.h, kc, yc, ldyc, 1,
                                                        P.coords, P.carry_row, P.carry_val);
            if (e != hipSuccess) return e;
            SPX_LAUNCH("spmm_fixup", k_spmm_fixup<X>,
                       dim3((unsigned)spx_div_up((int64_t)P.tiles * kc, 256)), dim3(256), 0, s,
                       P.carry_row, P.carry_val, P.tiles, kc, yc, ldyc, 1, A->m);
        }
        if (!row_major)
            SPX_LAUNCH("spmm_unstage", k_spmm_unstage<X>,
                       dim3((unsigned)spx_div_up(A->m, MM_STAGE_ROWS)), dim3(256), 0, s,
                       (const X*)P.w, A->m, kc, y + (int64_t)c0 * ldy, ldy);
    }
    return hipGetLastError();
}

int32_t spmm_chunk_cols(int32_t k) { return k < MM_KMAX ? k : MM_KMAX; }

hipError_t spmm_crs(const spx_matrix_s* A, const SpmmPlan& P, int32_t k, const void* x,
                    int64_t ldx, void* y, int64_t ldy, int row_major, hipStream_t s) {
    switch (A->value_type) {
        case SPX_F64:
            return spmm_t<double, double, double>(A, P, A->val, k, (const double*)x, ldx,
                                                  (double*)y, ldy, row_major, s);
        case SPX_F32:
            return spmm_t<float, float, float>(A, P, (const float*)A->val_lp, k,
                                               (const float*)x, ldx, (float*)y, ldy, row_major,
                                               s);
        default:
            return spmm_t<uint16_t, float, float>(A, P, (const uint16_t*)A->val_lp, k,
                                                  (const float*)x, ldx, (float*)y, ldy,
                                                  row_major, s);
    }
}
