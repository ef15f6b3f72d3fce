// k_spmv.hip -- y = A x for the compressed-sparse-block formats CSB, CSBH (FP64 values) and
// CSBR (FP64, FP32 or bfloat16 values), int32 indices, gfx950.  The CRS kernels are in
// k_spmv_crs.hip.  Matrix streams are read with non-temporal loads (ntload, dev_values.h), so
// that they do not displace x from L2.
#include "dev_common.h"
#include "dev_values.h"
#include "spx_internal.h"

// ================================================================== CSBH (Sections 3.1, 4.1)
//
// Work unit u = entries [k0, k1) of block row br (at most the unit size).  The workgroup keeps
// the block row's beta-entry slice of y in LDS and adds every product into it (LDS float atomics;
// the Hilbert order keeps consecutive entries of a block in nearby rows and columns).  The
// workgroup reads its entries in storage order, CB_NT consecutive entries per wave-row (loads of
// whole lines), CB_IPT rows in flight per thread; a thread's entries ascend, so it keeps the block
// of its last entry and moves forward: a few steps by walking the block pointers (staged in LDS
// when they fit), a longer move by binary search.  A unit that covers its whole block row writes
// the slice to y; otherwise it writes a partial slice to scratch and k_spmv_csbh_reduce adds the
// partial slices of the block row in unit order.

// Last block b >= b_from with bp[b] <= k (bp non-decreasing, bp[b_from] <= k, bp[nb] > k).
__device__ __forceinline__ int csb_block_of(const int32_t* __restrict__ bp, int b_from, int nb,
                                            int k) {
#pragma unroll
    for (int step = 0; step < 4; ++step) {
        if (b_from + 1 >= nb || bp[b_from + 1] > k) return b_from;
        ++b_from;
    }
    int lo = b_from, hi = nb - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (bp[mid] <= k) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

template <typename V, typename X>
__global__ __launch_bounds__(CB_NT) void k_spmv_csbh(const int32_t* __restrict__ blk_ptr,
                                                     const uint32_t* __restrict__ packed,
                                                     const V* __restrict__ val,
                                                     const X* __restrict__ x,
                                                     X* __restrict__ y,
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
    using T = decltype(vget(val));  // arithmetic type of a product
    int b = 0;  // block of this thread's current entry (bp[0] <= kb)
    for (int base = kb; base < ke; base += CB_NT * CB_IPT) {
        // matrix loads issued unconditionally (entries past ke read entry ke - 1 again and are
        // dropped), so none waits inside a branch
        int kc[CB_IPT];
#pragma unroll
        for (int q = 0; q < CB_IPT; ++q) kc[q] = min(base + q * CB_NT + tid, ke - 1);
        uint32_t p[CB_IPT];
        V raw[CB_IPT];
#pragma unroll
        for (int q = 0; q < CB_IPT; ++q) {
            p[q] = ntload(packed + kc[q]);
            raw[q] = ntload(val + kc[q]);
        }
        T xv[CB_IPT];
#pragma unroll
        for (int q = 0; q < CB_IPT; ++q) {
            xv[q] = (T)0;
            if (base + q * CB_NT + tid < ke) {
                b = csb_block_of(bp, b, nbc, kc[q]);
                xv[q] = (T)x[(b << k) + (int)(p[q] & lmask)];
            }
        }
#pragma unroll
        for (int q = 0; q < CB_IPT; ++q) {
            if (base + q * CB_NT + tid < ke)
                atomicAdd(&s_y[p[q] >> 16], (double)(vdec(raw[q]) * xv[q]));
        }
    }
    __syncthreads();
    const int row0 = br << k;
    const int rows = min(beta, m - row0);
    if (slot < 0) {
        for (int i = tid; i < rows; i += CB_NT) ntstore(y + row0 + i, (X)s_y[i]);
    } else {
        double* dst = partials + (int64_t)slot * beta;
        for (int i = tid; i < rows; i += CB_NT) dst[i] = s_y[i];
    }
}

// Split block row S.x: y = sum of its S.z partial slices (slots S.y ..), added in slot order.
// Workgroup = (split row, chunk of 256 rows); each thread keeps 8 slot loads in flight.
#define CB_RED_NT 256
template <typename X>
__device__ __forceinline__ void csb_reduce_body(const int4* __restrict__ split,
                                                const double* __restrict__ partials,
                                                X* __restrict__ y, int k, int32_t m) {
    const int beta = 1 << k;
    const int chunks = (beta + CB_RED_NT - 1) / CB_RED_NT;
    const int4 S = split[blockIdx.x / chunks];
    const int i = (blockIdx.x % chunks) * CB_RED_NT + threadIdx.x;
    const int row0 = S.x << k;
    const int rows = min(beta, m - row0);
    if (i >= rows) return;
    const double* p = partials + (int64_t)S.y * beta + i;
    double acc = 0.0;
    int q = 0;
    for (; q + 8 <= S.z; q += 8) {
        double t[8];
#pragma unroll
        for (int u = 0; u < 8; ++u) t[u] = p[(int64_t)(q + u) * beta];
#pragma unroll
        for (int u = 0; u < 8; ++u) acc = acc + t[u];
    }
    for (; q < S.z; ++q) acc = acc + p[(int64_t)q * beta];
    y[row0 + i] = (X)acc;
}

template <typename X>
__global__ __launch_bounds__(CB_RED_NT) void k_spmv_csbh_reduce(const int4* __restrict__ split,
                                                               const double* __restrict__ partials,
                                                               X* __restrict__ y, int k,
                                                               int32_t m) {
    csb_reduce_body(split, partials, y, k, m);
}

// the same reduction for CSBR panels (a kernel of its own, so profiles tell the formats apart)
__global__ __launch_bounds__(CB_RED_NT) void k_spmv_csbr_reduce(const int4* __restrict__ split,
                                                               const double* __restrict__ partials,
                                                               double* __restrict__ y, int k,
                                                               int32_t m) {
    csb_reduce_body(split, partials, y, k, m);
}

template <typename V, typename X>
static hipError_t csbh_run(const spx_matrix_s* A, const V* val, const X* x, X* y,
                           hipStream_t s) {
    if (A->cb_nunits <= 0) return hipSuccess;
    const int beta = 1 << A->log2_beta;
    const int stage_bp = (A->nbc + 1 <= CB_BP_STAGE_MAX) ? 1 : 0;
    const size_t lds = (size_t)beta * sizeof(double) + (stage_bp ? (size_t)(A->nbc + 1) * 4 : 0);
    if (lds > 64 * 1024) {
        hipError_t e = hipFuncSetAttribute((const void*)k_spmv_csbh<V, X>,
                                           hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
        if (e != hipSuccess) return e;
    }
    SPX_LAUNCH("spmv_csbh", (k_spmv_csbh<V, X>), dim3(A->cb_nunits), dim3(CB_NT), lds, s,
               A->blk_ptr, A->packed, val, x, y, A->cb_partials, A->cb_units, A->log2_beta,
               (int32_t)A->nbc, A->m, stage_bp);
    if (A->cb_nsplit > 0)
        SPX_LAUNCH("spmv_csbh_reduce", k_spmv_csbh_reduce<X>,
                   dim3(A->cb_nsplit * (((1 << A->log2_beta) + CB_RED_NT - 1) / CB_RED_NT)),
                   dim3(CB_RED_NT), 0, s, A->cb_split, A->cb_partials, y, A->log2_beta, A->m);
    return hipGetLastError();
}

hipError_t spmv_csbh(const spx_matrix_s* A, const double* x, double* y, hipStream_t s) {
    return csbh_run<double, double>(A, A->val, x, y, s);
}

hipError_t spmv_csbh_f32(const spx_matrix_s* A, const float* x, float* y, hipStream_t s) {
    if (A->value_type == SPX_F32)
        return csbh_run<float, float>(A, (const float*)A->val_lp, x, y, s);
    return csbh_run<uint16_t, float>(A, (const uint16_t*)A->val_lp, x, y, s);
}

// ================================================================== CSBR (Section 3.1 blocks over
// ranked rows and columns)
//
// x_r[i] = x[order[i]]: the ranked copy of x that the product reads (FP64, or FP32 for the
// reduced-precision forms).
template <typename X>
__global__ void k_csbr_xrank(const int32_t* __restrict__ order, int32_t nr,
                             const X* __restrict__ x, X* __restrict__ xr) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < nr) xr[i] = x[order[i]];
}

// Work unit u = entries [k0, k1) of panel p (2^CR_PB row ranks).  The workgroup keeps the panel's
// slice of y_r (y in row-rank order) in LDS.  Entries are read in storage order, CR_NT
// consecutive entries per wave-row, so the lanes of a wave hold ascending column ranks: their x_r
// loads fall on few cache lines, and the lines of the most frequent columns stay in L2 for every
// panel.  An entry's column rank is its block's segment (found from the panel's block starts)
// times 2^CR_RB plus the packed rank field.  Products are added into the slice with LDS float
// atomics; a unit covering its whole panel writes the slice to y_r, otherwise to its partial
// slot, reduced in slot order afterwards.  V / X: stored value and vector types (double /
// double, or float or bfloat16 bits / float); a product is formed in the value's arithmetic type
// (FP64, or FP32 for the reduced forms) and every sum is FP64 (the slice, the partial slices and
// their reduction).
template <typename V, typename X, int IPT, bool SERIAL>
__global__ __launch_bounds__(CR_NT) void k_spmv_csbr(const int32_t* __restrict__ blk_ptr,
                                                     const uint32_t* __restrict__ packed,
                                                     const V* __restrict__ val,
                                                     const X* __restrict__ xr,
                                                     double* __restrict__ yr,
                                                     double* __restrict__ partials,
                                                     const int4* __restrict__ units,
                                                     int32_t nseg, int32_t nrows) {
    extern __shared__ double s_dyn[];
    double* s_y = s_dyn;                                // 2^CR_PB doubles
    int32_t* s_seg = (int32_t*)(s_dyn + (1 << CR_PB));  // CR_SEG_LDS block starts
    const int tid = threadIdx.x;
    const int4 U = units[blockIdx.x];
    const int panel = U.x, k0 = U.y, k1 = U.z, slot = U.w;
    const int32_t* gseg = blk_ptr + (int64_t)panel * nseg;
    const bool lds_seg = nseg + 1 <= CR_SEG_LDS;
    for (int i = tid; i < (1 << CR_PB); i += CR_NT) s_y[i] = 0.0;
    if (lds_seg)
        for (int i = tid; i <= nseg; i += CR_NT) s_seg[i] = gseg[i];
    __syncthreads();
    const int32_t* seg = lds_seg ? s_seg : gseg;
    constexpr uint32_t lmask = (1u << CR_PB) - 1u;
    // segment of this thread's first entry: the last s with seg[s] <= k (seg[0] <= k0)
    int sg = 0;
    {
        const int kf = k0 + tid;
        int lo = 0, hi = nseg - 1;
        while (lo < hi) {
            const int mid = (lo + hi + 1) >> 1;
            if (seg[mid] <= kf) lo = mid;
            else hi = mid - 1;
        }
        sg = lo;
    }
    int next = sg + 1 < nseg ? seg[sg + 1] : INT32_MAX;
    using T = decltype(vget(val));  // arithmetic type of a product
    for (int base = k0; base < k1; base += CR_NT * IPT) {
        // the matrix loads of a round are issued before any is used, without branches: entries
        // past k1 read entry k1 - 1 again (base < k1) and their products are dropped
        int kc[IPT];
#pragma unroll
        for (int q = 0; q < IPT; ++q) kc[q] = min(base + q * CR_NT + tid, k1 - 1);
        uint32_t p[IPT];
        V raw[IPT];
#pragma unroll
        for (int q = 0; q < IPT; ++q) {
            p[q] = ntload(packed + kc[q]);
            raw[q] = ntload(val + kc[q]);
        }
        T xv[IPT];
        if constexpr (SERIAL) {
            // one x gather in flight per thread: each waits for the previous (the branch on the
            // entry's range orders them)
#pragma unroll
            for (int q = 0; q < IPT; ++q) {
                while (kc[q] >= next) {  // entries ascend per thread: walk the segments forward
                    ++sg;
                    next = sg + 1 < nseg ? seg[sg + 1] : INT32_MAX;
                }
                xv[q] = base + q * CR_NT + tid < k1
                            ? (T)xr[((int64_t)sg << CR_RB) + (p[q] >> CR_PB)]
                            : (T)0;
            }
        } else {
            // all the round's x gathers in flight together
            int sq[IPT];
#pragma unroll
            for (int q = 0; q < IPT; ++q) {
                while (kc[q] >= next) {
                    ++sg;
                    next = sg + 1 < nseg ? seg[sg + 1] : INT32_MAX;
                }
                sq[q] = sg;
            }
#pragma unroll
            for (int q = 0; q < IPT; ++q)
                xv[q] = (T)xr[((int64_t)sq[q] << CR_RB) + (p[q] >> CR_PB)];
        }
#pragma unroll
        for (int q = 0; q < IPT; ++q) {
            if (base + q * CR_NT + tid < k1)
                atomicAdd(&s_y[p[q] & lmask], (double)(vdec(raw[q]) * xv[q]));
        }
    }
    __syncthreads();
    const int row0 = panel << CR_PB;
    const int rows = min(1 << CR_PB, nrows - row0);
    if (slot < 0) {
        for (int i = tid; i < rows; i += CR_NT) yr[row0 + i] = s_y[i];
    } else {
        double* dst = partials + ((int64_t)slot << CR_PB);
        for (int i = tid; i < rows; i += CR_NT) dst[i] = s_y[i];
    }
}

static constexpr size_t kCsbrLds =
    ((size_t)1 << CR_PB) * sizeof(double) + CR_SEG_LDS * sizeof(int32_t);

// Raises the product kernels' dynamic LDS limit on the current device (called at conversion, so
// that products, which may be captured in a graph, make no attribute calls).
// Rounds per thread and gather order by value type, measured at R-MAT scale 24 (product kernel,
// ms, rounds of 2 / 4 / 8 entries, all gathers of a round together): FP64 0.89 / 0.86 / 0.84 and
// 0.79 with 4 entries and one gather at a time; FP32 0.82 / 0.61 / 0.56; bfloat16 0.71 / 0.53 /
// 0.48.  With FP64 x_r (16 values per line) more gathers in flight fetch more lines.
#ifndef CSBR_F64_IPT
#define CSBR_F64_IPT 4
#endif
#ifndef CSBR_F64_SERIAL
#define CSBR_F64_SERIAL true
#endif
#ifndef CSBR_LP_IPT
#define CSBR_LP_IPT 8
#endif
template <typename V>
struct CsbrShape {
    static constexpr int ipt = CSBR_LP_IPT;
    static constexpr bool serial = false;
};
template <>
struct CsbrShape<double> {
    static constexpr int ipt = CSBR_F64_IPT;
    static constexpr bool serial = CSBR_F64_SERIAL;
};
template <typename V, typename X>
static const void* csbr_kernel() {
    return (const void*)k_spmv_csbr<V, X, CsbrShape<V>::ipt, CsbrShape<V>::serial>;
}

template <typename V, typename X>
static hipError_t csbr_prepare_one() {
    return hipFuncSetAttribute(csbr_kernel<V, X>(), hipFuncAttributeMaxDynamicSharedMemorySize,
                               (int)kCsbrLds);
}

hipError_t csbr_prepare_kernel() {
    if (kCsbrLds <= 64 * 1024) return hipSuccess;
    hipError_t e = csbr_prepare_one<double, double>();
    if (e == hipSuccess) e = csbr_prepare_one<float, float>();
    if (e == hipSuccess) e = csbr_prepare_one<uint16_t, float>();
    return e;
}

// y[r] = y_r[row_rank[r]]; rows without entries (rank >= nrows) get 0.
template <typename X>
__global__ void k_csbr_yperm(const int32_t* __restrict__ row_rank, int32_t m, int32_t nrows,
                             const double* __restrict__ yr, X* __restrict__ y) {
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= m) return;
    const int32_t rr = ntload(row_rank + r);
    ntstore(y + r, (X)(rr < nrows ? yr[rr] : 0.0));
}

template <typename V, typename X>
static hipError_t csbr_run(const spx_matrix_s* A, const V* val, const X* x, X* y,
                           hipStream_t s) {
    constexpr size_t lds = kCsbrLds;
    X* xr = (X*)A->cr_xr;  // sized for FP64, so it holds either type
    if (A->cr_nranked > 0)
        SPX_LAUNCH("csbr_xrank", k_csbr_xrank<X>, dim3(spx_div_up(A->cr_nranked, 256)),
                   dim3(256), 0, s, A->cr_order, A->cr_nranked, x, xr);
    if (A->cb_nunits > 0)
        SPX_LAUNCH("spmv_csbr",
                   (k_spmv_csbr<V, X, CsbrShape<V>::ipt, CsbrShape<V>::serial>),
                   dim3(A->cb_nunits), dim3(CR_NT), lds, s,
                   A->blk_ptr, A->packed, val, (const X*)xr, A->cr_yr, A->cb_partials,
                   A->cb_units, (int32_t)A->nbc, A->cr_nrows);
    if (A->cb_nsplit > 0)
        SPX_LAUNCH("spmv_csbr_reduce", k_spmv_csbr_reduce,
                   dim3(A->cb_nsplit * (((1 << CR_PB) + CB_RED_NT - 1) / CB_RED_NT)),
                   dim3(CB_RED_NT), 0, s, A->cb_split, A->cb_partials, A->cr_yr, CR_PB,
                   A->cr_nrows);
    if (A->m > 0)
        SPX_LAUNCH("csbr_yperm", k_csbr_yperm<X>, dim3(spx_div_up(A->m, 256)), dim3(256), 0, s,
                   A->cr_row_rank, A->m, A->cr_nrows, A->cr_yr, y);
    return hipGetLastError();
}

hipError_t spmv_csbr(const spx_matrix_s* A, const double* x, double* y, hipStream_t s) {
    return csbr_run<double, double>(A, A->val, x, y, s);
}

hipError_t spmv_csbr_f32(const spx_matrix_s* A, const float* x, float* y, hipStream_t s) {
    if (A->value_type == SPX_F32)
        return csbr_run<float, float>(A, (const float*)A->val_lp, x, y, s);
    return csbr_run<uint16_t, float>(A, (const uint16_t*)A->val_lp, x, y, s);
}
