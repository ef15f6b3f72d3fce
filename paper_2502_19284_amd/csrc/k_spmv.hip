// k_spmv.hip -- y = A x for the compressed-sparse-block formats CSB and CSBH (gfx950, FP64
// values, int32 indices).  The CRS kernels are in k_spmv_crs.hip.
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
    int b = 0;  // block of this thread's current entry (bp[0] <= kb)
    for (int base = kb; base < ke; base += CB_NT * CB_IPT) {
        uint32_t p[CB_IPT];
        double v[CB_IPT];
#pragma unroll
        for (int q = 0; q < CB_IPT; ++q) {
            const int kk = base + q * CB_NT + tid;
            p[q] = kk < ke ? ntload(packed + kk) : 0u;
            v[q] = kk < ke ? ntload(val + kk) : 0.0;
        }
        double xv[CB_IPT];
#pragma unroll
        for (int q = 0; q < CB_IPT; ++q) {
            const int kk = base + q * CB_NT + tid;
            xv[q] = 0.0;
            if (kk < ke) {
                b = csb_block_of(bp, b, nbc, kk);
                xv[q] = x[(b << k) + (int)(p[q] & lmask)];
            }
        }
#pragma unroll
        for (int q = 0; q < CB_IPT; ++q) {
            const int kk = base + q * CB_NT + tid;
            if (kk < ke) atomicAdd(&s_y[p[q] >> 16], v[q] * xv[q]);
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

// Split block row S.x: y = sum of its S.z partial slices (slots S.y ..), added in slot order.
// Workgroup = (split row, chunk of 256 rows); each thread keeps 8 slot loads in flight.
#define CB_RED_NT 256
__device__ __forceinline__ void csb_reduce_body(const int4* __restrict__ split,
                                                const double* __restrict__ partials,
                                                double* __restrict__ y, int k, int32_t m) {
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
    y[row0 + i] = acc;
}

__global__ __launch_bounds__(CB_RED_NT) void k_spmv_csbh_reduce(const int4* __restrict__ split,
                                                               const double* __restrict__ partials,
                                                               double* __restrict__ y, int k,
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
        SPX_LAUNCH("spmv_csbh_reduce", k_spmv_csbh_reduce,
                   dim3(A->cb_nsplit * (((1 << A->log2_beta) + CB_RED_NT - 1) / CB_RED_NT)),
                   dim3(CB_RED_NT), 0, s, A->cb_split,
                           A->cb_partials, y, A->log2_beta, A->m);
    return hipGetLastError();
}

// ================================================================== CSBR (Section 3.1 blocks over
// ranked rows and columns)
//
// x_r[i] = x[order[i]]: the ranked copy of x that the product reads.
__global__ void k_csbr_xrank(const int32_t* __restrict__ order, int32_t nr,
                             const double* __restrict__ x, double* __restrict__ xr) {
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
// slot, reduced in slot order afterwards.
__global__ __launch_bounds__(CR_NT) void k_spmv_csbr(const int32_t* __restrict__ blk_ptr,
                                                     const uint32_t* __restrict__ packed,
                                                     const double* __restrict__ val,
                                                     const double* __restrict__ xr,
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
    for (int base = k0; base < k1; base += CR_NT * CR_IPT) {
        uint32_t p[CR_IPT];
        double v[CR_IPT];
#pragma unroll
        for (int q = 0; q < CR_IPT; ++q) {
            const int k = base + q * CR_NT + tid;
            p[q] = k < k1 ? ntload(packed + k) : 0u;
            v[q] = k < k1 ? ntload(val + k) : 0.0;
        }
        double xv[CR_IPT];
#pragma unroll
        for (int q = 0; q < CR_IPT; ++q) {
            const int k = base + q * CR_NT + tid;
            while (k >= next) {  // entries ascend per thread: walk the segments forward
                ++sg;
                next = sg + 1 < nseg ? seg[sg + 1] : INT32_MAX;
            }
            xv[q] = k < k1 ? xr[((int64_t)sg << CR_RB) + (p[q] >> CR_PB)] : 0.0;
        }
#pragma unroll
        for (int q = 0; q < CR_IPT; ++q) {
            const int k = base + q * CR_NT + tid;
            if (k < k1) atomicAdd(&s_y[p[q] & lmask], v[q] * xv[q]);
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

// Raises the product kernel's dynamic LDS limit on the current device (called at conversion, so
// that products, which may be captured in a graph, make no attribute calls).
hipError_t csbr_prepare_kernel() {
    if (kCsbrLds <= 64 * 1024) return hipSuccess;
    return hipFuncSetAttribute((const void*)k_spmv_csbr,
                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)kCsbrLds);
}

// y[r] = y_r[row_rank[r]]; rows without entries (rank >= nrows) get 0.
__global__ void k_csbr_yperm(const int32_t* __restrict__ row_rank, int32_t m, int32_t nrows,
                             const double* __restrict__ yr, double* __restrict__ y) {
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= m) return;
    const int32_t rr = ntload(row_rank + r);
    ntstore(y + r, rr < nrows ? yr[rr] : 0.0);
}

hipError_t spmv_csbr(const spx_matrix_s* A, const double* x, double* y, hipStream_t s) {
    constexpr size_t lds = kCsbrLds;
    if (A->cr_nranked > 0)
        SPX_LAUNCH("csbr_xrank", k_csbr_xrank, dim3(spx_div_up(A->cr_nranked, 256)), dim3(256), 0,
                   s, A->cr_order, A->cr_nranked, x, A->cr_xr);
    if (A->cb_nunits > 0) {
        SPX_LAUNCH("spmv_csbr", k_spmv_csbr, dim3(A->cb_nunits), dim3(CR_NT), lds, s, A->blk_ptr,
                   A->packed, A->val, A->cr_xr, A->cr_yr, A->cb_partials, A->cb_units,
                   (int32_t)A->nbc, A->cr_nrows);
    }
    if (A->cb_nsplit > 0)
        SPX_LAUNCH("spmv_csbr_reduce", k_spmv_csbr_reduce,
                   dim3(A->cb_nsplit * (((1 << CR_PB) + CB_RED_NT - 1) / CB_RED_NT)),
                   dim3(CB_RED_NT), 0, s, A->cb_split, A->cb_partials, A->cr_yr, CR_PB,
                   A->cr_nrows);
    if (A->m > 0)
        SPX_LAUNCH("csbr_yperm", k_csbr_yperm, dim3(spx_div_up(A->m, 256)), dim3(256), 0, s,
                   A->cr_row_rank, A->m, A->cr_nrows, A->cr_yr, y);
    return hipGetLastError();
}
