// k_hot.hip -- hot-column compaction of x for the CRS formats (gfx950).
//
// On power-law matrices a few columns take most of the x gathers, but they are spread over the
// whole of x, so each hot 8-byte value drags a 128-byte line into L2.  At conversion the most
// frequent columns (at most `hot_max`) get dense ranks; their entries store ~rank (a negative
// index) instead of the column.  Each product first gathers x_hot[h] = x[hot_cols[h]], a compact
// array whose lines are all hot, and the kernels read x_hot[~c] for negative c.  Results are
// unchanged: only the address a value is read from moves.
#include "dev_scan.h"
#include "spx_internal.h"

// sampled column frequencies: every `stride`-th stored entry
__global__ void k_hot_count(const int32_t* __restrict__ col, int64_t nnz, int64_t stride,
                            uint32_t* __restrict__ freq) {
    for (int64_t i = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) * stride; i < nnz;
         i += (int64_t)gridDim.x * blockDim.x * stride)
        atomicAdd(&freq[col[i]], 1u);
}

hipError_t launch_hot_count(const int32_t* col, int64_t nnz, int64_t stride, uint32_t* freq,
                            hipStream_t s) {
    if (nnz <= 0) return hipSuccess;
    int64_t samples = (nnz + stride - 1) / stride;
    int64_t g = (samples + 255) / 256;
    if (g > 8192) g = 8192;
    SPX_LAUNCH("hot_count", k_hot_count, dim3((unsigned)g), dim3(256), 0, s, col, nnz, stride,
               freq);
    return hipGetLastError();
}

struct LoadGe {
    const uint32_t* freq;
    uint32_t tau;
    __device__ uint32_t operator()(int64_t c) const { return freq[c] >= tau ? 1u : 0u; }
};

// number of columns with sampled frequency >= tau, written to *total
hipError_t launch_hot_count_ge(const uint32_t* freq, int64_t n, uint32_t tau, uint32_t* tile_sums,
                               uint32_t* total, hipStream_t s) {
    return scan_phase12<uint32_t, OpSum<uint32_t>>(LoadGe{freq, tau}, n, tile_sums, total, s);
}

struct StoreHot {
    int32_t* colmap;
    int32_t* hot_cols;
    __device__ void operator()(int64_t c, uint32_t incl, uint32_t item) const {
        if (item) {
            colmap[c] = (int32_t)(incl - 1);
            hot_cols[incl - 1] = (int32_t)c;
        } else {
            colmap[c] = -1;
        }
    }
};

// colmap[c] = dense rank of c among hot columns (ascending column order) or -1
hipError_t launch_hot_ranks(const uint32_t* freq, int64_t n, uint32_t tau,
                            const uint32_t* tile_sums, int32_t* colmap, int32_t* hot_cols,
                            hipStream_t s) {
    return scan_phase3<uint32_t, OpSum<uint32_t>>(LoadGe{freq, tau}, StoreHot{colmap, hot_cols},
                                                  n, tile_sums, s);
}

__global__ void k_hot_remap(int32_t* __restrict__ col, int64_t nnz,
                            const int32_t* __restrict__ colmap) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nnz;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int32_t c = col[i];
        const int32_t h = colmap[c];
        col[i] = h >= 0 ? ~h : c;
    }
}

hipError_t launch_hot_remap(int32_t* col, int64_t nnz, const int32_t* colmap, hipStream_t s) {
    if (nnz <= 0) return hipSuccess;
    int64_t g = (nnz + 255) / 256;
    if (g > 65536) g = 65536;
    SPX_LAUNCH("hot_remap", k_hot_remap, dim3((unsigned)g), dim3(256), 0, s, col, nnz, colmap);
    return hipGetLastError();
}

__global__ void k_hot_gather(const int32_t* __restrict__ hot_cols, int32_t nhot,
                             const double* __restrict__ x, double* __restrict__ x_hot) {
    const int h = blockIdx.x * blockDim.x + threadIdx.x;
    if (h < nhot) x_hot[h] = x[hot_cols[h]];
}

hipError_t launch_hot_gather(const int32_t* hot_cols, int32_t nhot, const double* x,
                             double* x_hot, hipStream_t s) {
    if (nhot <= 0) return hipSuccess;
    SPX_LAUNCH("hot_gather", k_hot_gather, dim3(spx_div_up(nhot, 256)), dim3(256), 0, s,
               hot_cols, nhot, x, x_hot);
    return hipGetLastError();
}

// col_ind as the caller knows it: hot entries mapped back to their columns
__global__ void k_hot_unmap(const int32_t* __restrict__ col, int64_t nnz,
                            const int32_t* __restrict__ hot_cols, int32_t* __restrict__ out) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nnz;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int32_t c = col[i];
        out[i] = c < 0 ? hot_cols[~c] : c;
    }
}

hipError_t launch_hot_unmap(const int32_t* col, int64_t nnz, const int32_t* hot_cols,
                            int32_t* out, hipStream_t s) {
    if (nnz <= 0) return hipSuccess;
    int64_t g = (nnz + 255) / 256;
    if (g > 65536) g = 65536;
    SPX_LAUNCH("hot_unmap", k_hot_unmap, dim3((unsigned)g), dim3(256), 0, s, col, nnz, hot_cols,
               out);
    return hipGetLastError();
}
