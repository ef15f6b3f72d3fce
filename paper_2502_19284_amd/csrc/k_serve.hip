// k_serve.hip -- batch packing for the serving loop (gfx950).
//
// A batch of k requests against one matrix is run as one product with k right-hand sides in the
// row-major layout: the k input vectors are interleaved into X (n x k), and the k result columns
// of Y (m x k) are written back to the requests' outputs with their epilogue
// y_c = alpha_c * (A x_c) + beta_c (alpha 1, beta 0 for a plain product; d and (1 - d) / n for a
// PageRank step).  Both moves go through an LDS tile so that reads and writes stay coalesced.
#include "dev_common.h"
#include "dev_values.h"
#include "spx_internal.h"

#define SV_ROWS 64
#define SV_KMAX 64

// X[j*k + c] = xs[c][j]
__global__ __launch_bounds__(256) void k_serve_gather(const float* const* __restrict__ xs, int k,
                                                      int n, float* __restrict__ X) {
    __shared__ float s[SV_ROWS * (SV_KMAX + 1)];
    const int64_t j0 = (int64_t)blockIdx.x * SV_ROWS;
    const int rows = (int)min((int64_t)SV_ROWS, (int64_t)n - j0);
    for (int e = threadIdx.x; e < SV_ROWS * k; e += 256) {
        const int c = e / SV_ROWS, r = e % SV_ROWS;
        if (r < rows) s[r * (SV_KMAX + 1) + c] = xs[c][j0 + r];
    }
    __syncthreads();
    for (int e = threadIdx.x; e < rows * k; e += 256) {
        const int r = e / k, c = e % k;
        X[(j0 + r) * k + c] = s[r * (SV_KMAX + 1) + c];
    }
}

// ys[c][i] = alpha[c] * Y[i*k + c] + beta[c], one rounding
__global__ __launch_bounds__(256) void k_serve_scatter(const float* __restrict__ Y, int k, int m,
                                                       float* const* __restrict__ ys,
                                                       const float* __restrict__ alpha,
                                                       const float* __restrict__ beta) {
    __shared__ float s[SV_ROWS * (SV_KMAX + 1)];
    const int64_t i0 = (int64_t)blockIdx.x * SV_ROWS;
    const int rows = (int)min((int64_t)SV_ROWS, (int64_t)m - i0);
    for (int e = threadIdx.x; e < rows * k; e += 256) {
        const int r = e / k, c = e % k;
        s[r * (SV_KMAX + 1) + c] = Y[(i0 + r) * k + c];
    }
    __syncthreads();
    for (int e = threadIdx.x; e < SV_ROWS * k; e += 256) {
        const int c = e / SV_ROWS, r = e % SV_ROWS;
        if (r < rows) ys[c][i0 + r] = __fmaf_rn(alpha[c], s[r * (SV_KMAX + 1) + c], beta[c]);
    }
}

// y = alpha * y + beta in place (epilogue of a single-request launch)
__global__ void k_serve_axpb(float* __restrict__ y, int m, float alpha, float beta) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < m;
         i += (int64_t)gridDim.x * blockDim.x)
        y[i] = __fmaf_rn(alpha, y[i], beta);
}

hipError_t launch_serve_gather(const float* const* xs, int k, int n, float* X, hipStream_t s) {
    if (n <= 0 || k <= 0) return hipSuccess;
    if (k > SV_KMAX) return hipErrorInvalidValue;
    SPX_LAUNCH("serve_gather", k_serve_gather, dim3((unsigned)spx_div_up(n, SV_ROWS)), dim3(256),
               0, s, xs, k, n, X);
    return hipGetLastError();
}

hipError_t launch_serve_scatter(const float* Y, int k, int m, float* const* ys,
                                const float* alpha, const float* beta, hipStream_t s) {
    if (m <= 0 || k <= 0) return hipSuccess;
    if (k > SV_KMAX) return hipErrorInvalidValue;
    SPX_LAUNCH("serve_scatter", k_serve_scatter, dim3((unsigned)spx_div_up(m, SV_ROWS)),
               dim3(256), 0, s, Y, k, m, ys, alpha, beta);
    return hipGetLastError();
}

hipError_t launch_serve_axpb(float* y, int m, float alpha, float beta, hipStream_t s) {
    if (m <= 0) return hipSuccess;
    int64_t g = spx_div_up(m, 256);
    if (g > 4096) g = 4096;
    SPX_LAUNCH("serve_axpb", k_serve_axpb, dim3((unsigned)g), dim3(256), 0, s, y, m, alpha, beta);
    return hipGetLastError();
}
