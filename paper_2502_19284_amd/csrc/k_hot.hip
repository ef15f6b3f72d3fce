// k_hot.hip -- hot-column compaction of x for the CRS formats (gfx950).
//
// On power-law matrices a few columns take most of the x gathers, but they are spread over the
// whole of x, so each hot 8-byte value drags a 128-byte line into L2.  At conversion the most
// frequent columns (at most `hot_max`) get dense ranks; their entries store ~rank (a negative
// index) instead of the column.  Each product first gathers x_hot[h] = x[hot_cols[h]], a compact
// array whose lines are all hot, and the kernels read x_hot[~c] for negative c.  Results are
// unchanged: only the address a value is read from moves.
//
// The set is a bitmap over columns plus a prefix count per 64-bit word, packed into one 16-byte
// word per 64 columns (4 MB for 2^24 columns, L2-resident), so rank(c) = prefix + popcount(bits
// below c) costs one cached load.
#include "dev_scan.h"
#include "spx_internal.h"

// Sampled column frequencies.  Sample s is the column of sorted key (s / HOT_RUN) * HOT_RUN *
// stride + s % HOT_RUN (stride 1: key s), i.e. runs of HOT_RUN consecutive keys, one run per
// HOT_RUN * stride keys.  The samples are sorted by column (radix sort) and each wave adds the
// length of every run of equal columns among its 64 positions with one atomic, so a hot column
// costs one atomic per wave that holds it instead of one per sample.
__global__ void k_hot_sample(const uint64_t* __restrict__ keys, int64_t stride, int64_t ns,
                             uint64_t cmask, uint64_t* __restrict__ S) {
    for (int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; s < ns;
         s += (int64_t)gridDim.x * blockDim.x) {
        const int64_t i = stride == 1 ? s : (s / HOT_RUN) * HOT_RUN * stride + s % HOT_RUN;
        S[s] = keys[i] & cmask;
    }
}

hipError_t launch_hot_sample(const uint64_t* keys, int64_t stride, int64_t ns, uint64_t cmask,
                             uint64_t* S, hipStream_t s) {
    if (ns <= 0) return hipSuccess;
    const int64_t g = spx_div_up(ns, 256) < 8192 ? spx_div_up(ns, 256) : 8192;
    SPX_LAUNCH("hot_sample", k_hot_sample, dim3((unsigned)g), dim3(256), 0, s, keys, stride, ns,
               cmask, S);
    return hipGetLastError();
}

__global__ __launch_bounds__(256) void k_hot_count_sorted(const uint64_t* __restrict__ S,
                                                          int64_t ns,
                                                          uint32_t* __restrict__ freq) {
    const int lane = __lane_id();
    const int64_t wave = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / SPX_WAVE;
    const int64_t nwaves = (int64_t)gridDim.x * blockDim.x / SPX_WAVE;
    for (int64_t c0 = wave * SPX_WAVE; c0 < ns; c0 += nwaves * SPX_WAVE) {
        const int64_t p = c0 + lane;
        const bool valid = p < ns;
        const uint64_t c = valid ? S[p] : 0ull;
        const bool start = valid && (lane == 0 || S[p - 1] != c);
        const uint64_t starts = __ballot(start);
        const int nvalid = (int)__popcll(__ballot(valid));  // valid lanes form a prefix
        if (start) {
            const uint64_t above = lane == SPX_WAVE - 1 ? 0ull : starts >> (lane + 1);
            int next = above ? lane + 1 + __builtin_ctzll(above) : SPX_WAVE;
            if (next > nvalid) next = nvalid;
            atomicAdd(&freq[c], (uint32_t)(next - lane));
        }
    }
}

hipError_t launch_hot_count_sorted(const uint64_t* S, int64_t ns, uint32_t* freq, hipStream_t s) {
    if (ns <= 0) return hipSuccess;
    const int64_t g = spx_div_up(ns, 256) < 8192 ? spx_div_up(ns, 256) : 8192;
    SPX_LAUNCH("hot_count", k_hot_count_sorted, dim3((unsigned)g), dim3(256), 0, s, S, ns, freq);
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

// bitmap word w covers columns [64w, 64w+64); cnt[w] = its population
__global__ void k_hot_bits(const uint32_t* __restrict__ freq, int64_t n, uint32_t tau,
                           uint64_t* __restrict__ bits, uint32_t* __restrict__ cnt,
                           int64_t nwords) {
    const int64_t w = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (w >= nwords) return;
    uint64_t b = 0;
    for (int j = 0; j < 64; ++j) {
        const int64_t c = w * 64 + j;
        if (c < n && freq[c] >= tau) b |= 1ull << j;
    }
    bits[w] = b;
    cnt[w] = (uint32_t)__popcll(b);
}

struct LoadU32H {
    const uint32_t* p;
    __device__ uint32_t operator()(int64_t i) const { return p[i]; }
};
struct StoreExclH {
    uint32_t* p;
    __device__ void operator()(int64_t i, uint32_t incl, uint32_t item) const { p[i] = incl - item; }
};

__global__ void k_hot_list(const uint64_t* __restrict__ bits, const uint32_t* __restrict__ pre,
                           int64_t nwords, int32_t* __restrict__ hot_cols) {
    const int64_t w = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (w >= nwords) return;
    uint64_t b = bits[w];
    uint32_t r = pre[w];
    while (b) {
        const int j = __ffsll((unsigned long long)b) - 1;
        hot_cols[r++] = (int32_t)(w * 64 + j);
        b &= b - 1;
    }
}

// bits/pre for the columns with frequency >= tau (pre: exclusive prefix of word populations),
// hot_cols in ascending column order.  cnt must hold nwords entries and may alias pre.
hipError_t launch_hot_set(const uint32_t* freq, int64_t n, uint32_t tau, uint64_t* bits,
                          uint32_t* pre, int32_t* hot_cols, uint32_t* tile_sums, hipStream_t s) {
    const int64_t nwords = (n + 63) / 64;
    SPX_LAUNCH("hot_bits", k_hot_bits, dim3(spx_div_up(nwords, 256)), dim3(256), 0, s, freq, n,
               tau, bits, pre, nwords);
    hipError_t e = scan_phase12<uint32_t, OpSum<uint32_t>>(LoadU32H{pre}, nwords, tile_sums,
                                                           (uint32_t*)nullptr, s);
    if (e != hipSuccess) return e;
    e = scan_phase3<uint32_t, OpSum<uint32_t>>(LoadU32H{pre}, StoreExclH{pre}, nwords, tile_sums,
                                               s);
    if (e != hipSuccess) return e;
    SPX_LAUNCH("hot_list", k_hot_list, dim3(spx_div_up(nwords, 256)), dim3(256), 0, s, bits, pre,
               nwords, hot_cols);
    return hipGetLastError();
}

__global__ void k_hot_pack(const uint64_t* __restrict__ bits, const uint32_t* __restrict__ pre,
                           int64_t nwords, uint4* __restrict__ words) {
    const int64_t w = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (w >= nwords) return;
    const uint64_t b = bits[w];
    words[w] = make_uint4((uint32_t)b, (uint32_t)(b >> 32), pre[w], 0u);
}

hipError_t launch_hot_pack(const uint64_t* bits, const uint32_t* pre, int64_t nwords,
                           uint4* words, hipStream_t s) {
    if (nwords <= 0) return hipSuccess;
    SPX_LAUNCH("hot_pack", k_hot_pack, dim3(spx_div_up(nwords, 256)), dim3(256), 0, s, bits, pre,
               nwords, words);
    return hipGetLastError();
}

// Histogram of the sampled column counts (the last bin collects every count >= bins-1), kept per
// workgroup in LDS and added once per bin.
__global__ __launch_bounds__(256) void k_hot_freq_hist(const uint32_t* __restrict__ freq,
                                                       int64_t n, uint32_t* __restrict__ hist) {
    __shared__ uint32_t h[HOT_HIST_BINS];
    for (int i = threadIdx.x; i < HOT_HIST_BINS; i += 256) h[i] = 0;
    __syncthreads();
    for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < n;
         c += (int64_t)gridDim.x * blockDim.x) {
        const uint32_t f = freq[c];
        atomicAdd(&h[f < HOT_HIST_BINS - 1 ? f : HOT_HIST_BINS - 1], 1u);
    }
    __syncthreads();
    for (int i = threadIdx.x; i < HOT_HIST_BINS; i += 256)
        if (h[i]) atomicAdd(&hist[i], h[i]);
}

hipError_t launch_hot_freq_hist(const uint32_t* freq, int64_t n, uint32_t* hist, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    int64_t g = spx_div_up(n, 256);
    if (g > 1024) g = 1024;
    SPX_LAUNCH("hot_freq_hist", k_hot_freq_hist, dim3((unsigned)g), dim3(256), 0, s, freq, n,
               hist);
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
