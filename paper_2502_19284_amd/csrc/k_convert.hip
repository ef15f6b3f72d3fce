// k_convert.hip -- triplet -> format conversion kernels (gfx950).
//
// The conversion follows the two steps of Section 5.1: (1) sort the entries into the order the
// format needs, (2) fill and compress the format's arrays.  Step 1 is a stable radix sort of a
// 64-bit key that carries each triplet's value along (MSD levels split the keys into segments of
// at most 4096, each finished in LDS); step 2 sums repeated coordinates in increasing triplet
// index and turns per-row (per-block) end marks into row_ptr (blk_ptr) with a max-scan.
#include "dev_curves.h"
#include "dev_scan.h"
#include "spx_internal.h"

// ------------------------------------------------------------------ small utilities

__global__ void k_fill_i32(int32_t* p, int64_t n, int32_t v) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

static unsigned grid_for(int64_t n, int nt, unsigned cap = 1u << 20) {
    int64_t g = (n + nt - 1) / nt;
    if (g < 1) g = 1;
    if (g > cap) g = cap;
    return (unsigned)g;
}

hipError_t launch_fill_i32(int32_t* p, int64_t n, int32_t v, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    SPX_LAUNCH("fill_i32", k_fill_i32, dim3(grid_for(n, 256)), dim3(256), 0, s, p, n, v);
    return hipGetLastError();
}

__global__ void k_init_readback(Readback* rb) {
    rb->err = 0;
    rb->pad = 0;
    rb->masks[0] = 0ull;
    rb->masks[1] = ~0ull;
    for (int i = 0; i < 4; ++i) rb->totals[i] = 0;
}

hipError_t launch_init_readback(Readback* rb, hipStream_t s) {
    SPX_LAUNCH("init_readback", k_init_readback, dim3(1), dim3(1), 0, s, rb);
    return hipGetLastError();
}

size_t scan_tile_count(int64_t n) { return n <= 0 ? 1 : (size_t)spx_div_up(n, SCAN_TILE); }

// ------------------------------------------------------------------ sort keys

template <typename KeyFn>
__device__ __forceinline__ void keys_body(const int32_t* __restrict__ row,
                                          const int32_t* __restrict__ col, int64_t E, int32_t m,
                                          int32_t n, uint64_t* __restrict__ keys, uint32_t* err,
                                          unsigned long long* masks, KeyFn fn) {
    unsigned long long orv = 0, andv = ~0ull;
    uint32_t bad = 0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < E;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int32_t r = row[i], c = col[i];
        const bool ok = (r >= 0) & (r < m) & (c >= 0) & (c < n);
        bad |= ok ? 0u : 1u;
        const uint64_t key = ok ? fn((uint32_t)r, (uint32_t)c) : 0ull;
        keys[i] = key;
        orv |= key;
        andv &= key;
    }
    // one atomic per workgroup (the grid is capped at KEYS_MAX_GRID workgroups)
    __shared__ unsigned long long s_or[4], s_and[4];
    __shared__ uint32_t s_bad[4];
    orv = wave_reduce<unsigned long long, OpOr<unsigned long long>>(orv);
    andv = wave_reduce<unsigned long long, OpAnd<unsigned long long>>(andv);
    const uint64_t anybad = __ballot(bad != 0);
    const int w = threadIdx.x / SPX_WAVE;
    if (__lane_id() == 0) {
        s_or[w] = orv;
        s_and[w] = andv;
        s_bad[w] = anybad ? 1u : 0u;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int i = 1; i < 4; ++i) {
            orv |= s_or[i];
            andv &= s_and[i];
        }
        atomicOr(&masks[0], orv);
        atomicAnd(&masks[1], andv);
        if (s_bad[0] | s_bad[1] | s_bad[2] | s_bad[3]) atomicOr(err, 1u);
    }
}

#define KEYS_MAX_GRID 2048

struct KeyCsr {
    int cbits;
    __device__ uint64_t operator()(uint32_t r, uint32_t c) const {
        return ((uint64_t)r << cbits) | (uint64_t)c;
    }
    // the key with its low order_bits() bits cleared, and their count (none here)
    __device__ uint64_t high_part(uint32_t r, uint32_t c) const { return (*this)(r, c); }
    __device__ int order_bits() const { return 0; }
};

template <bool HILBERT>
struct KeyCsb {
    int k;
    uint64_t nbc;
    __device__ uint64_t operator()(uint32_t r, uint32_t c) const {
        const uint32_t mask = (1u << k) - 1u;
        const uint64_t blk = (uint64_t)(r >> k) * nbc + (uint64_t)(c >> k);
        const uint32_t d = HILBERT ? hilbert_xy2d(k, c & mask, r & mask)
                                   : zmorton_xy2d(k, c & mask, r & mask);
        return (blk << (2 * k)) | (uint64_t)d;
    }
    // the key without the position inside the block (the curve index), and that index's width
    __device__ uint64_t high_part(uint32_t r, uint32_t c) const {
        return ((uint64_t)(r >> k) * nbc + (uint64_t)(c >> k)) << (2 * k);
    }
    __device__ int order_bits() const { return 2 * k; }
};

// BCOHC: (partition, Hilbert index of the block, row-wise position inside the block);
// BCOHCH: (partition, Hilbert index of (row, col) at level K2 + k), whose leading 2*K2 bits are
// the block's Hilbert index.
template <bool HIL>
struct KeyBcoh {
    const int32_t* part_of;
    int k, K2;
    __device__ uint64_t operator()(uint32_t r, uint32_t c) const {
        const int pshift = 2 * (K2 + k);
        const uint64_t p = (uint64_t)part_of[r];
        uint64_t d;
        if (HIL) {
            d = hilbert_xy2d64(K2 + k, c, r);
        } else {
            const uint32_t mask = (1u << k) - 1u;
            const uint64_t hb = hilbert_xy2d64(K2, c >> k, r >> k);
            d = (hb << (2 * k)) | ((uint64_t)(r & mask) << k) | (uint64_t)(c & mask);
        }
        return (pshift < 64 ? (p << pshift) : 0ull) | d;
    }
};

// CSBR: (panel, rank of the column, row inside the panel); the rank field is rbits wide, so the
// key shifted right by 32 (= CR_RB + CR_PB) is the block index panel * segments + segment
// (rr, c) = (row rank, column) of a triplet
struct KeyCsbr {
    const int32_t* rank_of;
    int rbits;
    __device__ uint64_t operator()(uint32_t rr, uint32_t c) const {
        const uint64_t panel = rr >> CR_PB;
        const uint64_t rank = (uint32_t)rank_of[c];
        return (panel << (rbits + CR_PB)) | (rank << CR_PB) |
               (uint64_t)(rr & ((1u << CR_PB) - 1u));
    }
};

template <typename KeyFn>
__global__ __launch_bounds__(256) void k_keys(const int32_t* row, const int32_t* col, int64_t E,
                                              int32_t m, int32_t n, uint64_t* keys, uint32_t* err,
                                              unsigned long long* masks, KeyFn fn) {
    keys_body(row, col, E, m, n, keys, err, masks, fn);
}

hipError_t launch_keys_csr(const int32_t* row, const int32_t* col, int64_t E, int32_t m,
                           int32_t n, int cbits, uint64_t* keys, uint32_t* err,
                           unsigned long long* masks, hipStream_t s) {
    SPX_LAUNCH("keys", (k_keys<KeyCsr>), dim3(grid_for(E, 256, KEYS_MAX_GRID)), dim3(256), 0, s, row,
                       col, E, m, n, keys, err, masks, KeyCsr{cbits});
    return hipGetLastError();
}

hipError_t launch_keys_csb(const int32_t* row, const int32_t* col, int64_t E, int32_t m,
                           int32_t n, int k, int64_t nbc, bool hilbert, uint64_t* keys,
                           uint32_t* err, unsigned long long* masks, hipStream_t s) {
    if (hilbert)
        SPX_LAUNCH("keys", (k_keys<KeyCsb<true>>), dim3(grid_for(E, 256, KEYS_MAX_GRID)),
                   dim3(256), 0, s, row, col, E, m, n, keys, err, masks,
                   KeyCsb<true>{k, (uint64_t)nbc});
    else
        SPX_LAUNCH("keys", (k_keys<KeyCsb<false>>), dim3(grid_for(E, 256, KEYS_MAX_GRID)),
                   dim3(256), 0, s, row, col, E, m, n, keys, err, masks,
                   KeyCsb<false>{k, (uint64_t)nbc});
    return hipGetLastError();
}

hipError_t launch_keys_csbr(const int32_t* rrank, const int32_t* col, int64_t E, int32_t m,
                            int32_t n, const int32_t* rank_of, int rbits, uint64_t* keys,
                            uint32_t* err, unsigned long long* masks, hipStream_t s) {
    SPX_LAUNCH("keys", (k_keys<KeyCsbr>), dim3(grid_for(E, 256, KEYS_MAX_GRID)), dim3(256), 0, s,
               rrank, col, E, m, n, keys, err, masks, KeyCsbr{rank_of, rbits});
    return hipGetLastError();
}

__global__ void k_rank_keys(const uint32_t* __restrict__ counts,
                            const uint32_t* __restrict__ first, const uint32_t* __restrict__ last,
                            int32_t n, int eb, int pbits, int ib, int ishift,
                            uint64_t* __restrict__ keys, uint64_t* __restrict__ cols) {
    const uint64_t cmax = (1ull << eb) - 1ull;
    for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < n;
         c += (int64_t)gridDim.x * blockDim.x) {
        const uint32_t k = counts[c];
        const uint64_t f = k && first ? first[c] : 0u, l = k && last ? last[c] : 0u;
        keys[c] = ((cmax - k) << (2 * pbits + ib)) | (f << (pbits + ib)) | (l << ib) |
                  ((uint64_t)c >> ishift);
        cols[c] = (uint64_t)c;
    }
}

hipError_t launch_rank_keys(const uint32_t* counts, const uint32_t* first, const uint32_t* last,
                            int32_t n, int eb, int pbits, int ib, int ishift, uint64_t* keys,
                            uint64_t* cols, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    SPX_LAUNCH("rank_keys", k_rank_keys, dim3(grid_for(n, 256)), dim3(256), 0, s, counts, first,
               last, n, eb, pbits, ib, ishift, keys, cols);
    return hipGetLastError();
}

// Sorted position i holds index cols[i]; its count is zero when the count field of the key is
// all ones, and the counted indices come first.
__global__ void k_rank_scatter(const uint64_t* __restrict__ sorted,
                               const uint64_t* __restrict__ cols, int32_t n, int eb, int fshift,
                               int32_t* __restrict__ order, int32_t* __restrict__ rank_of,
                               uint32_t* __restrict__ nranked) {
    const uint64_t cmax = (1ull << eb) - 1ull;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        const int32_t c = (int32_t)cols[i];
        rank_of[c] = (int32_t)i;
        if ((sorted[i] >> fshift) != cmax) {
            order[i] = c;
            const bool last = i + 1 == n || (sorted[i + 1] >> fshift) == cmax;
            if (last) *nranked = (uint32_t)(i + 1);
        }
    }
}

hipError_t launch_rank_scatter(const uint64_t* sorted, const uint64_t* cols, int32_t n, int eb,
                               int fshift, int32_t* order, int32_t* rank_of, uint32_t* nranked,
                               hipStream_t s) {
    if (n <= 0) return hipSuccess;
    SPX_LAUNCH("rank_scatter", k_rank_scatter, dim3(grid_for(n, 256)), dim3(256), 0, s, sorted,
               cols, n, eb, fshift, order, rank_of, nranked);
    return hipGetLastError();
}

hipError_t launch_keys_bcoh(const int32_t* row, const int32_t* col, int64_t E, int32_t m,
                            int32_t n, const int32_t* part_of, int k, int K2, bool hilbert,
                            uint64_t* keys, uint32_t* err, unsigned long long* masks,
                            hipStream_t s) {
    if (hilbert)
        SPX_LAUNCH("keys", (k_keys<KeyBcoh<true>>), dim3(grid_for(E, 256, KEYS_MAX_GRID)),
                   dim3(256), 0, s, row, col, E, m, n, keys, err, masks,
                   KeyBcoh<true>{part_of, k, K2});
    else
        SPX_LAUNCH("keys", (k_keys<KeyBcoh<false>>), dim3(grid_for(E, 256, KEYS_MAX_GRID)),
                   dim3(256), 0, s, row, col, E, m, n, keys, err, masks,
                   KeyBcoh<false>{part_of, k, K2});
    return hipGetLastError();
}

// ------------------------------------------------------------------ radix sort
//
// One pass per 8-bit digit (least significant first):
//   upsweep   : per-tile digit histogram, stored digit-major: hist[d * tiles + t]
//   scan      : exclusive scan of hist gives each (digit, tile) its first output slot
//   downsweep : each tile ranks its keys stably (original order within equal digits), reorders
//               them in LDS by digit, and writes each digit's run contiguously.
// Stable ranking: wave w of the tile takes the w-th of RSORT_NT / 64 equal slices of the tile in
// rounds of 64 consecutive keys; lanes holding the same digit find each other with 8 ballots (one per
// digit bit) and rank by lower-lane count; a per-wave LDS counter per digit carries the running
// count across rounds.  Wave offsets are then added per digit in wave order.
// Both kernels visit tiles in the XCD-contiguous order of rs_tile_of.

#define RSORT_WAVES (RSORT_NT / SPX_WAVE)
#define RSORT_ROUNDS (RSORT_TILE / RSORT_WAVES / SPX_WAVE)
static_assert(RSORT_NT >= 256 && RSORT_NT % SPX_WAVE == 0, "one thread per digit value");

size_t radix_hist_elems(int64_t E) { return (size_t)256 * spx_div_up(E, RSORT_TILE); }

// Tile of workgroup b.  Workgroups are dealt to the 8 XCDs in turn (b mod 8); here each XCD takes
// one contiguous range of tiles instead, so neighbouring tiles, which share histogram lines and
// the partial lines at the ends of their output runs, go through one L2.  A bijection onto
// [0, tiles) for any tile count.
__device__ __forceinline__ int64_t rs_tile_of(int64_t b, int64_t tiles) {
    const int64_t q = tiles >> 3, r = tiles & 7;
    const int64_t x = b & 7, i = b >> 3;
    return x * q + (x < r ? x : r) + i;
}

// Key sources of the counting and scatter passes: a key array, or keys built from triplets by a
// format's key function (0 for an index outside the matrix, which is reported separately).
struct KeyArr {
    const uint64_t* k;
    __device__ uint64_t operator()(int64_t i) const { return k[i]; }
};
template <typename KeyFn>
struct KeyFromTriplets {
    const int32_t* row;
    const int32_t* col;
    int32_t m, n;
    KeyFn fn;
    __device__ bool valid(int32_t r, int32_t c) const {
        return (r >= 0) & (r < m) & (c >= 0) & (c < n);
    }
    __device__ uint64_t operator()(int64_t i) const {
        const int32_t r = row[i], c = col[i];
        return valid(r, c) ? fn((uint32_t)r, (uint32_t)c) : 0ull;
    }
};

// Lanes of the wave whose 8-bit digit equals this lane's, among the valid lanes: for each bit,
// the lanes that differ from this lane are the bit's ballot xor this lane's bit spread over 32
// bits (0 or all ones); one OR per bit collects them.
__device__ __forceinline__ uint64_t wave_digit_peers(uint32_t d, bool valid) {
    uint32_t mb[RS_RADIX_BITS];
    uint64_t bal[RS_RADIX_BITS];
#pragma unroll
    for (int b = 0; b < RS_RADIX_BITS; ++b) {  // all ballots first: no wait on each one
        mb[b] = (uint32_t)__builtin_amdgcn_sbfe((int)d, b, 1);
        bal[b] = __ballot((int)mb[b] < 0);
    }
    uint32_t mlo = 0u, mhi = 0u;
#pragma unroll
    for (int b = 0; b < RS_RADIX_BITS; ++b) {
        // acc | (ballot ^ mb) in one three-input bit operation per half (truth table 0xF6 for
        // the operand order acc, ballot, mb)
        mlo = __builtin_amdgcn_bitop3_b32(mlo, (uint32_t)bal[b], mb[b], 0xF6);
        mhi = __builtin_amdgcn_bitop3_b32(mhi, (uint32_t)(bal[b] >> 32), mb[b], 0xF6);
    }
    return __ballot(valid) & ~(((uint64_t)mhi << 32) | mlo);
}

// Digit counts of keys[lo, lo + n), n <= RSORT_TILE: digit d's count is stored at hist[hb + d * hs].
template <typename KeyLoad>
__device__ __forceinline__ void rs_count_tile(KeyLoad keys, int64_t lo, int n, int shift,
                                              uint32_t* __restrict__ hist, int64_t hb,
                                              int64_t hs) {
    __shared__ uint32_t cnt[RSORT_WAVES][256];
    for (int i = threadIdx.x; i < RSORT_WAVES * 256; i += RSORT_NT) (&cnt[0][0])[i] = 0;
    __syncthreads();
    const int w = threadIdx.x / SPX_WAVE;
#pragma unroll
    for (int i = 0; i < RSORT_IPT; ++i) {
        const int j = i * RSORT_NT + threadIdx.x;
        if (j < n) atomicAdd(&cnt[w][(uint32_t)(keys(lo + j) >> shift) & 255u], 1u);
    }
    __syncthreads();
    for (int d = threadIdx.x; d < 256; d += RSORT_NT) {
        uint32_t c = 0;
#pragma unroll
        for (int ww = 0; ww < RSORT_WAVES; ++ww) c += cnt[ww][d];
        hist[hb + d * hs] = c;
    }
}

// Stable scatter of the tile keys[lo, lo + n) (with payloads) by digit: the keys of digit d go,
// in tile order, to kout[goff_of(d) ...].  goff_of is called once per digit.
template <typename KeyLoad, typename GOff>
__device__ __forceinline__ void rs_scatter_tile(KeyLoad kin, const uint64_t* __restrict__ vin,
                                                uint64_t* __restrict__ kout,
                                                uint64_t* __restrict__ vout, int64_t lo, int n,
                                                int shift, GOff goff_of) {
    __shared__ uint32_t wcnt[RSORT_WAVES][256];
    __shared__ uint32_t dstart[256];
    __shared__ uint32_t goff[256];
    __shared__ uint32_t stmp[RSORT_WAVES];
    __shared__ uint64_t sbuf[RSORT_TILE];  // keys, then payloads, in tile-sorted order

    const int tid = threadIdx.x;
    const int w = tid / SPX_WAVE;
    const int lane = __lane_id();
    for (int i = tid; i < RSORT_WAVES * 256; i += RSORT_NT) (&wcnt[0][0])[i] = 0;
    __syncthreads();

    const int wave_off = w * (RSORT_TILE / RSORT_WAVES);  // tile-relative
    const uint64_t lt = spx_lanemask_lt();
    uint64_t key[RSORT_ROUNDS];
    uint32_t pos[RSORT_ROUNDS];
    uint64_t val[RSORT_ROUNDS];
#pragma unroll
    for (int r = 0; r < RSORT_ROUNDS; ++r) {
        const int j = wave_off + r * SPX_WAVE + lane;
        const bool valid = j < n;
        key[r] = valid ? kin(lo + j) : 0ull;
        val[r] = valid ? vin[lo + j] : 0ull;  // payload fetched early, written after the keys
        const uint32_t d = (uint32_t)(key[r] >> shift) & 255u;
        const uint64_t peers = wave_digit_peers(d, valid);
        const uint32_t below = (uint32_t)__popcll(peers & lt);
        const uint32_t count = (uint32_t)__popcll(peers);
        const uint32_t basec = wcnt[w][d];
        __builtin_amdgcn_wave_barrier();
        if (valid && below == 0) wcnt[w][d] = basec + count;
        __builtin_amdgcn_wave_barrier();
        pos[r] = basec + below;
    }
    __syncthreads();
    // per digit: exclusive offsets of the waves, then the tile's exclusive digit starts
    uint32_t run = 0;
    if (tid < 256) {
#pragma unroll
        for (int ww = 0; ww < RSORT_WAVES; ++ww) {
            const uint32_t t = wcnt[ww][tid];
            wcnt[ww][tid] = run;
            run += t;
        }
    }
    uint32_t tile_total;
    const uint32_t ex = block_excl_scan<RSORT_NT, uint32_t, OpSum<uint32_t>>(run, stmp, &tile_total);
    if (tid < 256) {
        dstart[tid] = ex;
        goff[tid] = goff_of(tid);
    }
    __syncthreads();
    // phase 1: keys
#pragma unroll
    for (int r = 0; r < RSORT_ROUNDS; ++r) {
        if (wave_off + r * SPX_WAVE + lane < n) {
            const uint32_t d = (uint32_t)(key[r] >> shift) & 255u;
            pos[r] += dstart[d] + wcnt[w][d];
            sbuf[pos[r]] = key[r];
        }
    }
    __syncthreads();
    uint32_t dst_lo[RSORT_IPT];  // output offset of LDS slot tid + q*NT, reused for the payload
#pragma unroll
    for (int q = 0; q < RSORT_IPT; ++q) {
        const int i = q * RSORT_NT + tid;
        if (i < n) {
            const uint64_t k = sbuf[i];
            const uint32_t d = (uint32_t)(k >> shift) & 255u;
            dst_lo[q] = goff[d] + (uint32_t)(i - (int)dstart[d]);
            kout[dst_lo[q]] = k;
        }
    }
    __syncthreads();
    // phase 2: payloads, through the same LDS slots
#pragma unroll
    for (int r = 0; r < RSORT_ROUNDS; ++r)
        if (wave_off + r * SPX_WAVE + lane < n) sbuf[pos[r]] = val[r];
    __syncthreads();
#pragma unroll
    for (int q = 0; q < RSORT_IPT; ++q) {
        const int i = q * RSORT_NT + tid;
        if (i < n) vout[dst_lo[q]] = sbuf[i];
    }
}

struct GOffLsd {  // digit-major histogram of equal tiles, scanned
    const uint32_t* hist;
    int64_t tiles, tile;
    __device__ uint32_t operator()(int d) const { return hist[(int64_t)d * tiles + tile]; }
};

__device__ __forceinline__ void rsort_upsweep(const uint64_t* __restrict__ keys, int64_t E,
                                              int shift, uint32_t* __restrict__ hist,
                                              int64_t tiles) {
    const int64_t tile = rs_tile_of(blockIdx.x, tiles);
    const int64_t lo = tile * RSORT_TILE;
    const int n = E - lo < RSORT_TILE ? (int)(E - lo) : RSORT_TILE;
    rs_count_tile(KeyArr{keys}, lo, n, shift, hist, tile, tiles);
}

__device__ __forceinline__ void rsort_downsweep(
    const uint64_t* __restrict__ kin, const uint64_t* __restrict__ vin,
    uint64_t* __restrict__ kout, uint64_t* __restrict__ vout, int64_t E, int shift,
    const uint32_t* __restrict__ hist, int64_t tiles) {
    const int64_t tile = rs_tile_of(blockIdx.x, tiles);
    const int64_t lo = tile * RSORT_TILE;
    const int n = E - lo < RSORT_TILE ? (int)(E - lo) : RSORT_TILE;
    rs_scatter_tile(KeyArr{kin}, vin, kout, vout, lo, n, shift, GOffLsd{hist, tiles, tile});
}

// LSD kernels: they sort the hot-column sample (the conversion itself uses the MSD sort below).
#define RSORT_KERNELS(UP, DOWN)                                                                 \
    __global__ __launch_bounds__(RSORT_NT) void UP(const uint64_t* __restrict__ keys, int64_t E, \
                                                   int shift, uint32_t* __restrict__ hist,      \
                                                   int64_t tiles) {                             \
        rsort_upsweep(keys, E, shift, hist, tiles);                                             \
    }                                                                                           \
    __global__ __launch_bounds__(RSORT_NT) void DOWN(                                           \
        const uint64_t* __restrict__ kin, const uint64_t* __restrict__ vin,                     \
        uint64_t* __restrict__ kout, uint64_t* __restrict__ vout, int64_t E, int shift,         \
        const uint32_t* __restrict__ hist, int64_t tiles) {                                     \
        rsort_downsweep(kin, vin, kout, vout, E, shift, hist, tiles);                           \
    }
RSORT_KERNELS(k_hot_rsort_upsweep, k_hot_rsort_downsweep)
#undef RSORT_KERNELS

struct LoadU32 {
    const uint32_t* p;
    __device__ uint32_t operator()(int64_t i) const { return p[i]; }
};
struct StoreExclU32 {
    uint32_t* p;
    __device__ void operator()(int64_t i, uint32_t incl, uint32_t item) const { p[i] = incl - item; }
};

hipError_t radix_sort_pairs(uint64_t* k0, uint64_t* v0, uint64_t* k1, uint64_t* v1,
                            const uint64_t* vfirst, int64_t E, uint64_t vary, uint32_t* hist,
                            uint32_t* tile_sums, hipStream_t s, const uint64_t** keys_sorted,
                            const uint64_t** vals_sorted) {
    *keys_sorted = k0;
    *vals_sorted = vfirst;
    if (E <= 0) return hipSuccess;
    const int64_t tiles = spx_div_up(E, RSORT_TILE);
    const int64_t hn = 256 * tiles;
    uint64_t* kin = k0;
    uint64_t* kout = k1;
    const uint64_t* vin = vfirst;  // the first executed pass reads the caller's values
    uint64_t* vout = v1;
    uint64_t* vnext = v0;
    for (int shift = 0; shift < 64; shift += RS_RADIX_BITS) {
        if (((vary >> shift) & 0xFFull) == 0) continue;  // digit constant: order unchanged
        SPX_LAUNCH("hot_rsort_upsweep", k_hot_rsort_upsweep, dim3((unsigned)tiles),
                   dim3(RSORT_NT), 0, s, kin, E, shift, hist, tiles);
        hipError_t e = scan_phase12<uint32_t, OpSum<uint32_t>>(LoadU32{hist}, hn, tile_sums,
                                                               (uint32_t*)nullptr, s);
        if (e != hipSuccess) return e;
        e = scan_phase3<uint32_t, OpSum<uint32_t>>(LoadU32{hist}, StoreExclU32{hist}, hn,
                                                   tile_sums, s);
        if (e != hipSuccess) return e;
        SPX_LAUNCH("hot_rsort_downsweep", k_hot_rsort_downsweep, dim3((unsigned)tiles),
                   dim3(RSORT_NT), 0, s, kin, vin, kout, vout, E, shift, hist, tiles);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
        uint64_t* kt = kin;
        kin = kout;
        kout = kt;
        vin = vout;
        uint64_t* vt = vout;
        vout = vnext;
        vnext = vt;
    }
    *keys_sorted = kin;
    *vals_sorted = vin;
    return hipGetLastError();
}

// ------------------------------------------------------------------ MSD radix sort, LDS finish
//
// The conversion sort.  Digits are taken from the most significant varying one down.  A segment
// is a range of positions whose keys agree on every digit above the current one; it starts as
// [0, E).  Each level splits every segment longer than RS_LOCAL_MAX by one digit with a stable
// counting pass (tiles never straddle segments; the digit offsets of all segments come from one
// scan of a segment-major, digit-major, tile-minor histogram).  Parts of at most RS_LOCAL_MAX
// keys leave the recursion: consecutive such parts of one segment are packed into chunks of at
// most RS_LOCAL_MAX keys, and each chunk is sorted by one workgroup in LDS on its remaining
// digits (stable passes over the digits that vary inside the chunk) and written to the output
// buffer.  Parts still longer after the last varying digit hold equal keys and are copied.
// Every pass is stable, so equal keys keep their input order: the result equals the LSD sort's.
//
// Buffers: level p reads B_p and writes B_{p+1}; B_0 = (k0, vfirst), B_odd = (k1, v1),
// B_even>0 = (k0, v0).  The output is (k1, v1).  A chunk records which buffer holds it.


struct MsdCounters {
    uint32_t nbig, ntiles, nchunks, err, bigkeys, pad;
    unsigned long long kor, kand;  // OR and AND of the keys (CRS keys built in the first level)
};

__global__ void k_msd_init(int64_t E, int64_t* seg_start, uint32_t* seg_len, uint32_t* tbase,
                           MsdChunk* chunks, MsdCounters* ctr) {
    ctr->nbig = 0;
    ctr->ntiles = 0;
    ctr->nchunks = 0;
    ctr->err = 0;
    ctr->bigkeys = 0;
    ctr->kor = 0ull;
    ctr->kand = ~0ull;
    if (E > RS_LOCAL_MAX) {
        seg_start[0] = 0;
        seg_len[0] = (uint32_t)E;
        tbase[0] = 0;  // the first level's table, for a first level that skips the tile scan
        tbase[1] = (uint32_t)((E + RSORT_TILE - 1) / RSORT_TILE);
    } else {
        chunks[0] = MsdChunk{0, (uint32_t)E, 64u};  // all bits, source B_0
        ctr->nchunks = 1;
    }
}

__global__ void k_msd_next_level(MsdCounters* ctr) {
    ctr->nbig = 0;
    ctr->ntiles = 0;
    ctr->bigkeys = 0;
}

struct LoadNt {
    const uint32_t* len;
    __device__ uint32_t operator()(int64_t i) const {
        return (len[i] + RSORT_TILE - 1) / RSORT_TILE;
    }
};

// tile_seg[g] = the segment whose tiles include g (tbase strictly increasing, nb + 1 entries)
__global__ void k_msd_tile_seg(const uint32_t* __restrict__ tbase, uint32_t nb, uint32_t T,
                               uint32_t* __restrict__ tile_seg) {
    const uint32_t g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= T) return;
    uint32_t lo = 0, hi = nb - 1;  // last s with tbase[s] <= g
    while (lo < hi) {
        const uint32_t mid = (lo + hi + 1) >> 1;
        if (tbase[mid] <= g) lo = mid;
        else hi = mid - 1;
    }
    tile_seg[g] = lo;
}

struct MsdTile {
    int64_t lo;
    int n;
    int64_t hb;  // histogram index of (segment, digit 0, this tile)
    int64_t hs;  // tiles of the segment (histogram stride between digits)
    int64_t h0;  // histogram index of (segment, digit 0, tile 0)
    int64_t start;
};

__device__ __forceinline__ MsdTile msd_tile(const int64_t* seg_start, const uint32_t* seg_len,
                                            const uint32_t* tbase, const uint32_t* tile_seg,
                                            uint32_t T) {
    const uint32_t g = (uint32_t)rs_tile_of(blockIdx.x, T);
    const uint32_t sg = tile_seg[g];
    const uint32_t tb = tbase[sg];
    const uint32_t t = g - tb;
    const int64_t len = seg_len[sg];
    MsdTile m;
    m.start = seg_start[sg];
    m.lo = m.start + (int64_t)t * RSORT_TILE;
    const int64_t rem = len - (int64_t)t * RSORT_TILE;
    m.n = rem < RSORT_TILE ? (int)rem : RSORT_TILE;
    m.hs = tbase[sg + 1] - tb;
    m.h0 = (int64_t)tb * 256;
    m.hb = m.h0 + t;
    return m;
}

__global__ __launch_bounds__(RSORT_NT) void k_msd_count(const uint64_t* __restrict__ keys,
                                                        const int64_t* __restrict__ seg_start,
                                                        const uint32_t* __restrict__ seg_len,
                                                        const uint32_t* __restrict__ tbase,
                                                        const uint32_t* __restrict__ tile_seg,
                                                        uint32_t T, int shift,
                                                        uint32_t* __restrict__ hist) {
    const MsdTile m = msd_tile(seg_start, seg_len, tbase, tile_seg, T);
    rs_count_tile(KeyArr{keys}, m.lo, m.n, shift, hist, m.hb, m.hs);
}

struct GOffMsd {  // segment start + scanned (segment, digit, tile) entry - segment's first entry
    const uint32_t* hist;
    int64_t hb, hs, base;
    __device__ uint32_t operator()(int d) const {
        return (uint32_t)(base + (int64_t)hist[hb + (int64_t)d * hs]);
    }
};

__global__ __launch_bounds__(RSORT_NT) void k_msd_scatter(
    const uint64_t* __restrict__ kin, const uint64_t* __restrict__ vin,
    uint64_t* __restrict__ kout, uint64_t* __restrict__ vout,
    const int64_t* __restrict__ seg_start, const uint32_t* __restrict__ seg_len,
    const uint32_t* __restrict__ tbase, const uint32_t* __restrict__ tile_seg, uint32_t T,
    int shift, const uint32_t* __restrict__ hist) {
    const MsdTile m = msd_tile(seg_start, seg_len, tbase, tile_seg, T);
    const int64_t base = m.start - (int64_t)hist[m.h0];
    rs_scatter_tile(KeyArr{kin}, vin, kout, vout, m.lo, m.n, shift, GOffMsd{hist, m.hb, m.hs, base});
}

// First level of a CRS conversion, straight from the triplets: digit counts of the tile (one
// segment [0, E), equal tiles in the XCD order), the OR / AND of the keys and the index check.
template <typename KeyFn>
__global__ __launch_bounds__(RSORT_NT) void k_msd_count0(
    KeyFromTriplets<KeyFn> kf, int64_t E, int shift, uint32_t T0, uint32_t* __restrict__ hist,
    unsigned long long* __restrict__ tile_masks, MsdCounters* ctr) {
    __shared__ uint32_t cnt[RSORT_WAVES][256];
    __shared__ unsigned long long s_or[RSORT_WAVES], s_and[RSORT_WAVES];
    __shared__ uint32_t s_bad[RSORT_WAVES];
    for (int i = threadIdx.x; i < RSORT_WAVES * 256; i += RSORT_NT) (&cnt[0][0])[i] = 0;
    __syncthreads();
    const int w = threadIdx.x / SPX_WAVE;
    const int64_t g = rs_tile_of(blockIdx.x, T0);
    const int64_t lo = g * RSORT_TILE;
    const int n = E - lo < RSORT_TILE ? (int)(E - lo) : RSORT_TILE;
    unsigned long long orv = 0ull, andv = ~0ull;
    uint32_t bad = 0;
    // When the digit lies above the within-block curve index (CSB), the index is not computed
    // here: its bits are taken as varying (OR all ones, AND zero).  That only costs a split on a
    // digit that turns out constant, on inputs whose entries all share those bits.
    const int ob = kf.fn.order_bits();
    const bool high_only = ob > 0 && shift >= ob;
    const unsigned long long lowm = ob >= 64 ? ~0ull : (1ull << ob) - 1ull;
#pragma unroll
    for (int i = 0; i < RSORT_IPT; ++i) {
        const int j = i * RSORT_NT + threadIdx.x;
        if (j < n) {
            const int32_t r = kf.row[lo + j], c = kf.col[lo + j];
            const bool ok = kf.valid(r, c);
            bad |= ok ? 0u : 1u;
            uint64_t key;
            if (high_only) {
                key = ok ? kf.fn.high_part((uint32_t)r, (uint32_t)c) : 0ull;
                orv |= key | lowm;
            } else {
                key = ok ? kf.fn((uint32_t)r, (uint32_t)c) : 0ull;
                orv |= key;
            }
            andv &= key;
            atomicAdd(&cnt[w][(uint32_t)(key >> shift) & 255u], 1u);
        }
    }
    orv = wave_reduce<unsigned long long, OpOr<unsigned long long>>(orv);
    andv = wave_reduce<unsigned long long, OpAnd<unsigned long long>>(andv);
    const uint64_t anybad = __ballot(bad != 0);
    if (__lane_id() == 0) {
        s_or[w] = orv;
        s_and[w] = andv;
        s_bad[w] = anybad ? 1u : 0u;
    }
    __syncthreads();
    for (int d = threadIdx.x; d < 256; d += RSORT_NT) {
        uint32_t c = 0;
#pragma unroll
        for (int ww = 0; ww < RSORT_WAVES; ++ww) c += cnt[ww][d];
        hist[(int64_t)d * T0 + g] = c;
    }
    if (threadIdx.x == 0) {
        uint32_t b = 0;
        for (int ww = 0; ww < RSORT_WAVES; ++ww) {
            orv |= s_or[ww];
            andv &= s_and[ww];
            b |= s_bad[ww];
        }
        // the tile's OR / AND are combined by k_msd_masks: no global read or atomic here, so
        // the workgroup's last wave does not wait on a round trip before its slots free up
        tile_masks[2 * g] = orv;
        tile_masks[2 * g + 1] = andv;
        if (b) atomicOr(&ctr->err, 1u);
    }
}

static_assert(sizeof(MsdChunk) == 2 * sizeof(unsigned long long), "one tile's pair per chunk");

// OR / AND over the first level's per-tile pairs, into the counters (one atomic each per
// workgroup).
#define MSD_MASK_NT 256
__global__ __launch_bounds__(MSD_MASK_NT) void k_msd_masks(
    const unsigned long long* __restrict__ tile_masks, uint32_t T0, MsdCounters* ctr) {
    constexpr int NW = MSD_MASK_NT / SPX_WAVE;
    __shared__ unsigned long long s_or[NW], s_and[NW];
    unsigned long long orv = 0ull, andv = ~0ull;
    for (uint32_t t = blockIdx.x * MSD_MASK_NT + threadIdx.x; t < T0;
         t += gridDim.x * MSD_MASK_NT) {
        orv |= tile_masks[2 * (int64_t)t];
        andv &= tile_masks[2 * (int64_t)t + 1];
    }
    orv = wave_reduce<unsigned long long, OpOr<unsigned long long>>(orv);
    andv = wave_reduce<unsigned long long, OpAnd<unsigned long long>>(andv);
    const int w = threadIdx.x / SPX_WAVE;
    if (__lane_id() == 0) {
        s_or[w] = orv;
        s_and[w] = andv;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int ww = 1; ww < NW; ++ww) {
            orv |= s_or[ww];
            andv &= s_and[ww];
        }
        atomicOr(&ctr->kor, orv);
        atomicAnd(&ctr->kand, andv);
    }
}

template <typename KeyFn>
__global__ __launch_bounds__(RSORT_NT) void k_msd_scatter0(
    KeyFromTriplets<KeyFn> kf, const uint64_t* __restrict__ vin, uint64_t* __restrict__ kout,
    uint64_t* __restrict__ vout, int64_t E, int shift, uint32_t T0,
    const uint32_t* __restrict__ hist) {
    const int64_t g = rs_tile_of(blockIdx.x, T0);
    const int64_t lo = g * RSORT_TILE;
    const int n = E - lo < RSORT_TILE ? (int)(E - lo) : RSORT_TILE;
    rs_scatter_tile(kf, vin, kout, vout, lo, n, shift, GOffLsd{hist, (int64_t)T0, g});
}

// Segments still large when no varying digit is left hold equal keys: copy chunks.
__global__ void k_msd_flush(const int64_t* __restrict__ seg_start,
                            const uint32_t* __restrict__ seg_len, uint32_t nb, uint32_t meta,
                            MsdChunk* __restrict__ chunks, uint32_t cap_chunks, MsdCounters* ctr) {
    const uint32_t sg = blockIdx.x * blockDim.x + threadIdx.x;
    if (sg >= nb) return;
    const uint32_t i = atomicAdd(&ctr->nchunks, 1u);
    if (i < cap_chunks) chunks[i] = MsdChunk{seg_start[sg], seg_len[sg], meta};
    else atomicOr(&ctr->err, 8u);
}

// One wave per segment: each lane loads the sizes of 4 of the 256 parts; the wave walks them in
// digit order, packing consecutive small parts into chunks and listing the large ones for the
// next level (or as copy chunks after the last varying digit); it then reserves its list entries
// with one atomic per list and writes them in parallel.
#define MSD_CLS_NT 256
__global__ __launch_bounds__(MSD_CLS_NT) void k_msd_classify(
    const int64_t* __restrict__ seg_start, const uint32_t* __restrict__ seg_len,
    const uint32_t* __restrict__ tbase, uint32_t nb, const uint32_t* __restrict__ hist, int last,
    uint32_t meta, int64_t* __restrict__ nstart, uint32_t* __restrict__ nlen, uint32_t cap_big,
    MsdChunk* __restrict__ chunks, uint32_t cap_chunks, MsdCounters* ctr) {
    constexpr int NW = MSD_CLS_NT / SPX_WAVE;
    __shared__ uint32_t s_olen[NW][256];   // outputs in digit order: length,
    __shared__ uint32_t s_ooff[NW][256];   // offset in the segment,
    __shared__ uint8_t s_obig[NW][256];    // 1: next-level segment, 0: chunk
    __shared__ uint32_t s_nout[NW], s_cbase[NW], s_bbase[NW];
    const int w = threadIdx.x / SPX_WAVE;
    const int lane = __lane_id();
    const uint32_t sg = blockIdx.x * NW + w;
    if (sg >= nb) return;  // whole waves leave; no workgroup barrier below
    const int64_t st = seg_start[sg];
    const uint32_t len = seg_len[sg];
    const int64_t hs = tbase[sg + 1] - tbase[sg];
    const int64_t h0 = (int64_t)tbase[sg] * 256;
    const uint32_t x0 = hist[h0];
    uint32_t cnt[4], off[4];  // lane l: digits l, l + 64, l + 128, l + 192
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const int d = lane + 64 * q;
        const uint32_t xd = hist[h0 + d * hs];
        const uint32_t xe = d < 255 ? hist[h0 + (d + 1) * hs] : x0 + len;
        cnt[q] = xe - xd;
        off[q] = xd - x0;
    }
    // the walk in digit order is wave-uniform: every lane runs it on values read from their
    // owning lanes (scalar reads), and lane 0 records the outputs
    uint32_t no = 0, nbig = 0, tiles = 0, coff = 0, cl = 0, bigkeys = 0;
    auto emit = [&](uint32_t len_, uint32_t off_, uint8_t big_) {
        if (lane == 0) {
            s_olen[w][no] = len_;
            s_ooff[w][no] = off_;
            s_obig[w][no] = big_;
        }
        ++no;
    };
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        for (int l = 0; l < SPX_WAVE; ++l) {
            const uint32_t c = (uint32_t)__builtin_amdgcn_readlane((int)cnt[q], l);
            if (c == 0) continue;
            const uint32_t o = (uint32_t)__builtin_amdgcn_readlane((int)off[q], l);
            if (c <= RS_LOCAL_MAX) {
                if (cl > 0 && cl + c <= RS_LOCAL_MAX) {
                    cl += c;
                    continue;
                }
                if (cl > 0) emit(cl, coff, 0);
                coff = o;
                cl = c;
            } else {
                if (cl > 0) emit(cl, coff, 0);
                cl = 0;
                const bool big = !last;  // after the last varying digit: equal keys, copied
                emit(c, o, big ? 1 : 0);
                if (big) {
                    ++nbig;
                    tiles += (c + RSORT_TILE - 1) / RSORT_TILE;
                    bigkeys += c;
                }
            }
        }
    }
    if (cl > 0) emit(cl, coff, 0);
    if (lane == 0) {
        s_nout[w] = no;
        s_cbase[w] = no - nbig > 0 ? atomicAdd(&ctr->nchunks, no - nbig) : 0u;
        s_bbase[w] = nbig > 0 ? atomicAdd(&ctr->nbig, nbig) : 0u;
        if (tiles > 0) {
            atomicAdd(&ctr->ntiles, tiles);
            atomicAdd(&ctr->bigkeys, bigkeys);
        }
    }
    __builtin_amdgcn_wave_barrier();
    uint32_t cb = s_cbase[w], bb = s_bbase[w];
    for (uint32_t o0 = 0; o0 < no; o0 += SPX_WAVE) {  // outputs in order, ranked by ballots
        const uint32_t o = o0 + lane;
        const bool valid = o < no;
        const bool big = valid && s_obig[w][o];
        const uint64_t bbal = __ballot(big), cbal = __ballot(valid && !big);
        const uint64_t lt = spx_lanemask_lt();
        if (valid) {
            const int64_t sub = st + s_ooff[w][o];
            const uint32_t c = s_olen[w][o];
            if (big) {
                const uint32_t i = bb + (uint32_t)__popcll(bbal & lt);
                if (i < cap_big) {
                    nstart[i] = sub;
                    nlen[i] = c;
                } else {
                    atomicOr(&ctr->err, 8u);
                }
            } else {
                const uint32_t i = cb + (uint32_t)__popcll(cbal & lt);
                if (i < cap_chunks) chunks[i] = MsdChunk{sub, c, meta};
                else atomicOr(&ctr->err, 8u);
            }
        }
        bb += (uint32_t)__popcll(bbal);
        cb += (uint32_t)__popcll(cbal);
    }
}

#ifndef MSD_LNT
#define MSD_LNT 512
#endif
#define MSD_LWAVES (MSD_LNT / SPX_WAVE)
#define MSD_LROUNDS (RS_LOCAL_MAX / MSD_LNT)
static_assert(MSD_LNT >= 256 && RS_LOCAL_MAX % MSD_LNT == 0, "local sort shape");
static_assert(RS_LOCAL_MAX <= SCAN_TILE, "a chunk meets at most two tiles of head counts");

// One workgroup per chunk: keys and payloads of at most RS_LOCAL_MAX positions, stable LSD
// passes in LDS over the digits below `hi` that vary inside the chunk, then the keys and the
// payloads (each to its final position) are written to (kf, vf).  Chunks longer than
// RS_LOCAL_MAX hold equal keys and are copied.
__global__ __launch_bounds__(MSD_LNT) void k_msd_local(
    const MsdChunk* __restrict__ chunks, const uint64_t* k0, const uint64_t* vfirst,
    const uint64_t* v0, uint64_t* kf, uint64_t* vf, uint32_t* __restrict__ head_tiles) {
    __shared__ uint64_t skey[RS_LOCAL_MAX];
    __shared__ uint16_t sidx[RS_LOCAL_MAX];
    __shared__ uint32_t wcnt[MSD_LWAVES][256];
    __shared__ uint32_t dstart[256];
    __shared__ uint32_t stmp[MSD_LWAVES];
    __shared__ uint64_t sred[2][MSD_LWAVES];
    const MsdChunk c = chunks[blockIdx.x];
    const int src = (int)(c.meta >> 8);  // 0: B_0, 1: (k1, v1) = output, 2: (k0, v0)
    const int hi = (int)(c.meta & 255u);
    const uint64_t* ks = src == 1 ? kf : k0;
    const uint64_t* vs = src == 0 ? vfirst : src == 1 ? vf : v0;
    const int tid = threadIdx.x;
    if (c.len > RS_LOCAL_MAX) {  // equal keys, already in input order
        if (src != 1)
            for (int64_t i = tid; i < c.len; i += MSD_LNT) {
                kf[c.start + i] = ks[c.start + i];
                vf[c.start + i] = vs[c.start + i];
            }
        return;
    }
    const int n = (int)c.len;
    const int w = tid / SPX_WAVE;
    const int lane = __lane_id();
    const int wave_off = w * (RS_LOCAL_MAX / MSD_LWAVES);
    const uint64_t lt = spx_lanemask_lt();
    uint64_t key[MSD_LROUNDS], val[MSD_LROUNDS];
    uint32_t idx[MSD_LROUNDS];
    uint64_t vor = 0, vand = ~0ull;
#pragma unroll
    for (int r = 0; r < MSD_LROUNDS; ++r) {
        const int j = wave_off + r * SPX_WAVE + lane;
        key[r] = j < n ? ks[c.start + j] : 0ull;
        idx[r] = (uint32_t)j;
        if (j < n) {
            vor |= key[r];
            vand &= key[r];
        }
    }
    // the key loads have landed before any thread can write the chunk back (it may be in place)
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
    vor = wave_reduce<uint64_t, OpOr<uint64_t>>(vor);
    vand = wave_reduce<uint64_t, OpAnd<uint64_t>>(vand);
    if (lane == 0) {
        sred[0][w] = vor;
        sred[1][w] = vand;
    }
    __syncthreads();
    vor = 0;
    vand = ~0ull;
#pragma unroll
    for (int ww = 0; ww < MSD_LWAVES; ++ww) {
        vor |= sred[0][ww];
        vand &= sred[1][ww];
    }
    const uint64_t vm = (vor ^ vand) & (hi >= 64 ? ~0ull : ((1ull << hi) - 1ull));
    // a wave ranks against, and scatters with, its own row of wcnt only, so it clears that row
    // itself: ahead of the first pass, and after each pass's last read of it (the scatter)
    for (int i = lane; i < 256; i += SPX_WAVE) wcnt[w][i] = 0;
    __builtin_amdgcn_wave_barrier();
    for (int ds = 0; ds < hi; ds += RS_RADIX_BITS) {
        if (((vm >> ds) & 255ull) == 0) continue;  // uniform: vm is the same in every thread
        uint32_t pos[MSD_LROUNDS];
#pragma unroll
        for (int r = 0; r < MSD_LROUNDS; ++r) {
            const bool valid = wave_off + r * SPX_WAVE + lane < n;
            const uint32_t d = (uint32_t)(key[r] >> ds) & 255u;
            const uint64_t peers = wave_digit_peers(d, valid);
            const uint32_t below = (uint32_t)__popcll(peers & lt);
            const uint32_t count = (uint32_t)__popcll(peers);
            const uint32_t basec = wcnt[w][d];
            __builtin_amdgcn_wave_barrier();
            if (valid && below == 0) wcnt[w][d] = basec + count;
            __builtin_amdgcn_wave_barrier();
            pos[r] = basec + below;
        }
        __syncthreads();
        uint32_t run = 0;
        if (tid < 256) {
#pragma unroll
            for (int ww = 0; ww < MSD_LWAVES; ++ww) {
                const uint32_t t = wcnt[ww][tid];
                wcnt[ww][tid] = run;
                run += t;
            }
        }
        uint32_t total;
        const uint32_t ex =
            block_excl_scan<MSD_LNT, uint32_t, OpSum<uint32_t>>(run, stmp, &total);
        if (tid < 256) dstart[tid] = ex;
        __syncthreads();
#pragma unroll
        for (int r = 0; r < MSD_LROUNDS; ++r) {
            if (wave_off + r * SPX_WAVE + lane < n) {
                const uint32_t d = (uint32_t)(key[r] >> ds) & 255u;
                const uint32_t p = dstart[d] + wcnt[w][d] + pos[r];
                skey[p] = key[r];
                sidx[p] = (uint16_t)idx[r];
            }
        }
        __syncthreads();
#pragma unroll
        for (int r = 0; r < MSD_LROUNDS; ++r) {
            const int j = wave_off + r * SPX_WAVE + lane;
            if (j < n) {
                key[r] = skey[j];
                idx[r] = sidx[j];
            }
        }
        // the next pass writes skey / sidx only after its two barriers, which every thread
        // reaches after these reads; its scan rewrites wcnt only after the first of them
        __builtin_amdgcn_wave_barrier();
        for (int i = lane; i < 256; i += SPX_WAVE) wcnt[w][i] = 0;
        __builtin_amdgcn_wave_barrier();
    }
    __syncthreads();  // the last pass's reads of skey / sidx are done before the writes below
    // payloads fetched after the passes (fewer live registers during them); every thread uses
    // its loads before the barrier ahead of the payload writes, so an in-place chunk is read
    // completely before it is written
#pragma unroll
    for (int r = 0; r < MSD_LROUNDS; ++r) {
        const int j = wave_off + r * SPX_WAVE + lane;
        val[r] = j < n ? vs[c.start + j] : 0ull;
    }
    // keys in order; the payload of input position j is staged at the final position of j (in
    // the key buffer, whose last reads are behind the pass loop's barrier) and written in order
#pragma unroll
    for (int r = 0; r < MSD_LROUNDS; ++r) {
        const int j = wave_off + r * SPX_WAVE + lane;
        if (j < n) {
            kf[c.start + j] = key[r];
            sidx[idx[r]] = (uint16_t)j;
            if (head_tiles) skey[j] = key[r];
        }
    }
    __syncthreads();
    if (head_tiles) {
        // run heads at positions 1..n-1 of the chunk (position 0 is settled by
        // k_msd_heads_first), counted per SCAN_TILE of positions: a chunk meets at most two
        const int64_t ta = c.start / SCAN_TILE;
        uint32_t ha = 0, hb = 0;
#pragma unroll
        for (int r = 0; r < MSD_LROUNDS; ++r) {
            const int j = wave_off + r * SPX_WAVE + lane;
            if (j >= 1 && j < n && skey[j] != skey[j - 1]) {
                if ((c.start + j) / SCAN_TILE == ta) ++ha;
                else ++hb;
            }
        }
        ha = wave_reduce<uint32_t, OpSum<uint32_t>>(ha);
        hb = wave_reduce<uint32_t, OpSum<uint32_t>>(hb);
        if (lane == 0) {
            if (ha) atomicAdd(&head_tiles[ta], ha);
            if (hb) atomicAdd(&head_tiles[ta + 1], hb);
        }
        __syncthreads();  // skey is reused for the payloads below
    }
#pragma unroll
    for (int r = 0; r < MSD_LROUNDS; ++r) {
        const int j = wave_off + r * SPX_WAVE + lane;
        if (j < n) skey[sidx[j]] = val[r];
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < MSD_LROUNDS; ++r) {
        const int j = wave_off + r * SPX_WAVE + lane;
        if (j < n) vf[c.start + j] = skey[j];
    }
}

// Position 0 of every chunk is a run head when it is position 0 of the array or its key differs
// from the key before it (which another chunk wrote).
__global__ void k_msd_heads_first(const MsdChunk* __restrict__ chunks, uint32_t nchunks,
                                  const uint64_t* __restrict__ kf,
                                  uint32_t* __restrict__ head_tiles) {
    const uint32_t i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nchunks) return;
    const int64_t p = chunks[i].start;
    if (p == 0 || kf[p] != kf[p - 1]) atomicAdd(&head_tiles[p / SCAN_TILE], 1u);
}

MsdSizes msd_sizes(int64_t E) {
    MsdSizes z;
    const int64_t tiles = spx_div_up(E > 0 ? E : 1, RSORT_TILE);
    z.cap_big = E / (RS_LOCAL_MAX + 1) + 2;
    z.cap_tiles = tiles + z.cap_big;
    // per level at most 4 E / RS_LOCAL_MAX + 2 chunks (consecutive packed chunks of one segment
    // hold more than RS_LOCAL_MAX keys together), at most 8 levels, copies, the single chunk
    z.cap_chunks = 33 * spx_div_up(E > 0 ? E : 1, RS_LOCAL_MAX) + 32;
    z.hist = 256 * z.cap_tiles;
    z.tile_sums = scan_tile_count(z.hist) > scan_tile_count(z.cap_big + 1)
                      ? scan_tile_count(z.hist)
                      : scan_tile_count(z.cap_big + 1);
    return z;
}

static hipError_t msd_read(MsdCounters* host, const MsdCounters* dev, hipStream_t s) {
    hipError_t e = hipMemcpyAsync(host, dev, sizeof *host, hipMemcpyDeviceToHost, s);
    if (e != hipSuccess) return e;
    return hipStreamSynchronize(s);
}

// The first level straight from the triplets: digit counts with the index check and the key
// masks, the scan of the (digit, tile) table, the scatter of keys and values into (k1, v1).
template <typename KeyFn>
static hipError_t msd_first_level(const KeyFromTriplets<KeyFn>& kf, const char* count_name,
                                  const char* scatter_name, const uint64_t* vfirst, uint64_t* k1,
                                  uint64_t* v1, int64_t E, int shift0, uint32_t T,
                                  const MsdScratch& sc, unsigned long long* tile_masks,
                                  MsdCounters* ctr, hipStream_t s) {
    SPX_LAUNCH(count_name, k_msd_count0<KeyFn>, dim3(T), dim3(RSORT_NT), 0, s, kf, E, shift0, T,
               sc.hist, tile_masks, ctr);
    const uint32_t gm = T < 256u * MSD_MASK_NT ? (T + MSD_MASK_NT - 1) / MSD_MASK_NT : 256u;
    SPX_LAUNCH("msd_masks", k_msd_masks, dim3(gm), dim3(MSD_MASK_NT), 0, s,
               (const unsigned long long*)tile_masks, T, ctr);
    const int64_t hn = (int64_t)256 * T;
    hipError_t e = scan_phase12<uint32_t, OpSum<uint32_t>>(LoadU32{sc.hist}, hn, sc.tile_sums,
                                                           (uint32_t*)nullptr, s);
    if (e != hipSuccess) return e;
    e = scan_phase3<uint32_t, OpSum<uint32_t>>(LoadU32{sc.hist}, StoreExclU32{sc.hist}, hn,
                                               sc.tile_sums, s);
    if (e != hipSuccess) return e;
    SPX_LAUNCH(scatter_name, k_msd_scatter0<KeyFn>, dim3(T), dim3(RSORT_NT), 0, s, kf, vfirst,
               k1, v1, E, shift0, T, sc.hist);
    return hipGetLastError();
}

hipError_t radix_sort_msd(uint64_t* k0, uint64_t* v0, uint64_t* k1, uint64_t* v1,
                          const uint64_t* vfirst, int64_t E, uint64_t vary, const MsdScratch& sc,
                          hipStream_t s, const uint64_t** keys_sorted,
                          const uint64_t** vals_sorted, int* failed, MsdStats* stats,
                          const MsdTripletSource* trip, uint32_t* head_tiles,
                          int* heads_counted) {
    *keys_sorted = k0;
    *vals_sorted = vfirst;
    *failed = 0;
    *stats = MsdStats{};
    if (heads_counted) *heads_counted = 0;
    if (E <= 0) return hipSuccess;
    if (!trip && vary == 0) return hipSuccess;  // no key differs: the input order stands
    if (head_tiles) {
        hipError_t e0 = launch_fill_i32((int32_t*)head_tiles, spx_div_up(E, SCAN_TILE), 0, s);
        if (e0 != hipSuccess) return e0;
    }
    if (trip && E <= RS_LOCAL_MAX) return hipErrorInvalidValue;  // caller builds keys first
    MsdCounters* ctr = (MsdCounters*)sc.counters;
    MsdCounters h{};
    SPX_LAUNCH("msd_init", k_msd_init, dim3(1), dim3(1), 0, s, E, sc.seg_start[0], sc.seg_len[0],
               sc.tbase, sc.chunks, ctr);
    uint32_t nb = E > RS_LOCAL_MAX ? 1u : 0u;
    uint32_t T = nb ? (uint32_t)spx_div_up(E, RSORT_TILE) : 0u;
    int p = 0;  // levels done
    int64_t level_keys = E;
    int top = 64 - RS_RADIX_BITS;
    hipError_t e;
    if (trip) {
        // first level from the triplets, on the top digit the matrix shape allows
        uint64_t kmax;
        if (trip->order == 0) {
            kmax = ((uint64_t)(trip->m - 1) << trip->cbits) | (uint64_t)(trip->n - 1);
        } else {
            int64_t nbr = ((int64_t)trip->m + (1ll << trip->k) - 1) >> trip->k;
            if (nbr < 1) nbr = 1;
            kmax = ((uint64_t)(nbr * trip->nbc - 1) << (2 * trip->k)) |
                   ((1ull << (2 * trip->k)) - 1ull);
        }
        int tb = 0;
        while (tb < 63 && (kmax >> (tb + 1)) != 0) ++tb;
        const int shift0 = tb / RS_RADIX_BITS * RS_RADIX_BITS;
        // the per-tile OR / AND pairs borrow the chunk list, first written by the classification
        // below (16 bytes per chunk, at least as many chunks as tiles)
        if ((int64_t)T > sc.z.cap_chunks) return hipErrorInvalidValue;
        unsigned long long* tile_masks = (unsigned long long*)sc.chunks;
        if (trip->order == 0) {
            const KeyFromTriplets<KeyCsr> kf{trip->row, trip->col, trip->m, trip->n,
                                             KeyCsr{trip->cbits}};
            e = msd_first_level(kf, "msd_count0_csr", "msd_scatter0_csr", vfirst, k1, v1, E,
                                shift0, T, sc, tile_masks, ctr, s);
        } else if (trip->order == 1) {
            const KeyFromTriplets<KeyCsb<true>> kf{trip->row, trip->col, trip->m, trip->n,
                                                   KeyCsb<true>{trip->k, (uint64_t)trip->nbc}};
            e = msd_first_level(kf, "msd_count0_csb", "msd_scatter0_csb", vfirst, k1, v1, E,
                                shift0, T, sc, tile_masks, ctr, s);
        } else {
            const KeyFromTriplets<KeyCsb<false>> kf{trip->row, trip->col, trip->m, trip->n,
                                                    KeyCsb<false>{trip->k, (uint64_t)trip->nbc}};
            e = msd_first_level(kf, "msd_count0_csb", "msd_scatter0_csb", vfirst, k1, v1, E,
                                shift0, T, sc, tile_masks, ctr, s);
        }
        if (e != hipSuccess) return e;
        SPX_LAUNCH("msd_next_level", k_msd_next_level, dim3(1), dim3(1), 0, s, ctr);
        const uint32_t meta = (uint32_t)(shift0 + RS_RADIX_BITS) | (1u << 8);
        SPX_LAUNCH("msd_classify", k_msd_classify, dim3(1), dim3(MSD_CLS_NT), 0, s,
                   sc.seg_start[0], sc.seg_len[0], sc.tbase, 1u, sc.hist, shift0 == 0 ? 1 : 0,
                   meta, sc.seg_start[1], sc.seg_len[1], (uint32_t)sc.z.cap_big, sc.chunks,
                   (uint32_t)sc.z.cap_chunks, ctr);
        e = msd_read(&h, ctr, s);
        if (e != hipSuccess) return e;
        if (h.err & 1u) {
            *failed = 2;  // an index outside the matrix
            return hipSuccess;
        }
        if (h.err) {
            *failed = 1;
            return hipSuccess;
        }
        vary = (uint64_t)(h.kor ^ h.kand);
        stats->split_keys = E;
        stats->levels = 1;
        stats->first_fused = 1;
        level_keys = h.bigkeys;
        nb = h.nbig;
        T = h.ntiles;
        p = 1;
        top = shift0 - RS_RADIX_BITS;
    }
    for (int shift = top; shift >= 0 && nb > 0; shift -= RS_RADIX_BITS) {
        if (((vary >> shift) & 0xFFull) == 0) continue;  // constant digit: no split
        const bool last = shift == 0 || (vary & ((1ull << shift) - 1ull)) == 0;
        const int cur = p & 1;
        const uint64_t* kin = p == 0 ? k0 : (p & 1) ? k1 : k0;
        const uint64_t* vin = p == 0 ? vfirst : (p & 1) ? v1 : v0;
        uint64_t* kout = (p & 1) ? k0 : k1;
        uint64_t* vout = (p & 1) ? v0 : v1;
        const uint32_t out_code = (p & 1) ? 2u : 1u;  // buffer that holds level p's output
        // tiles of the level's segments
        e = scan_phase12<uint32_t, OpSum<uint32_t>>(LoadNt{sc.seg_len[cur]}, nb, sc.tile_sums,
                                                    sc.tbase + nb, s);
        if (e != hipSuccess) return e;
        e = scan_phase3<uint32_t, OpSum<uint32_t>>(LoadNt{sc.seg_len[cur]},
                                                   StoreExclU32{sc.tbase}, nb, sc.tile_sums, s);
        if (e != hipSuccess) return e;
        SPX_LAUNCH("msd_tile_seg", k_msd_tile_seg, dim3(spx_div_up(T, 256)), dim3(256), 0, s,
                   sc.tbase, nb, T, sc.tile_seg);
        SPX_LAUNCH("msd_count", k_msd_count, dim3(T), dim3(RSORT_NT), 0, s, kin,
                   sc.seg_start[cur], sc.seg_len[cur], sc.tbase, sc.tile_seg, T, shift, sc.hist);
        const int64_t hn = (int64_t)256 * T;
        e = scan_phase12<uint32_t, OpSum<uint32_t>>(LoadU32{sc.hist}, hn, sc.tile_sums,
                                                    (uint32_t*)nullptr, s);
        if (e != hipSuccess) return e;
        e = scan_phase3<uint32_t, OpSum<uint32_t>>(LoadU32{sc.hist}, StoreExclU32{sc.hist}, hn,
                                                   sc.tile_sums, s);
        if (e != hipSuccess) return e;
        SPX_LAUNCH("msd_scatter", k_msd_scatter, dim3(T), dim3(RSORT_NT), 0, s, kin, vin, kout,
                   vout, sc.seg_start[cur], sc.seg_len[cur], sc.tbase, sc.tile_seg, T, shift,
                   sc.hist);
        SPX_LAUNCH("msd_next_level", k_msd_next_level, dim3(1), dim3(1), 0, s, ctr);
        const uint32_t meta = (uint32_t)(shift + RS_RADIX_BITS) | (out_code << 8);
        SPX_LAUNCH("msd_classify", k_msd_classify,
                   dim3(spx_div_up(nb, MSD_CLS_NT / SPX_WAVE)), dim3(MSD_CLS_NT), 0, s,
                   sc.seg_start[cur], sc.seg_len[cur], sc.tbase, nb, sc.hist, last ? 1 : 0, meta,
                   sc.seg_start[cur ^ 1], sc.seg_len[cur ^ 1], (uint32_t)sc.z.cap_big, sc.chunks,
                   (uint32_t)sc.z.cap_chunks, ctr);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
        e = msd_read(&h, ctr, s);
        if (e != hipSuccess) return e;
        if (h.err) {
            *failed = 1;
            return hipSuccess;
        }
        stats->split_keys += level_keys;
        stats->levels = p + 1;
        level_keys = h.bigkeys;
        nb = h.nbig;
        T = h.ntiles;
        ++p;
    }
    if (p == 0) h.nchunks = 1;  // E <= RS_LOCAL_MAX: the single chunk written by k_msd_init
    if (nb > 0) {
        // large segments with no varying digit left (a first level on a digit that turned out
        // to be the last varying one): equal keys, copied from the last level's output
        const uint32_t meta = 64u | (((p - 1) & 1) ? 2u : 1u) << 8;
        SPX_LAUNCH("msd_flush", k_msd_flush, dim3(spx_div_up(nb, 256)), dim3(256), 0, s,
                   sc.seg_start[p & 1], sc.seg_len[p & 1], nb, meta, sc.chunks,
                   (uint32_t)sc.z.cap_chunks, ctr);
        e = msd_read(&h, ctr, s);
        if (e != hipSuccess) return e;
        if (h.err) {
            *failed = 1;
            return hipSuccess;
        }
    }
    if (h.nchunks > 0) {
        SPX_LAUNCH("msd_local", k_msd_local, dim3(h.nchunks), dim3(MSD_LNT), 0, s, sc.chunks,
                   (const uint64_t*)k0, vfirst, (const uint64_t*)v0, k1, v1, head_tiles);
        if (head_tiles) {
            SPX_LAUNCH("msd_heads_first", k_msd_heads_first, dim3(spx_div_up(h.nchunks, 256)),
                       dim3(256), 0, s, sc.chunks, h.nchunks, (const uint64_t*)k1, head_tiles);
            if (heads_counted) *heads_counted = 1;
        }
    }
    *keys_sorted = k1;
    *vals_sorted = v1;
    return hipGetLastError();
}

// ------------------------------------------------------------------ repeats, gather, offsets

struct LoadHead {
    const uint64_t* keys;
    __device__ uint32_t operator()(int64_t i) const {
        return (i == 0 || keys[i] != keys[i - 1]) ? 1u : 0u;
    }
};
hipError_t launch_head_tiles_scan(uint32_t* tile_counts, int64_t E, uint32_t* total,
                                  hipStream_t s) {
    SPX_LAUNCH("scan_tile_sums", (scan_tile_sums<uint32_t, OpSum<uint32_t>>), dim3(1),
               dim3(SCAN_NT), 0, s, tile_counts, spx_div_up(E, SCAN_TILE), total);
    return hipGetLastError();
}

hipError_t launch_dedup_count(const uint64_t* keys, int64_t E, uint32_t* tile_sums,
                              uint32_t* total, hipStream_t s) {
    return scan_phase12<uint32_t, OpSum<uint32_t>>(LoadHead{keys}, E, tile_sums, total, s);
}

// Output entry u covers sorted positions [s, e): s = head_pos[u] (or u without summing), e the
// next head (or E).  Its value is vals[s] + vals[s+1] + ... in increasing position, i.e. in
// increasing triplet index, because the sort that carried the values is stable.  The last entry
// of each row (block) writes u+1 at its row (block), for the max-scan that follows.
// MODE 0: CRS (column index), 1: CSB Hilbert, 2: CSB Z-Morton (packed local row/column),
// 5: CSBR (the low 32 bits of the key are the packed (column rank, row rank) position inside the
// block)
template <int MODE>
__global__ __launch_bounds__(256) void k_gather(const uint64_t* __restrict__ keys,
                                                const double* __restrict__ vals,
                                                const int32_t* __restrict__ head_pos, int64_t E,
                                                int64_t nnz_out, int shiftbits, HotMap hm,
                                                int32_t* __restrict__ idx_out,
                                                double* __restrict__ val_out,
                                                int32_t* __restrict__ ends) {
    for (int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; u < nnz_out;
         u += (int64_t)gridDim.x * blockDim.x) {
        const int64_t s = head_pos ? head_pos[u] : u;
        const int64_t e = head_pos ? (u + 1 < nnz_out ? (int64_t)head_pos[u + 1] : E) : u + 1;
        const uint64_t key = keys[s];
        double acc = vals[s];
        for (int64_t j = s + 1; j < e; ++j) acc = acc + vals[j];
        val_out[u] = acc;
        const uint64_t major = key >> shiftbits;
        if (MODE == 5) {
            idx_out[u] = (int32_t)(uint32_t)(key & ((1ull << shiftbits) - 1ull));
        } else if (MODE != 0) {
            const int k = shiftbits >> 1;
            const uint32_t d = (uint32_t)(key & ((1ull << shiftbits) - 1ull));
            uint32_t lc, lr;
            if (MODE == 1) hilbert_d2xy(k, d, &lc, &lr);
            else zmorton_d2xy(k, d, &lc, &lr);
            idx_out[u] = (int32_t)((lr << 16) | lc);
        } else {
            idx_out[u] = hm.map((uint32_t)(key & ((1ull << shiftbits) - 1ull)));
        }
        const bool last = (e >= E) || ((keys[e] >> shiftbits) != major);
        if (last) ends[major] = (int32_t)(u + 1);
    }
}

hipError_t launch_gather_csr(const uint64_t* keys, const double* vals, const int32_t* head_pos,
                             int64_t E, int64_t nnz_out, int cbits, HotMap hm, int32_t* col_out,
                             double* val_out, int32_t* row_end, hipStream_t s) {
    if (nnz_out <= 0) return hipSuccess;
    SPX_LAUNCH("gather", (k_gather<0>), dim3(grid_for(nnz_out, 256)), dim3(256), 0, s, keys,
               vals, head_pos, E, nnz_out, cbits, hm, col_out, val_out, row_end);
    return hipGetLastError();
}

hipError_t launch_gather_csbr(const uint64_t* keys, const double* vals, const int32_t* head_pos,
                              int64_t E, int64_t nnz_out, uint32_t* packed_out, double* val_out,
                              int32_t* blk_end, hipStream_t s) {
    if (nnz_out <= 0) return hipSuccess;
    SPX_LAUNCH("gather", (k_gather<5>), dim3(grid_for(nnz_out, 256)), dim3(256), 0, s, keys, vals,
               head_pos, E, nnz_out, 32, HotMap{}, (int32_t*)packed_out, val_out, blk_end);
    return hipGetLastError();
}

hipError_t launch_gather_csb(const uint64_t* keys, const double* vals, const int32_t* head_pos,
                             int64_t E, int64_t nnz_out, int k, bool hilbert, uint32_t* packed_out,
                             double* val_out, int32_t* blk_end, hipStream_t s) {
    if (nnz_out <= 0) return hipSuccess;
    if (hilbert)
        SPX_LAUNCH("gather", (k_gather<1>), dim3(grid_for(nnz_out, 256)), dim3(256), 0, s, keys,
                   vals, head_pos, E, nnz_out, 2 * k, HotMap{}, (int32_t*)packed_out, val_out,
                   blk_end);
    else
        SPX_LAUNCH("gather", (k_gather<2>), dim3(grid_for(nnz_out, 256)), dim3(256), 0, s, keys,
                   vals, head_pos, E, nnz_out, 2 * k, HotMap{}, (int32_t*)packed_out, val_out,
                   blk_end);
    return hipGetLastError();
}

// Fused repeat summing + populate.  Workgroup b owns the sorted positions of scan tile b (the
// same SCAN_TILE tiling as launch_dedup_count, whose scanned tile counts give each tile's first
// output index).  The tile's keys are staged in LDS and every item's value is loaded up front;
// run heads are ranked by ballots in strided item order (each ballot covers 64 consecutive
// positions, so the ballots also form the tile's head bitmap).  Each head writes its index and
// marks the end of its row (block) for the max-scan; its value is the run's sum in increasing
// position (= increasing triplet index, the sort being stable), formed strictly left to right:
//   * a run of at most DG_SHORT entries that ends inside the tile is summed by its head thread
//     (loads issued four at a time ahead of the additions);
//   * every other run (longer, or reaching past the tile) is summed by one wave: 64 positions are
//     loaded at a time and one chain of additions walks them in order, up to the end of the run,
//     wherever that is.
// So a run of length L costs O(L) chained additions on one wave and O(L / 64) loads.
#ifndef DG_NT
#define DG_NT 1024
#endif
#define DG_IPT (SCAN_TILE / DG_NT)
#define DG_TILE SCAN_TILE
#define DG_SHORT 16
#define DG_LONG_MAX 256
static_assert(DG_TILE / (DG_SHORT + 1) + 1 <= DG_LONG_MAX, "list of the tile's long runs");
static_assert(DG_TILE == DG_IPT * DG_NT && DG_NT % SPX_WAVE == 0, "tile layout");
static_assert(DG_IPT * (DG_NT / SPX_WAVE) == SPX_WAVE, "one wave scans the (row, wave) counts");

__device__ __forceinline__ double dg_lane(double v, int k) {  // v of lane k (k wave-uniform)
    const int lo = __builtin_amdgcn_readlane(__double2loint(v), k);
    const int hi = __builtin_amdgcn_readlane(__double2hiint(v), k);
    return __hiloint2double(hi, lo);
}

template <int MODE>
__device__ __forceinline__ void dg_mark_end(int32_t* ends, uint64_t key, int shiftbits, int64_t u,
                                            bool more, uint64_t next) {
    if (MODE == 3 || MODE == 4) return;  // block starts are marked by the head
    const uint64_t major = key >> shiftbits;
    if (!more || (next >> shiftbits) != major) ends[major] = (int32_t)(u + 1);
}

template <int MODE>
__global__ __launch_bounds__(DG_NT) void k_dedup_gather(
    const uint64_t* __restrict__ keys, const double* __restrict__ vals, int64_t E,
    const uint32_t* __restrict__ tile_off, int shiftbits, HotMap hm,
    int32_t* __restrict__ idx_out, double* __restrict__ val_out, int32_t* __restrict__ ends,
    int K, uint64_t* __restrict__ majors) {
    constexpr int NW = DG_NT / SPX_WAVE;
    constexpr int NWORDS = DG_TILE / SPX_WAVE;
    __shared__ uint64_t s_key[DG_TILE + 1];  // s_key[i+1] = keys[base+i]
    __shared__ uint32_t s_pre[DG_IPT][NW];   // heads before (row j, wave w) within the tile
    __shared__ uint64_t s_hb[NWORDS];        // head bitmap: bit i & 63 of word i >> 6
    __shared__ uint32_t s_long_i[DG_LONG_MAX], s_long_u[DG_LONG_MAX];
    __shared__ uint32_t s_nlong;
    const int tid = threadIdx.x;
    const int w = tid / SPX_WAVE;
    const int lane = __lane_id();
    const int64_t base = (int64_t)blockIdx.x * DG_TILE;
    const int64_t rem = E - base;
    const int cnt = rem < DG_TILE ? (int)rem : DG_TILE;
    // keys staged in LDS; every item's own value loaded up front (coalesced, all in flight)
    double v[DG_IPT];
#pragma unroll
    for (int j = 0; j < DG_IPT; ++j) {
        const int i = tid + j * DG_NT;
        if (i < cnt) s_key[i + 1] = keys[base + i];
        v[j] = i < cnt ? vals[base + i] : 0.0;
    }
    if (tid == 0) {
        s_key[0] = base > 0 ? keys[base - 1] : ~keys[0];  // position 0 is a head
        s_nlong = 0;
    }
    __syncthreads();
    // output index of each head: heads are ranked in item order i = tid + j * DG_NT, so a
    // ballot per (row j, wave) and a prefix over the DG_IPT x NW wave counts suffice
    const uint64_t lt = spx_lanemask_lt();
    uint32_t rank[DG_IPT];
    uint32_t heads = 0;
#pragma unroll
    for (int j = 0; j < DG_IPT; ++j) {
        const int i = tid + j * DG_NT;
        const bool head = i < cnt && s_key[i + 1] != s_key[i];
        const uint64_t bal = __ballot(head);
        rank[j] = (uint32_t)__popcll(bal & lt);
        heads |= (head ? 1u : 0u) << j;
        if (lane == 0) {
            s_pre[j][w] = (uint32_t)__popcll(bal);
            s_hb[j * NW + w] = bal;  // positions [j * DG_NT + 64 w, +64)
        }
    }
    const uint64_t lowmask = (1ull << shiftbits) - 1ull;
    // CRS: the hot-column map words of every head, all loads in flight across the prefix scan
    uint4 hw[DG_IPT];
#pragma unroll
    for (int j = 0; j < DG_IPT; ++j) {
        hw[j] = make_uint4(0u, 0u, 0u, 0u);
        if (MODE == 0 && ((heads >> j) & 1u))
            hw[j] = hm.word((uint32_t)(s_key[tid + j * DG_NT + 1] & lowmask));
    }
    __syncthreads();
    if (w == 0) {  // exclusive prefix over the DG_IPT x NW counts in (row, wave) order
        const uint32_t c = s_pre[lane / NW][lane % NW];
        const uint32_t incl = wave_incl_scan<uint32_t, OpSum<uint32_t>>(c);
        s_pre[lane / NW][lane % NW] = tile_off[blockIdx.x] + incl - c;
    }
    __syncthreads();
#pragma unroll
    for (int j = 0; j < DG_IPT; ++j) {
        if (!((heads >> j) & 1u)) continue;
        const int i = tid + j * DG_NT;
        const uint64_t key = s_key[i + 1];
        const int64_t u = s_pre[j][w] + rank[j];
        // end of the run inside the tile: the next head, else the tile's end
        int e = cnt;
        {
            int wi = i >> 6;
            uint64_t b = (i & 63) == 63 ? 0ull : s_hb[wi] & (~0ull << ((i & 63) + 1));
            while (b == 0ull && ++wi < NWORDS) b = s_hb[wi];
            if (b != 0ull) e = wi * 64 + __builtin_ctzll(b);
        }
        const bool more = base + e < E;
        const uint64_t next = e < cnt ? s_key[e + 1] : (more ? keys[base + e] : 0ull);
        if ((!more || next != key) && e - i <= DG_SHORT) {
            double acc = v[j];
            for (int q0 = i + 1; q0 < e; q0 += 4) {  // four loads in flight, then add in order
                double t[4];
#pragma unroll
                for (int q = 0; q < 4; ++q) t[q] = q0 + q < e ? vals[base + q0 + q] : 0.0;
#pragma unroll
                for (int q = 0; q < 4; ++q)
                    if (q0 + q < e) acc = acc + t[q];
            }
            val_out[u] = acc;
            dg_mark_end<MODE>(ends, key, shiftbits, u, more, next);
        } else {
            const uint32_t slot = atomicAdd(&s_nlong, 1u);
            s_long_i[slot] = (uint32_t)i;
            s_long_u[slot] = (uint32_t)u;
        }
        const uint64_t major = key >> shiftbits;
        const uint32_t d = (uint32_t)(key & lowmask);
        if (MODE == 5) {  // CSBR: the packed position is the key's low half
            idx_out[u] = (int32_t)d;
        } else if (MODE == 3 || MODE == 4) {  // BCOHC / BCOHCH: packed local position, block-start flag
            const int k = shiftbits >> 1;
            const uint32_t mask = (1u << k) - 1u;
            uint32_t lc, lr;
            if (MODE == 3) {
                lr = d >> k;
                lc = d & mask;
            } else {
                uint32_t x, y;
                hilbert_d2xy64(K, key & ((1ull << (2 * K)) - 1ull), &x, &y);
                lr = y & mask;
                lc = x & mask;
            }
            idx_out[u] = (int32_t)((lr << 16) | lc);
            const bool bstart = (s_key[i] >> shiftbits) != major;
            ends[u] = bstart ? 1 : 0;
            if (bstart) majors[u] = major;
        } else if (MODE != 0) {
            const int k = shiftbits >> 1;
            uint32_t lc, lr;
            if (MODE == 1) hilbert_d2xy(k, d, &lc, &lr);
            else zmorton_d2xy(k, d, &lc, &lr);
            idx_out[u] = (int32_t)((lr << 16) | lc);
        } else {
            idx_out[u] = hm.words ? hm.map_word(d, hw[j]) : (int32_t)d;
        }
    }
    __syncthreads();
    // the tile's long runs, one wave each: chunks of 64 positions, one chain of additions
    const uint32_t nlong = s_nlong;
    for (uint32_t r = w; r < nlong; r += NW) {
        const int64_t p0 = base + s_long_i[r];
        const int64_t u = s_long_u[r];
        const uint64_t key = s_key[s_long_i[r] + 1];
        int64_t p = p0;
        uint64_t kc = p + lane < E ? keys[p + lane] : ~key;
        double vc = p + lane < E ? vals[p + lane] : 0.0;
        double acc = dg_lane(vc, 0);  // position p0 is the head itself
        int k0 = 1;
        bool more;
        uint64_t next;
        for (;;) {
            const uint64_t match = __ballot(kc == key);
            const int n1 = ~match == 0ull ? 64 : __builtin_ctzll(~match);  // leading run lanes
            uint64_t kn = ~key;
            double vn = 0.0;
            if (n1 == 64) {  // the run fills the chunk: fetch the next one before adding
                kn = p + 64 + lane < E ? keys[p + 64 + lane] : ~key;
                vn = p + 64 + lane < E ? vals[p + 64 + lane] : 0.0;
            }
            for (int k = k0; k < n1; ++k) acc = acc + dg_lane(vc, k);
            k0 = 0;
            if (n1 < 64) {
                more = p + n1 < E;
                const int lo = __builtin_amdgcn_readlane((int)(uint32_t)kc, n1);
                const int hi = __builtin_amdgcn_readlane((int)(uint32_t)(kc >> 32), n1);
                next = ((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo;
                break;
            }
            p += 64;
            kc = kn;
            vc = vn;
        }
        if (lane == 0) {
            val_out[u] = acc;
            dg_mark_end<MODE>(ends, key, shiftbits, u, more, next);
        }
    }
}

hipError_t launch_dedup_gather(const uint64_t* keys, const double* vals, int64_t E,
                               const uint32_t* tile_sums, int mode, int shiftbits, HotMap hm,
                               int32_t* idx_out, double* val_out, int32_t* ends, hipStream_t s,
                               int K, uint64_t* majors) {
    if (E <= 0) return hipSuccess;
    const unsigned g = spx_div_up(E, DG_TILE);
#define DG_CASE(M)                                                                              \
    case M:                                                                                     \
        SPX_LAUNCH("dedup_gather", (k_dedup_gather<M>), dim3(g), dim3(DG_NT), 0, s, keys, vals, \
                   E, tile_sums, shiftbits, hm, idx_out, val_out, ends, K, majors);             \
        break;
    switch (mode) {
        DG_CASE(0)
        DG_CASE(1)
        DG_CASE(2)
        DG_CASE(3)
        DG_CASE(4)
        DG_CASE(5)
        default: return hipErrorInvalidValue;
    }
#undef DG_CASE
    return hipGetLastError();
}

struct LoadI32 {
    const int32_t* p;
    __device__ int32_t operator()(int64_t i) const { return p[i]; }
};
struct StoreInclI32 {
    int32_t* p;
    __device__ void operator()(int64_t i, int32_t incl, int32_t) const { p[i] = incl; }
};

hipError_t launch_max_scan_i32(int32_t* ends, int64_t len, uint32_t* tile_sums, hipStream_t s) {
    if (len <= 0) return hipSuccess;
    int32_t* ts = (int32_t*)tile_sums;
    hipError_t e = scan_phase12<int32_t, OpMax<int32_t>>(LoadI32{ends}, len, ts, (int32_t*)nullptr,
                                                         s);
    if (e != hipSuccess) return e;
    return scan_phase3<int32_t, OpMax<int32_t>>(LoadI32{ends}, StoreInclI32{ends}, len, ts, s);
}
