// k_bcoh.hip -- BCOHC / BCOHCH: row-distributed blocks with compressed triplets (gfx950).
//
// The paper's workers (threads with a static share of rows of about equal entry count) become
// partitions, one workgroup each.  A partition is a range of whole rows of at most BH_WINDOW
// rows, so its output rows live in LDS for the whole product; its beta x beta blocks are stored
// in Hilbert order, and inside a block the entries are packed (local_row << 16) | local_col in
// row-wise order (BCOHC) or in the order of the Hilbert curve over the partition (BCOHCH).  The
// block level keeps an explicit (block row, block column) per block and the first entry of each
// block, where the paper keeps BICRS increments (which a single thread decodes in sequence).
#include "dev_common.h"
#include "dev_curves.h"
#include "dev_scan.h"
#include "dev_values.h"
#include "spx_internal.h"

// ------------------------------------------------------------------ conversion

struct LoadU32B {
    const uint32_t* p;
    __device__ uint32_t operator()(int64_t i) const { return p[i]; }
};

struct StoreExclU32B {
    uint32_t* p;
    __device__ void operator()(int64_t i, uint32_t incl, uint32_t item) const {
        p[i] = incl - item;
    }
};

// Raw entries per row without one global atomic per entry (random atomics run at about 20 G/s
// on this chip, so counting 2^28 entries that way costs ~14 ms): rows are bucketed by r >> wbits
// (at most RC_BUCKETS buckets of 2^wbits <= 2^RC_WBITS_MAX rows) with one counting pass over
// tiles of RC_TILE entries and one scatter of the row indices; then every bucket is counted in
// LDS, in slices of about RC_SLICE entries (at most RC_SLICES per bucket), and written with plain
// stores (one slice) or atomics (several).
#define RC_TILE 65536
#define RC_NT 1024
#define RC_BUCKETS 4096
#define RC_WBITS_MAX 14
#define RC_SLICE (1 << 18)
#define RC_SLICES 16

// Buckets are as wide as the count's LDS allows (fewer buckets: longer runs per bucket in each
// tile of the scatter, hence whole-line stores), narrower only when the rows fit fewer bits.
int bcoh_row_bucket_bits(int32_t m) {  // -1: too many rows for the bucketed count
    int w = 0;
    while (w < RC_WBITS_MAX && (1ll << w) < (int64_t)m) ++w;
    return (((int64_t)m + (1ll << w) - 1) >> w) <= RC_BUCKETS ? w : -1;
}

__global__ __launch_bounds__(RC_NT) void k_rowc_hist(const int32_t* __restrict__ row,
                                                     const int32_t* __restrict__ col, int64_t E,
                                                     int32_t m, int32_t n, int wbits, int nbk,
                                                     int64_t T, uint32_t* __restrict__ hist,
                                                     uint32_t* __restrict__ err) {
    __shared__ uint32_t cnt[RC_BUCKETS];
    for (int i = threadIdx.x; i < nbk; i += RC_NT) cnt[i] = 0;
    __syncthreads();
    const int64_t t = blockIdx.x;
    const int64_t lo = t * RC_TILE;
    const int64_t hi = lo + RC_TILE < E ? lo + RC_TILE : E;
    uint32_t bad = 0;
    for (int64_t i = lo + threadIdx.x; i < hi; i += RC_NT) {
        const int32_t r = row[i], c = col[i];
        const bool ok = (r >= 0) & (r < m) & (c >= 0) & (c < n);
        if (ok) atomicAdd(&cnt[r >> wbits], 1u);
        bad |= ok ? 0u : 1u;
    }
    if (__ballot(bad != 0) && __lane_id() == 0) atomicOr(err, 1u);
    __syncthreads();
    for (int b = threadIdx.x; b < nbk; b += RC_NT) hist[(int64_t)b * T + t] = cnt[b];
}

// rows_out[pos] = the row, or with_aux: (row mod 2^wbits) | aux << wbits with aux =
// map[col] >> aux_shift (map NULL: col >> aux_shift); the count needs only the row's position in
// its bucket.  keep (nullable, with a map) receives map[col] at the entry's own index.
// The scatter stages each sub-tile of RC_SUB entries in LDS grouped by bucket (a count, an
// exclusive scan and a placement), then writes every bucket's run of the sub-tile to consecutive
// output positions, so that the stores of a wave land on few lines; placing each entry straight
// from its LDS cursor spread a wave's stores over as many partly written lines as it has lanes.
#define RC_SUB (RC_NT * 8)
__global__ __launch_bounds__(RC_NT) void k_rowc_scatter(const int32_t* __restrict__ row,
                                                        const int32_t* __restrict__ col,
                                                        int64_t E, int32_t m, int32_t n,
                                                        int wbits, int nbk, int64_t T,
                                                        const uint32_t* __restrict__ hist,
                                                        int32_t* __restrict__ rows_out,
                                                        int with_aux, int aux_shift,
                                                        const int32_t* __restrict__ aux_map,
                                                        int32_t* __restrict__ keep) {
    static_assert(RC_BUCKETS == 4 * RC_NT, "the scan takes four buckets per thread");
    static_assert(RC_BUCKETS <= 65536, "staged bucket numbers are 16-bit");
    constexpr int U = RC_SUB / RC_NT;
    const uint32_t wmask = (1u << wbits) - 1u;
    __shared__ uint32_t cur[RC_BUCKETS];      // this tile's next output position of each bucket
    __shared__ uint32_t off[RC_BUCKETS + 1];  // a sub-tile's counts, then their exclusive prefix
    __shared__ int32_t stage[RC_SUB];         // the sub-tile's values grouped by bucket
    __shared__ uint16_t sbk[RC_SUB];          // the bucket of each staged value
    __shared__ uint32_t wtot[RC_NT / 64];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int64_t t = blockIdx.x;
    for (int b = tid; b < nbk; b += RC_NT) cur[b] = hist[(int64_t)b * T + t];
    const int64_t lo = t * RC_TILE;
    const int64_t hi = lo + RC_TILE < E ? lo + RC_TILE : E;
    for (int64_t s0 = lo; s0 < hi; s0 += RC_SUB) {
        for (int b = tid; b <= nbk; b += RC_NT) off[b] = 0;
        __syncthreads();
        int32_t r[U], c[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {  // every load of the sub-tile in flight together
            const int64_t i = s0 + u * RC_NT + tid;
            r[u] = i < hi ? row[i] : -1;
            c[u] = i < hi ? col[i] : -1;
        }
        int32_t v[U];
        int bk[U];
        uint32_t rk[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t i = s0 + u * RC_NT + tid;
            const bool ok = (i < hi) & (r[u] >= 0) & (r[u] < m) & (c[u] >= 0) & (c[u] < n);
            bk[u] = ok ? (r[u] >> wbits) : -1;
            v[u] = r[u];
            rk[u] = 0;
            if (ok) {
                if (with_aux) {
                    const int32_t mc = aux_map ? aux_map[c[u]] : c[u];
                    if (keep) keep[i] = mc;
                    v[u] = (int32_t)(((uint32_t)r[u] & wmask) |
                                     ((uint32_t)(mc >> aux_shift) << wbits));
                }
                rk[u] = atomicAdd(&off[bk[u]], 1u);
            }
        }
        __syncthreads();
        {  // exclusive scan of the counts: four buckets per thread, then waves, then the block
            uint32_t a[4], sum = 0;
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int b = tid * 4 + j;
                a[j] = b < nbk ? off[b] : 0u;
                sum += a[j];
            }
            uint32_t x = sum;
#pragma unroll
            for (int d = 1; d < 64; d <<= 1) {
                const uint32_t y = __shfl_up(x, d, 64);
                if (lane >= d) x += y;
            }
            if (lane == 63) wtot[wave] = x;
            __syncthreads();
            uint32_t base = 0;
            for (int w = 0; w < wave; ++w) base += wtot[w];
            uint32_t e = base + x - sum;
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                const int b = tid * 4 + j;
                if (b < nbk) off[b] = e;
                e += a[j];
            }
            if (tid == RC_NT - 1) off[nbk] = base + x;
        }
        __syncthreads();
#pragma unroll
        for (int u = 0; u < U; ++u) {
            if (bk[u] >= 0) {
                const uint32_t p = off[bk[u]] + rk[u];
                stage[p] = v[u];
                sbk[p] = (uint16_t)bk[u];
            }
        }
        __syncthreads();
        const uint32_t ns = off[nbk];
        for (uint32_t j = tid; j < ns; j += RC_NT) {
            const int b = sbk[j];
            rows_out[cur[b] + (j - off[b])] = stage[j];
        }
        __syncthreads();
        for (int b = tid; b < nbk; b += RC_NT) cur[b] += off[b + 1] - off[b];
        __syncthreads();
    }
}

// Workgroup (bucket b, slice q): positions [start_b, end_b) of rows_out hold bucket b's rows.
__global__ __launch_bounds__(RC_NT) void k_rowc_count(const int32_t* __restrict__ rows_out,
                                                      const uint32_t* __restrict__ hist,
                                                      const uint32_t* __restrict__ total,
                                                      int64_t T, int nbk, int wbits, int32_t m,
                                                      uint32_t* __restrict__ counts) {
    __shared__ uint32_t c[1 << RC_WBITS_MAX];
    const int b = blockIdx.x / RC_SLICES, q = blockIdx.x % RC_SLICES;
    const int64_t start = hist[(int64_t)b * T];
    const int64_t end = b + 1 < nbk ? (int64_t)hist[(int64_t)(b + 1) * T] : (int64_t)*total;
    const int64_t len = end - start;
    int slices = (int)((len + RC_SLICE - 1) / RC_SLICE);
    if (slices < 1) slices = 1;
    if (slices > RC_SLICES) slices = RC_SLICES;
    if (q >= slices) return;  // uniform over the workgroup
    const int W = 1 << wbits;
    for (int i = threadIdx.x; i < W; i += RC_NT) c[i] = 0;
    __syncthreads();
    const int64_t s0 = start + len * q / slices, s1 = start + len * (q + 1) / slices;
    int64_t i = s0 + threadIdx.x;
    for (; i + 3 * RC_NT < s1; i += 4 * RC_NT) {  // four loads in flight per thread
        int32_t v[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) v[u] = rows_out[i + u * RC_NT];
#pragma unroll
        for (int u = 0; u < 4; ++u) atomicAdd(&c[v[u] & (W - 1)], 1u);
    }
    for (; i < s1; i += RC_NT) atomicAdd(&c[rows_out[i] & (W - 1)], 1u);
    __syncthreads();
    const int64_t r0 = (int64_t)b << wbits;
    for (int i = threadIdx.x; i < W; i += RC_NT) {
        if (r0 + i >= m) break;
        if (slices == 1) counts[r0 + i] = c[i];
        else if (c[i]) atomicAdd(&counts[r0 + i], c[i]);
    }
}

// Workgroup (bucket b, slice q) as in k_rowc_count, over entries scattered with their aux value
// (row mod 2^wbits | aux << wbits): the least and greatest aux value of every row of the bucket
// (lo / hi, which start at 0xFFFFFFFF / 0), in LDS, then stored (one slice) or merged by
// atomics (several).  Dynamic LDS: 2 * 2^wbits words.
__global__ __launch_bounds__(RC_NT) void k_rowc_extent(const int32_t* __restrict__ rows_out,
                                                       const uint32_t* __restrict__ hist,
                                                       const uint32_t* __restrict__ total,
                                                       int64_t T, int nbk, int wbits, int32_t m,
                                                       uint32_t* __restrict__ lo,
                                                       uint32_t* __restrict__ hi) {
    extern __shared__ uint32_t s_ext[];
    const int W = 1 << wbits;
    uint32_t* s_lo = s_ext;
    uint32_t* s_hi = s_ext + W;
    const int b = blockIdx.x / RC_SLICES, q = blockIdx.x % RC_SLICES;
    const int64_t start = hist[(int64_t)b * T];
    const int64_t end = b + 1 < nbk ? (int64_t)hist[(int64_t)(b + 1) * T] : (int64_t)*total;
    const int64_t len = end - start;
    int slices = (int)((len + RC_SLICE - 1) / RC_SLICE);
    if (slices < 1) slices = 1;
    if (slices > RC_SLICES) slices = RC_SLICES;
    if (q >= slices) return;  // uniform over the workgroup
    for (int i = threadIdx.x; i < W; i += RC_NT) {
        s_lo[i] = 0xFFFFFFFFu;
        s_hi[i] = 0u;
    }
    __syncthreads();
    const int64_t s0 = start + len * q / slices, s1 = start + len * (q + 1) / slices;
    int64_t i = s0 + threadIdx.x;
    for (; i + 3 * RC_NT < s1; i += 4 * RC_NT) {  // four entries in flight per thread
        uint32_t v[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) v[u] = (uint32_t)rows_out[i + u * RC_NT];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            atomicMin(&s_lo[v[u] & (W - 1)], v[u] >> wbits);
            atomicMax(&s_hi[v[u] & (W - 1)], v[u] >> wbits);
        }
    }
    for (; i < s1; i += RC_NT) {
        const uint32_t v = (uint32_t)rows_out[i];
        atomicMin(&s_lo[v & (W - 1)], v >> wbits);
        atomicMax(&s_hi[v & (W - 1)], v >> wbits);
    }
    __syncthreads();
    const int64_t r0 = (int64_t)b << wbits;
    for (int j = threadIdx.x; j < W; j += RC_NT) {
        if (r0 + j >= m) break;
        if (slices == 1) {
            lo[r0 + j] = s_lo[j];
            hi[r0 + j] = s_hi[j];
        } else if (s_lo[j] != 0xFFFFFFFFu) {
            atomicMin(&lo[r0 + j], s_lo[j]);
            atomicMax(&hi[r0 + j], s_hi[j]);
        }
    }
}

hipError_t rowc_extent_prepare_kernel() {
    return hipFuncSetAttribute((const void*)k_rowc_extent,
                               hipFuncAttributeMaxDynamicSharedMemorySize,
                               (int)(2 * sizeof(uint32_t) << RC_WBITS_MAX));
}

hipError_t launch_bcoh_rows_bucketed(const int32_t* row, const int32_t* col, int64_t E,
                                     int32_t m, int32_t n, int wbits, uint32_t* hist,
                                     int32_t* rows_out, uint32_t* tile_sums, uint32_t* total,
                                     uint32_t* counts, uint32_t* err, hipStream_t s,
                                     int aux_shift, uint32_t* lo, uint32_t* hi,
                                     const int32_t* aux_map, int32_t* aux_keep) {
    if (E <= 0) return hipSuccess;
    const int nbk = (int)(((int64_t)m + (1ll << wbits) - 1) >> wbits);
    const int64_t T = (E + RC_TILE - 1) / RC_TILE;
    SPX_LAUNCH("bcoh_rows_hist", k_rowc_hist, dim3((unsigned)T), dim3(RC_NT), 0, s, row, col, E,
               m, n, wbits, nbk, T, hist, err);
    const int64_t hn = (int64_t)nbk * T;
    hipError_t e = scan_phase12<uint32_t, OpSum<uint32_t>>(LoadU32B{hist}, hn, tile_sums, total, s);
    if (e != hipSuccess) return e;
    e = scan_phase3<uint32_t, OpSum<uint32_t>>(LoadU32B{hist}, StoreExclU32B{hist}, hn, tile_sums,
                                               s);
    if (e != hipSuccess) return e;
    SPX_LAUNCH("bcoh_rows_scatter", k_rowc_scatter, dim3((unsigned)T), dim3(RC_NT), 0, s, row,
               col, E, m, n, wbits, nbk, T, hist, rows_out, lo != nullptr ? 1 : 0, aux_shift,
               aux_map, aux_keep);
    SPX_LAUNCH("bcoh_rows_count", k_rowc_count, dim3((unsigned)(nbk * RC_SLICES)), dim3(RC_NT), 0,
               s, rows_out, hist, total, T, nbk, wbits, m, counts);
    if (lo != nullptr)
        SPX_LAUNCH("bcoh_rows_extent", k_rowc_extent, dim3((unsigned)(nbk * RC_SLICES)),
                   dim3(RC_NT), (2 * sizeof(uint32_t)) << wbits, s, rows_out, hist, total, T, nbk,
                   wbits, m, lo, hi);
    return hipGetLastError();
}

size_t bcoh_rows_hist_elems(int32_t m, int64_t E, int wbits) {
    const int64_t nbk = ((int64_t)m + (1ll << wbits) - 1) >> wbits;
    return (size_t)(nbk * ((E + RC_TILE - 1) / RC_TILE));
}

// Row r starts a partition when it is row 0, a multiple of BH_WINDOW, or when the raw entries
// before it and before row r - 1 lie in different multiples of the target count.
struct LoadPartStart {
    const uint32_t* cum;
    uint32_t target;
    __device__ uint32_t operator()(int64_t r) const {
        if (r == 0 || r % BH_WINDOW == 0) return 1u;
        return (cum[r] / target) != (cum[r - 1] / target) ? 1u : 0u;
    }
};
struct StorePart {
    int32_t* part_of;
    int32_t* part_row;
    __device__ void operator()(int64_t r, uint32_t incl, uint32_t item) const {
        part_of[r] = (int32_t)incl - 1;
        if (item) part_row[incl - 1] = (int32_t)r;
    }
};

hipError_t launch_bcoh_partitions(const uint32_t* cum, int32_t m, uint32_t target,
                                  int32_t* part_of, int32_t* part_row, uint32_t* tile_sums,
                                  uint32_t* total, hipStream_t s) {
    const LoadPartStart ld{cum, target};
    hipError_t e = scan_phase12<uint32_t, OpSum<uint32_t>>(ld, m, tile_sums, total, s);
    if (e != hipSuccess) return e;
    return scan_phase3<uint32_t, OpSum<uint32_t>>(ld, StorePart{part_of, part_row}, m, tile_sums,
                                                  s);
}

struct StoreInclU32 {
    uint32_t* p;
    __device__ void operator()(int64_t i, uint32_t incl, uint32_t) const { p[i] = incl; }
};

hipError_t launch_incl_scan_u32(uint32_t* a, int64_t n, uint32_t* tile_sums, uint32_t* total,
                                hipStream_t s) {
    hipError_t e = scan_phase12<uint32_t, OpSum<uint32_t>>(LoadU32B{a}, n, tile_sums, total, s);
    if (e != hipSuccess) return e;
    return scan_phase3<uint32_t, OpSum<uint32_t>>(LoadU32B{a}, StoreInclU32{a}, n, tile_sums, s);
}

// Entry u starts a block when incl[u] exceeds incl[u-1]; the block's key (partition << 2*K2 |
// Hilbert block index) was stored at majors[u] by the populate step.
__global__ void k_bcoh_blocks(const uint32_t* __restrict__ incl,
                              const uint64_t* __restrict__ majors, int64_t nnz, int K2,
                              int32_t* __restrict__ blk_ptr, uint32_t* __restrict__ blk_coord,
                              int32_t* __restrict__ blk_part) {
    for (int64_t u = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; u < nnz;
         u += (int64_t)gridDim.x * blockDim.x) {
        const uint32_t c = incl[u];
        if (u > 0 && incl[u - 1] == c) continue;
        const uint32_t b = c - 1;
        const uint64_t mj = majors[u];
        const uint64_t hb = mj & ((1ull << (2 * K2)) - 1ull);
        uint32_t bc, br;
        hilbert_d2xy64(K2, hb, &bc, &br);
        blk_ptr[b] = (int32_t)u;
        blk_coord[b] = (br << 16) | bc;
        blk_part[b] = (int32_t)(mj >> (2 * K2));
    }
}

hipError_t launch_bcoh_blocks(const uint32_t* incl, const uint64_t* majors, int64_t nnz, int K2,
                              int32_t* blk_ptr, uint32_t* blk_coord, int32_t* blk_part,
                              hipStream_t s) {
    if (nnz <= 0) return hipSuccess;
    int64_t g = spx_div_up(nnz, 256);
    if (g > 65536) g = 65536;
    SPX_LAUNCH("bcoh_blocks", k_bcoh_blocks, dim3((unsigned)g), dim3(256), 0, s, incl, majors,
               nnz, K2, blk_ptr, blk_coord, blk_part);
    return hipGetLastError();
}

// part_blk[p] = first block whose partition is >= p (blocks are in partition order), p = 0..P
__global__ void k_bcoh_part_blk(const int32_t* __restrict__ blk_part, int64_t nb, int32_t P,
                                int32_t* __restrict__ part_blk) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p > P) return;
    int64_t lo = 0, hi = nb;
    while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if (blk_part[mid] < p) lo = mid + 1;
        else hi = mid;
    }
    part_blk[p] = (int32_t)lo;
}

hipError_t launch_bcoh_part_blk(const int32_t* blk_part, int64_t nb, int32_t P,
                                int32_t* part_blk, hipStream_t s) {
    SPX_LAUNCH("bcoh_part_blk", k_bcoh_part_blk, dim3(spx_div_up((int64_t)P + 1, 256)), dim3(256),
               0, s, blk_part, nb, P, part_blk);
    return hipGetLastError();
}

// ------------------------------------------------------------------ product
//
// Workgroup p owns the rows [part_row[p], part_row[p+1]) and their slice of y in LDS.  It reads
// the partition's entries in storage order, BH_NT consecutive entries per wave-row (loads of
// whole lines), BH_IPT rows in flight per thread; a thread's entries ascend, so it keeps the block
// of its last entry and moves forward (a few steps by walking the block pointers, a longer move by
// binary search); each product is added into the slice (LDS float atomics; BCOHC stores a block
// row by row, so neighbouring lanes often share a row, and such runs are summed across their
// lanes before one atomic each), and the slice is written to y at the end.  The partition's
// block pointers, and its block coordinates when they fit too, are staged in the LDS left over
// by the slice (BH_STAGE_WORDS words), so that the walk, which carries a dependence from one
// entry to the next, reads LDS instead of the L2.

#define BH_NT 512
#define BH_IPT 8
// LDS words after the output slice: two workgroups of 64 KiB + 16 KiB fill a CU's 160 KiB
#define BH_STAGE_WORDS 4096

// Most blocks whose pointers (nbk + 1 words) and coordinates (nbk words, after room for the
// pointers of that many blocks) both fit in `words` words.
__host__ __device__ constexpr int nbk_stage_max(int words) { return (words - 1) / 2; }

// Last block b in [b_from, b_end) with blk_ptr[b] <= k (blk_ptr[b_from] <= k < blk_ptr[b_end]).
__device__ __forceinline__ int bcoh_block_of(const int32_t* __restrict__ bp, int b_from, int b_end,
                                             int k) {
#pragma unroll
    for (int step = 0; step < 4; ++step) {
        if (b_from + 1 >= b_end || bp[b_from + 1] > k) return b_from;
        ++b_from;
    }
    int lo = b_from, hi = b_end - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (bp[mid] <= k) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

template <typename V, typename X>
__global__ __launch_bounds__(BH_NT) void k_spmv_bcoh(
    const int32_t* __restrict__ part_row, const int32_t* __restrict__ part_blk,
    const int32_t* __restrict__ blk_ptr, const uint32_t* __restrict__ blk_coord,
    const uint32_t* __restrict__ packed, const V* __restrict__ val,
    const X* __restrict__ x, X* __restrict__ y, int k) {
    extern __shared__ double s_y[];
    int32_t* s_bp = (int32_t*)(s_y + BH_WINDOW);  // nbk + 1 block pointers
    uint32_t* s_bc = (uint32_t*)(s_bp + nbk_stage_max(BH_STAGE_WORDS) + 1);  // nbk coordinates
    const int tid = threadIdx.x;
    const int p = blockIdx.x;
    const int r0 = part_row[p], rows = part_row[p + 1] - r0;
    const int b0 = part_blk[p], b1 = part_blk[p + 1];
    const int nbk = b1 - b0;
    const int e0 = blk_ptr[b0], e1 = blk_ptr[b1];
    const bool stage_bp = nbk + 1 <= BH_STAGE_WORDS;
    const bool stage_bc = nbk <= nbk_stage_max(BH_STAGE_WORDS);
    for (int i = tid; i < rows; i += BH_NT) s_y[i] = 0.0;
    if (stage_bp)
        for (int i = tid; i <= nbk; i += BH_NT) s_bp[i] = blk_ptr[b0 + i];
    if (stage_bc)
        for (int i = tid; i < nbk; i += BH_NT) s_bc[i] = blk_coord[b0 + i];
    __syncthreads();
    const int32_t* bp = stage_bp ? s_bp : blk_ptr + b0;  // partition-local block indices
    const uint32_t* bcs = stage_bc ? s_bc : blk_coord + b0;
    const uint32_t lmask = 0xFFFFu;
    using T = decltype(vget(val));  // arithmetic type of a product
    int b = 0;  // partition-local block of this thread's current entry
    uint32_t bc = nbk > 0 ? bcs[0] : 0u;
    for (int base = e0; base < e1; base += BH_NT * BH_IPT) {
        // matrix loads issued unconditionally (entries past e1 read entry e1 - 1 again and are
        // dropped), so none waits inside a branch
        int kc[BH_IPT];
#pragma unroll
        for (int q = 0; q < BH_IPT; ++q) kc[q] = min(base + q * BH_NT + tid, e1 - 1);
        uint32_t pk[BH_IPT];
        V raw[BH_IPT];
#pragma unroll
        for (int q = 0; q < BH_IPT; ++q) {
            pk[q] = ntload(packed + kc[q]);
            raw[q] = ntload(val + kc[q]);
        }
        T xv[BH_IPT];
        int rw[BH_IPT];
#pragma unroll
        for (int q = 0; q < BH_IPT; ++q) {
            xv[q] = (T)0;
            rw[q] = 0;
            if (base + q * BH_NT + tid < e1) {
                const int nb = bcoh_block_of(bp, b, nbk, kc[q]);
                if (nb != b) {
                    b = nb;
                    bc = bcs[b];
                }
                rw[q] = (int)((bc >> 16) << k) + (int)(pk[q] >> 16) - r0;
                xv[q] = (T)x[(int)((bc & lmask) << k) + (int)(pk[q] & lmask)];
            }
        }
#pragma unroll
        for (int q = 0; q < BH_IPT; ++q) {
            const int kk = base + q * BH_NT + tid;
            lds_add_runs(s_y, kk < e1 ? rw[q] : -1, (double)(vdec(raw[q]) * xv[q]));
        }
    }
    __syncthreads();
    for (int i = tid; i < rows; i += BH_NT) ntstore(y + r0 + i, (X)s_y[i]);
}

static constexpr size_t kBcohLds = (size_t)BH_WINDOW * sizeof(double) + BH_STAGE_WORDS * 4;

// The product's LDS exceeds the default 64 KiB limit of dynamic LDS: raised once per device, at
// conversion.
template <typename V, typename X>
static hipError_t bcoh_prepare_one() {
    return hipFuncSetAttribute((const void*)k_spmv_bcoh<V, X>,
                               hipFuncAttributeMaxDynamicSharedMemorySize, (int)kBcohLds);
}

hipError_t bcoh_prepare_kernel() {
    hipError_t e = bcoh_prepare_one<double, double>();
    if (e == hipSuccess) e = bcoh_prepare_one<float, float>();
    if (e == hipSuccess) e = bcoh_prepare_one<uint16_t, float>();
    return e;
}

template <typename V, typename X>
static hipError_t bcoh_run(const spx_matrix_s* A, const V* val, const X* x, X* y,
                           hipStream_t s) {
    if (A->bh_nparts <= 0) return hipSuccess;
    SPX_LAUNCH("spmv_bcoh", (k_spmv_bcoh<V, X>), dim3(A->bh_nparts), dim3(BH_NT), kBcohLds, s,
               A->bh_part_row, A->bh_part_blk, A->bh_blk_ptr, A->bh_blk_coord, A->packed, val,
               x, y, A->log2_beta);
    return hipGetLastError();
}

hipError_t spmv_bcoh(const spx_matrix_s* A, const double* x, double* y, hipStream_t s) {
    return bcoh_run<double, double>(A, A->val, x, y, s);
}

hipError_t spmv_bcoh_f32(const spx_matrix_s* A, const float* x, float* y, hipStream_t s) {
    if (A->value_type == SPX_F32)
        return bcoh_run<float, float>(A, (const float*)A->val_lp, x, y, s);
    return bcoh_run<uint16_t, float>(A, (const uint16_t*)A->val_lp, x, y, s);
}


hipError_t launch_excl_scan_u32(const uint32_t* in, uint32_t* out, int64_t n,
                                uint32_t* tile_sums, uint32_t* total, hipStream_t s) {
    hipError_t e = scan_phase12<uint32_t, OpSum<uint32_t>>(LoadU32B{in}, n, tile_sums, total, s);
    if (e != hipSuccess) return e;
    return scan_phase3<uint32_t, OpSum<uint32_t>>(LoadU32B{in}, StoreExclU32B{out}, n, tile_sums,
                                                  s);
}
