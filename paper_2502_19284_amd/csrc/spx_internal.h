// spx_internal.h -- handle layout and kernel launchers shared by the libspx sources.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <vector>

#include "../../include/spx.h"
#include "../../include/spx_batch.h"
#include "spx_prof.h"

// ------------------------------------------------------------------ tuning constants
// merge-path CRS: threads per tile and items (row ends + entries) per thread
#define MP_NT 256
#define MP_IPT 8
#define MP_TILE (MP_NT * MP_IPT)

// row-split CRS: a row block holds < RS_NNZ entries and <= RS_ROWS rows; rows longer than
// RS_LONG are split into chunks of RS_CHUNK entries whose partial sums are added in order
#define RS_NT 256
#define RS_LONG 1024
#define RS_NNZ 2048
#define RS_ROWS 1024
#define RS_CHUNK 4096

// CSBH: workgroup size and entries per thread per sweep; a work unit covers at most
// csbh_unit_nnz entries of one block row (default below, overridable by tile_items)
#define CB_NT 512
#define CB_IPT 8
#define CB_UNIT_DEFAULT (1 << 17)
#define CB_LDS_BUDGET (64 * 1024)    // bytes of the output slice kept in LDS
#define CB_BP_STAGE_MAX 8192         // block pointers staged in LDS when nbc+1 <= this

// CSBR: panels of 2^CR_PB row ranks (y slice in LDS: 128 KiB, one workgroup of 16 waves per
// CU), blocks of 2^CR_RB column ranks, workgroup size, default entries per work unit (2^17 /
// 2^18 / 2^19 / 2^20 measured 0.83 / 0.80 / 0.83 / 0.86 ms at R-MAT scale 24).  With rows as
// given: 2^13-row panels with 512-thread workgroups (two per CU) 1.38 ms, 2^14-row panels with
// 1024 threads 1.29 ms (fewer lines of x per entry, same waves).
#ifndef CR_PB
#define CR_PB 14
#endif
#define CR_RB (32 - CR_PB)  // the packed (column rank, row rank) position fills 32 bits
#ifndef CR_NT
#define CR_NT 1024
#endif
#define CR_UNIT_DEFAULT (1 << 18)
#define CR_SEG_LDS 1024  // segment starts of a panel staged in LDS when nseg + 1 <= this

// radix sort: 8-bit digits, 1024 threads x 4 keys per tile (measured best of 256..1024 threads
// and 2..16 keys per thread at 2^28 keys)
#define RS_RADIX_BITS 8
#ifndef RSORT_NT
#define RSORT_NT 1024
#endif
#ifndef RSORT_IPT
#define RSORT_IPT 4
#endif
#define RSORT_TILE (RSORT_NT * RSORT_IPT)

// statistics of the conversion sort (MSD radix sort with an LDS finish)
struct MsdStats {
    int32_t levels = 0;       // split levels run
    int64_t split_keys = 0;   // keys moved by them, summed over the levels
    int32_t first_fused = 0;  // 1: the first level built CRS keys from the triplets
};

struct spx_matrix_s {
    int32_t m = 0, n = 0;
    int64_t nnz = 0;
    spx_format fmt = 0;
    int32_t log2_beta = 0;
    int device = 0;
    MsdStats sort;  // the conversion sort's split levels
    int64_t bytes = 0;
    hipStream_t last_stream = nullptr;
    // CRS formats
    int32_t* row_ptr = nullptr;  // m+1
    int32_t* col = nullptr;      // nnz
    double* val = nullptr;       // nnz, FP64 matrices
    int32_t value_type = SPX_F64;  // stored value type
    void* val_lp = nullptr;      // nnz, FP32 or bfloat16 values of reduced-precision matrices
    // BCOHC / BCOHCH
    int32_t* bh_part_row = nullptr;   // P+1 first rows
    int32_t* bh_part_blk = nullptr;   // P+1 first blocks (stored right after bh_part_row)
    int32_t bh_nparts = 0;
    int32_t* bh_blk_ptr = nullptr;    // nb+1
    uint32_t* bh_blk_coord = nullptr; // nb, (block row << 16) | block column
    int64_t bh_nblocks = 0;
    // CSBH
    int32_t* blk_ptr = nullptr;  // nbr*nbc+1
    uint32_t* packed = nullptr;  // nnz
    int64_t nbr = 0, nbc = 0;
    // merge-path partition
    int2* mp_coords = nullptr;   // tiles+1
    int32_t mp_tiles = 0;
    int32_t* mp_carry_row = nullptr;
    double* mp_carry_val = nullptr;
    // row-split partition
    int32_t* rs_blocks = nullptr;  // nb+1 row starts
    int32_t rs_nb = 0;
    int32_t* rs_long_rows = nullptr;
    int32_t* rs_chunk_ptr = nullptr;  // nlong+1
    int32_t rs_nlong = 0, rs_nchunks = 0;
    double* rs_partials = nullptr;    // nchunks
    // CSBR: column of each column rank, ranked x copy (per-product scratch), rank of every row,
    // row of each row rank, y in row-rank order (per-product scratch); blk_ptr / packed / nbr
    // (panels) / nbc (rank segments per panel) and the cb_ unit tables as for CSBH
    int32_t* cr_order = nullptr;      // nranked
    int32_t cr_nranked = 0;
    double* cr_xr = nullptr;          // nranked
    int32_t* cr_row_rank = nullptr;   // m (ranks >= cr_nrows: rows without entries)
    int32_t* cr_row_order = nullptr;  // nrows
    int32_t cr_nrows = 0;
    double* cr_yr = nullptr;          // nrows
    // CSBH partition
    int4* cb_units = nullptr;       // {block row, first entry, end entry, partial slot or -1}
    int32_t cb_nunits = 0;
    int4* cb_split = nullptr;       // {block row, first slot, slots, 0}
    int32_t cb_nsplit = 0;
    int32_t cb_nslots = 0;
    double* cb_partials = nullptr;  // nslots * beta
    // hot-column compaction (CRS formats): entries with col < 0 read x_hot[~col]
    int32_t* hot_cols = nullptr;  // nhot original columns
    int32_t nhot = 0;
    double* x_hot = nullptr;      // per-product scratch, nhot values
    int64_t parts = 0;
    // SpMM scratch, grown on demand (freed by spx_matrix_destroy)
    int2* mm_coords = nullptr;      // merge tiles of row-split matrices (tiles+1)
    int32_t mm_tiles = 0;
    int32_t* mm_carry_row = nullptr;
    void* mm_carry = nullptr;       // tiles x chunk columns, FP64
    size_t mm_carry_bytes = 0;
    void* mm_z = nullptr;           // row-major copy of a column-major X chunk
    size_t mm_z_bytes = 0;
    void* mm_h = nullptr;           // hot rows of an X chunk
    size_t mm_h_bytes = 0;
    void* mm_w = nullptr;           // row-major results of a chunk for a column-major Y
    size_t mm_w_bytes = 0;
    std::vector<void*> owned;  // device allocations freed by spx_matrix_destroy
};

// Small device block read back by the host during conversion.
struct Readback {
    uint32_t err;
    uint32_t pad;
    unsigned long long masks[2];  // OR and AND of all sort keys
    uint32_t totals[4];
};

// ------------------------------------------------------------------ errors
// Sets the calling thread's last error message and returns s.
spx_status spx_fail(spx_status s, const char* msg);

// ------------------------------------------------------------------ serving kernels
hipError_t launch_serve_gather(const float* const* xs, int k, int n, float* X, hipStream_t s);
hipError_t launch_serve_scatter(const float* Y, int k, int m, float* const* ys,
                                const float* alpha, const float* beta, hipStream_t s);
hipError_t launch_serve_axpb(float* y, int m, float alpha, float beta, hipStream_t s);

// ------------------------------------------------------------------ batched products
// One matrix of a batch as the persistent product kernel sees it.
struct BatchMat {
    const int32_t* row_ptr;
    const int32_t* col;
    const void* val;            // FP32 values, or bfloat16 bits when bf16
    const int32_t* hot_cols;    // entries with col < 0 read x[hot_cols[~col]]
    const int2* coords;         // merge plans: tiles + 1 tile starts
    int32_t* carry_row;         // merge plans: one per tile
    double* carry_val;
    int32_t m, n;
    int32_t plan;               // SPX_PLAN_* (never AUTO here)
    int32_t tiles;              // work items of this matrix
    int32_t rows_per_tile;      // row plans
    int32_t bf16;
};
// product launch (grid workgroups, max_tile = largest merge tile of the batch, or 256) and the
// carry fix-up launch
hipError_t launch_batch_spmv(const BatchMat* mats, const int2* items, int32_t nitems,
                             int32_t grid, int32_t max_tile, const float* const* xs,
                             float* const* ys, hipStream_t s);
hipError_t launch_batch_maxlen(const int32_t* row_ptr, int32_t m, uint32_t* out, hipStream_t s);
hipError_t launch_fill_u32(uint32_t* p, int64_t n, uint32_t v, hipStream_t s);

// ------------------------------------------------------------------ allocation
void* spx_dev_alloc(size_t bytes, hipStream_t s);
void spx_dev_free(void* p, hipStream_t s);

// Stored column index of column c: ~rank for hot columns, c otherwise (words == null: no hot
// set).  One 16-byte word per 64 columns: {bitmap low half, bitmap high half, number of hot
// columns before the word, 0}, so a lookup is a single load.
struct HotMap {
    const uint4* words = nullptr;
    __device__ __forceinline__ int32_t map(uint32_t c) const {
        if (!words) return (int32_t)c;
        const uint4 wd = words[c >> 6];
        const uint64_t b = ((uint64_t)wd.y << 32) | (uint64_t)wd.x;
        const uint64_t bit = 1ull << (c & 63u);
        if (!(b & bit)) return (int32_t)c;
        return ~(int32_t)(wd.z + (uint32_t)__popcll(b & (bit - 1ull)));
    }
    // the map word of column c, for a caller that loads it ahead of use
    __device__ __forceinline__ uint4 word(uint32_t c) const {
        return words ? words[c >> 6] : make_uint4(0u, 0u, 0u, 0u);
    }
    // map() given the word of column c loaded by word()
    __device__ __forceinline__ int32_t map_word(uint32_t c, uint4 wd) const {
        const uint64_t b = ((uint64_t)wd.y << 32) | (uint64_t)wd.x;
        const uint64_t bit = 1ull << (c & 63u);
        if (!(b & bit)) return (int32_t)c;
        return ~(int32_t)(wd.z + (uint32_t)__popcll(b & (bit - 1ull)));
    }
};

// ------------------------------------------------------------------ conversion launchers
hipError_t launch_fill_i32(int32_t* p, int64_t n, int32_t v, hipStream_t s);
hipError_t launch_init_readback(Readback* rb, hipStream_t s);
hipError_t launch_keys_csr(const int32_t* row, const int32_t* col, int64_t E, int32_t m,
                           int32_t n, int cbits, uint64_t* keys, uint32_t* err,
                           unsigned long long* masks, hipStream_t s);
hipError_t launch_keys_csb(const int32_t* row, const int32_t* col, int64_t E, int32_t m,
                           int32_t n, int k, int64_t nbc, bool hilbert, uint64_t* keys,
                           uint32_t* err, unsigned long long* masks, hipStream_t s);
// Stable LSD radix sort of (keys in k0, 64-bit payloads read from vfirst).  Digits whose bits
// never vary (per `vary`) are skipped.  k1, v0, v1 are scratch of E elements; the sorted arrays
// are returned through keys_sorted / vals_sorted (one of the buffers, or vfirst if no pass ran).
// Used for the hot-column sample; its kernels carry hot_ names.
hipError_t radix_sort_pairs(uint64_t* k0, uint64_t* v0, uint64_t* k1, uint64_t* v1,
                            const uint64_t* vfirst, int64_t E, uint64_t vary, uint32_t* hist,
                            uint32_t* tile_sums, hipStream_t s, const uint64_t** keys_sorted,
                            const uint64_t** vals_sorted);
size_t radix_hist_elems(int64_t E);
// MSD radix sort with an LDS finish (the conversion sort): same result as radix_sort_pairs (a
// stable sort by the full key), sorted arrays returned in (k1, v1).  Scratch sizes from
// msd_sizes(E); *failed is set when a device-side list overflowed (not expected by the bounds).
struct MsdChunk {
    int64_t start;
    uint32_t len;
    uint32_t meta;  // bits below which the chunk is unsorted | source buffer << 8
};
struct MsdSizes {
    int64_t cap_big = 0, cap_tiles = 0, cap_chunks = 0, hist = 0, tile_sums = 0;
};
struct MsdScratch {
    MsdSizes z;
    int64_t* seg_start[2] = {nullptr, nullptr};
    uint32_t* seg_len[2] = {nullptr, nullptr};
    uint32_t* tbase = nullptr;     // cap_big + 1
    uint32_t* tile_seg = nullptr;  // cap_tiles
    uint32_t* hist = nullptr;      // z.hist
    uint32_t* tile_sums = nullptr; // z.tile_sums
    MsdChunk* chunks = nullptr;    // cap_chunks
    void* counters = nullptr;      // 40 bytes, 8-byte aligned
};
// Keys built from the triplets inside the sort's first level; only for E > RS_LOCAL_MAX.  An
// index outside the matrix sets *failed = 2.
//   order 0 (CRS): row << cbits | col
//   order 1 / 2 (CSB with Hilbert / Z-Morton order inside blocks of 2^k x 2^k):
//     (block_row * nbc + block_col) << 2k | order_k(local_col, local_row)
struct MsdTripletSource {
    const int32_t* row;
    const int32_t* col;
    int32_t m, n;
    int order;
    int cbits;    // order 0
    int k;        // orders 1, 2
    int64_t nbc;  // orders 1, 2
};
// segments of at most this many keys are finished in LDS by one workgroup
#ifndef RS_LOCAL_MAX
#define RS_LOCAL_MAX RSORT_TILE
#endif
MsdSizes msd_sizes(int64_t E);
hipError_t radix_sort_msd(uint64_t* k0, uint64_t* v0, uint64_t* k1, uint64_t* v1,
                          const uint64_t* vfirst, int64_t E, uint64_t vary, const MsdScratch& sc,
                          hipStream_t s, const uint64_t** keys_sorted,
                          const uint64_t** vals_sorted, int* failed, MsdStats* stats,
                          const MsdTripletSource* trip = nullptr, uint32_t* head_tiles = nullptr,
                          int* heads_counted = nullptr);
// head_tiles (nullable, ceil(E / SCAN_TILE) words): when *heads_counted comes back 1, it holds
// the number of run heads (first keys of runs of equal keys) in each SCAN_TILE of sorted
// positions, ready for launch_head_tiles_scan (exclusive offsets in place, total to *total).
hipError_t launch_head_tiles_scan(uint32_t* tile_counts, int64_t E, uint32_t* total,
                                  hipStream_t s);
hipError_t launch_dedup_count(const uint64_t* keys, int64_t E, uint32_t* tile_sums,
                              uint32_t* total, hipStream_t s);
// Fused: scan of run heads (tile counts from launch_dedup_count) + run sums + index/value
// output + row (block) end marks.  mode 0 CRS, 1 CSB Hilbert, 2 CSB Z-Morton; 3 BCOHC and
// 4 BCOHCH (K = total Hilbert level of mode 4), where ends[u] receives 1 for an entry that starts
// a block and 0 otherwise, and majors[u] the block key (key >> shiftbits) of block starts.
hipError_t launch_dedup_gather(const uint64_t* keys, const double* vals, int64_t E,
                               const uint32_t* tile_sums, int mode, int shiftbits, HotMap hm,
                               int32_t* idx_out, double* val_out, int32_t* ends, hipStream_t s,
                               int K = 0, uint64_t* majors = nullptr);
hipError_t launch_gather_csr(const uint64_t* keys, const double* vals, const int32_t* head_pos,
                             int64_t E, int64_t nnz_out, int cbits, HotMap hm, int32_t* col_out,
                             double* val_out, int32_t* row_end, hipStream_t s);
hipError_t launch_gather_csb(const uint64_t* keys, const double* vals, const int32_t* head_pos,
                             int64_t E, int64_t nnz_out, int k, bool hilbert, uint32_t* packed_out,
                             double* val_out, int32_t* blk_end, hipStream_t s);
hipError_t launch_gather_csbr(const uint64_t* keys, const double* vals, const int32_t* head_pos,
                              int64_t E, int64_t nnz_out, uint32_t* packed_out, double* val_out,
                              int32_t* blk_end, hipStream_t s);
static inline bool spx_is_csb(spx_format f) { return f == SPX_CSB_HILBERT || f == SPX_CSB_ZMORTON; }
static inline bool spx_is_bcoh(spx_format f) { return f == SPX_BCOHC || f == SPX_BCOHCH; }
static inline bool spx_is_crs(spx_format f) { return f == SPX_CSR_ROWSPLIT || f == SPX_CSR_MERGE; }

// ------------------------------------------------------------------ CSBR conversion
// keys (panel << (rbits + CR_PB)) | (rank_of[col] << CR_PB) | (row rank mod 2^CR_PB) with
// panel = row rank >> CR_PB, from each triplet's row rank (rrank, E words) and column; index check
hipError_t launch_keys_csbr(const int32_t* rrank, const int32_t* col, int64_t E, int32_t m,
                            int32_t n, const int32_t* rank_of, int rbits, uint64_t* keys,
                            uint32_t* err, unsigned long long* masks, hipStream_t s);
// ranking keys ((2^eb - 1 - count) << 2 pbits | first << pbits | last) << ib | (index >> ishift),
// with the index as payload (cols[c] = c): in a stable ascending sort, decreasing count, then
// increasing first and last panel, then increasing index (its high bits in the key keep runs of
// equal keys short).  count < 2^eb, panels < 2^pbits, eb + 2 pbits + ib <= 64; the panels of an
// uncounted index are taken as 0, and so are all panels when first / last are NULL (pbits = 0).
hipError_t launch_rank_keys(const uint32_t* counts, const uint32_t* first, const uint32_t* last,
                            int32_t n, int eb, int pbits, int ib, int ishift, uint64_t* keys,
                            uint64_t* cols, hipStream_t s);
// from the sorted ranking keys and indices (count field above bit fshift): rank_of[c] for every
// index, order[i] = index of rank i for the counted indices, *nranked = their number (left
// untouched when nothing is counted)
hipError_t launch_rank_scatter(const uint64_t* sorted, const uint64_t* cols, int32_t n, int eb,
                               int fshift, int32_t* order, int32_t* rank_of, uint32_t* nranked,
                               hipStream_t s);

// ------------------------------------------------------------------ BCOHC / BCOHCH
#define BH_WINDOW 8192       // rows of one partition at most (its output slice lives in LDS)
#define BH_PARTS_TARGET 2048 // partitions by entry count: target = max(2^16, ceil(E / this))
// row counts of the raw triplets (validating every index; err set on a bad one)
// Exact raw entries per row by bucketing (no per-entry global atomics); wbits from
// bcoh_row_bucket_bits(m) (-1: more than 2^26 rows, beyond what a 64-bit BCOH key can hold).
// hist: bcoh_rows_hist_elems words, rows_out: E words, total: one word, counts: m + 1 zeroed
// words.  With lo / hi (m words each, filled with 0xFFFFFFFF / 0 beforehand) also the least and
// greatest aux = map[col] >> aux_shift (map NULL: col >> aux_shift) of every row (rows without
// entries keep the fill); aux must fit 32 - wbits bits, and rowc_extent_prepare_kernel() must
// have run on the device first.  aux_keep (E words, nullable; with a map) receives map[col[i]].
int bcoh_row_bucket_bits(int32_t m);
size_t bcoh_rows_hist_elems(int32_t m, int64_t E, int wbits);
hipError_t rowc_extent_prepare_kernel();
hipError_t launch_bcoh_rows_bucketed(const int32_t* row, const int32_t* col, int64_t E,
                                     int32_t m, int32_t n, int wbits, uint32_t* hist,
                                     int32_t* rows_out, uint32_t* tile_sums, uint32_t* total,
                                     uint32_t* counts, uint32_t* err, hipStream_t s,
                                     int aux_shift = 0, uint32_t* lo = nullptr,
                                     uint32_t* hi = nullptr, const int32_t* aux_map = nullptr,
                                     int32_t* aux_keep = nullptr);

// partitions from the exclusive row-count scan cum[0..m): part_of[r] for every row, part_row[p]
// for every partition (part_row[P] = m written by the caller); *total = P
hipError_t launch_bcoh_partitions(const uint32_t* cum, int32_t m, uint32_t target,
                                  int32_t* part_of, int32_t* part_row, uint32_t* tile_sums,
                                  uint32_t* total, hipStream_t s);
hipError_t launch_keys_bcoh(const int32_t* row, const int32_t* col, int64_t E, int32_t m,
                            int32_t n, const int32_t* part_of, int k, int K2, bool hilbert,
                            uint64_t* keys, uint32_t* err, unsigned long long* masks,
                            hipStream_t s);
// block table from the block-head flags of the populate step (flags scanned in place into
// inclusive counts) and the heads' block keys (partition << 2*K2 | Hilbert block index)
hipError_t launch_bcoh_blocks(const uint32_t* incl, const uint64_t* majors, int64_t nnz, int K2,
                              int32_t* blk_ptr, uint32_t* blk_coord, int32_t* blk_part,
                              hipStream_t s);
hipError_t launch_bcoh_part_blk(const int32_t* blk_part, int64_t nb, int32_t P,
                                int32_t* part_blk, hipStream_t s);
hipError_t launch_incl_scan_u32(uint32_t* a, int64_t n, uint32_t* tile_sums, uint32_t* total,
                                hipStream_t s);
hipError_t launch_excl_scan_u32(const uint32_t* in, uint32_t* out, int64_t n,
                                uint32_t* tile_sums, uint32_t* total, hipStream_t s);
// In-place inclusive max-scan of ends[0..len) (turns "end of last entry" marks into pointers).
hipError_t launch_max_scan_i32(int32_t* ends, int64_t len, uint32_t* tile_sums, hipStream_t s);
size_t scan_tile_count(int64_t n);

// ------------------------------------------------------------------ hot columns
#define HOT_AUTO_MAX (1 << 19)
#define HOT_AUTO_MIN_N (1 << 19)
#define HOT_MAX_SAMPLES (1 << 23)
#ifndef HOT_RUN
#define HOT_RUN 8  // sampled keys come in runs of this many consecutive keys
#endif
hipError_t launch_hot_sample(const uint64_t* keys, int64_t stride, int64_t ns, uint64_t cmask,
                             uint64_t* S, hipStream_t s);
hipError_t launch_hot_count_sorted(const uint64_t* S, int64_t ns, uint32_t* freq, hipStream_t s);
hipError_t launch_hot_count_ge(const uint32_t* freq, int64_t n, uint32_t tau, uint32_t* tile_sums,
                               uint32_t* total, hipStream_t s);
hipError_t launch_hot_set(const uint32_t* freq, int64_t n, uint32_t tau, uint64_t* bits,
                          uint32_t* pre, int32_t* hot_cols, uint32_t* tile_sums, hipStream_t s);
// words[w] = {bits[w] low, bits[w] high, pre[w], 0}
hipError_t launch_hot_pack(const uint64_t* bits, const uint32_t* pre, int64_t nwords,
                           uint4* words, hipStream_t s);
// hist[min(freq[c], bins-1)] += 1 over all columns (hist zeroed by the caller)
#define HOT_HIST_BINS 4096
hipError_t launch_hot_freq_hist(const uint32_t* freq, int64_t n, uint32_t* hist, hipStream_t s);
hipError_t launch_hot_unmap(const int32_t* col, int64_t nnz, const int32_t* hot_cols,
                            int32_t* out, hipStream_t s);


// ------------------------------------------------------------------ partitions
// tile t starts on diagonal t * tile_items
hipError_t launch_merge_coords(const int32_t* row_ptr, int32_t m, int64_t nnz, int2* coords,
                               int32_t tiles, hipStream_t s, int32_t tile_items = MP_TILE);
// row-split: phase 1 counts (blocks+sentinel, long rows); phase 2 fills
hipError_t rowsplit_count(const int32_t* row_ptr, int32_t m, uint32_t* tile_sums_a,
                          uint32_t* tile_sums_b, uint32_t* totals, hipStream_t s);
hipError_t rowsplit_fill(const int32_t* row_ptr, int32_t m, const uint32_t* tile_sums_a,
                         const uint32_t* tile_sums_b, int32_t* blocks, int32_t* long_rows,
                         hipStream_t s);
hipError_t rowsplit_chunks(const int32_t* row_ptr, const int32_t* long_rows, int32_t nlong,
                           int32_t* chunk_ptr, uint32_t* tile_sums, uint32_t* total,
                           hipStream_t s);
// CSBH: plan = per block row unit and slot counts (scanned), then the unit table
hipError_t csbh_plan(const int32_t* blk_ptr, int64_t nbr, int64_t nbc, int64_t unit_nnz,
                     int32_t* unit_ptr, int32_t* slot_ptr, int32_t* split_ptr, uint32_t* totals,
                     hipStream_t s);
hipError_t csbh_units(const int32_t* blk_ptr, int64_t nbr, int64_t nbc, int64_t unit_nnz,
                      const int32_t* unit_ptr, const int32_t* slot_ptr, const int32_t* split_ptr,
                      int4* units, int4* split, hipStream_t s);

// ------------------------------------------------------------------ products
hipError_t spmv_merge(const spx_matrix_s* A, const double* x, double* y, hipStream_t s);
// CRS product of a reduced-precision (FP32 / bfloat16) matrix with FP32 x and y
hipError_t spmv_crs_f32(const spx_matrix_s* A, const float* x, float* y, hipStream_t s);
// FP64 values -> FP32 (round to nearest) or bfloat16 bits (round to nearest even)
hipError_t launch_round_values(const double* in, int64_t n, int32_t vt, void* out, hipStream_t s);
hipError_t spmv_rowsplit(const spx_matrix_s* A, const double* x, double* y, hipStream_t s);
// Y = A X with k right-hand sides (CRS formats): merge tiles, carries and X staging buffers
struct SpmmPlan {
    const int2* coords = nullptr;
    int32_t tiles = 0;
    int32_t* carry_row = nullptr;
    double* carry_val = nullptr;  // tiles x spmm_chunk_cols(k)
    void* z = nullptr;            // n x chunk, column-major X only
    void* w = nullptr;            // m x chunk, row-major results for a column-major Y
    void* h = nullptr;            // nhot x chunk
};
int32_t spmm_chunk_cols(int32_t k);
// y = A x with the single-vector merge-path kernels on the plan's tiles and scratch (P.h holds the
// hot x copy); used for one-column products on contiguous vectors
hipError_t spmv_merge_on_plan(const spx_matrix_s* A, const SpmmPlan& P, const void* x, void* y,
                              hipStream_t s);
hipError_t spmm_crs(const spx_matrix_s* A, const SpmmPlan& P, int32_t k, const void* x,
                    int64_t ldx, void* y, int64_t ldy, int row_major, hipStream_t s);
hipError_t spmv_csbh(const spx_matrix_s* A, const double* x, double* y, hipStream_t s);
hipError_t spmv_bcoh(const spx_matrix_s* A, const double* x, double* y, hipStream_t s);
// reduced-precision CSB / CSBH and BCOHC / BCOHCH (value_type FP32 or bfloat16): FP32 x and y,
// FP32 products, FP64 sums
hipError_t spmv_csbh_f32(const spx_matrix_s* A, const float* x, float* y, hipStream_t s);
hipError_t spmv_bcoh_f32(const spx_matrix_s* A, const float* x, float* y, hipStream_t s);
hipError_t spmv_csbr(const spx_matrix_s* A, const double* x, double* y, hipStream_t s);
// reduced-precision CSBR (value_type FP32 or bfloat16): FP32 x and y
hipError_t spmv_csbr_f32(const spx_matrix_s* A, const float* x, float* y, hipStream_t s);
hipError_t csbr_prepare_kernel();
hipError_t bcoh_prepare_kernel();

// ------------------------------------------------------------------ memory probe
int64_t probe_out_len();
hipError_t launch_probe_gather(const double* x, int64_t window, int64_t n, double* out,
                               hipStream_t s);
