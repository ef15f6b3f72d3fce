/*
 * spx.h -- C ABI of libspx, sparse matrix-vector multiplication y = A x on AMD MI355X (gfx950).
 *
 * The operations follow the problem statement of Bergmans, Meerbergen and Vandebril, "Algorithms
 * for Parallel Shared-Memory Sparse Matrix-Vector Multiplication on Unstructured Matrices"
 * (arXiv 2502.19284):
 *   - A is an m x n sparse matrix with nnz stored entries, x and y are dense, y = A x (Section 1);
 *   - A arrives in the triplet (coordinate) format: row_ind, col_ind, data (Section 2);
 *   - before any product the triplets are converted to the format an algorithm needs, and the
 *     conversion cost is measured and reported beside the product (Sections 5.1 and 6.2).
 *
 * Conventions of every entry point
 *   - Pointers named "device" must point to memory of the current HIP device; host pointers are
 *     marked "host".  Nothing here takes ownership of caller memory.
 *   - `stream` is a hipStream_t passed as void*; NULL means the default stream.  All device work
 *     is enqueued on it.
 *   - Return value: SPX_OK (0) or a negative spx_status.  No C++ exception crosses the ABI.
 *     Argument errors are reported before any device work is enqueued.  A thread-local message
 *     with details is available from spx_last_error_message().
 *   - Indices are 0-based int32.  Values and vectors are IEEE binary64 unless stated otherwise.
 */
#ifndef SPX_H
#define SPX_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ------------------------------------------------------------------ status codes */
typedef int32_t spx_status;
#define SPX_OK 0
#define SPX_ERR_INVALID_ARG -1 /* null pointer, negative size, unknown enum value        */
#define SPX_ERR_INDEX -2       /* a triplet index outside [0,m) x [0,n)                   */
#define SPX_ERR_RANGE -3       /* a size beyond the int32 index range (nnz >= 2^31 ...)   */
#define SPX_ERR_ALIAS -4       /* x and y overlap                                          */
#define SPX_ERR_NOMEM -5       /* device allocation failed                                 */
#define SPX_ERR_HIP -6         /* a HIP runtime call failed                                */
#define SPX_ERR_UNSUPPORTED -7 /* valid request that this build does not implement         */
#define SPX_ERR_DEVICE -8      /* a device-side bound was exceeded; the results are void    */

/* ------------------------------------------------------------------ enums */
typedef int32_t spx_format;
/* CRS (Section 2) with rows split among workgroups: short rows are grouped into row blocks of
 * bounded size, rows longer than a threshold are split into chunks whose partial sums are added
 * in chunk order.  Row-parallel like the paper's ParCRS baseline (Section 5.1). */
#define SPX_CSR_ROWSPLIT 0
/* CRS processed by merge-path bands of equal length over (row ends, entries) (Section 3.3). */
#define SPX_CSR_MERGE 1
/* Compressed sparse blocks with Hilbert order inside each block, CSBH (Sections 3.1 and 4.1). */
#define SPX_CSB_HILBERT 2
/* Compressed sparse blocks with Z-Morton order inside each block, CSB (Section 3.1). */
#define SPX_CSB_ZMORTON 3
/* Row-distributed blocks with compressed triplets, BCOHC (Section 3.2, hybrid variants): the rows
 * are cut into partitions of about equal entry count (one per workgroup, each at most 8192 rows),
 * a partition's beta x beta blocks are stored in Hilbert order, and inside a block the entries are
 * packed (local_row << 16) | local_col in row-wise order.  The block level keeps an explicit block
 * coordinate per block instead of the paper's BICRS increments (GPU threads need random access). */
#define SPX_BCOHC 4
/* BCOHCH: as BCOHC with every partition's entries sorted by the Hilbert curve over (row, col). */
#define SPX_BCOHCH 5
/* Compressed sparse blocks over ranked rows and columns, CSBR (the block idea of Section 3.1 -- a
 * block row keeps its slice of y on chip and reads only part of x -- laid out for a GPU):
 *   - rows are ranked by decreasing raw triplet count, ties by increasing row index; only rows
 *     with at least one triplet are ranked (the others get y = 0), rank i holds row
 *     row_order[i];
 *   - block rows (panels) are 2^14 consecutive row ranks, whose y slice lives in LDS during a
 *     product;
 *   - columns are ranked by decreasing raw triplet count; equal counts by increasing first panel
 *     (the least panel among the column's triplets), then increasing last panel (the greatest),
 *     then increasing column index; only columns with at least one triplet are ranked, and rank
 *     i holds column col_order[i];
 *   - a block is (panel, 2^18 consecutive column ranks); blocks are stored panel by panel in
 *     rank order;
 *   - inside a block, entries are stored column-major: by column rank, then by row rank; each
 *     entry packs (column rank mod 2^18) << 14 | (row rank mod 2^14) into 32 bits.
 * A product first gathers x into rank order (x_r[i] = x[col_order[i]]); a wave then reads
 * consecutive entries whose ranks ascend, so lanes that share a column, or neighbouring ranks,
 * share cache lines of x_r, and the most frequent columns occupy the first lines.  Ranking the
 * rows gathers the longest rows into the first panels, and the panel tie-break puts rare columns
 * that meet the same panels next to each other: both cut the x_r lines a product fetches.  The
 * panels' slices form y in row-rank order, which a last pass permutes into y.
 * Rows and columns are limited to 2^26 (their counts are bucketed in LDS).  Values FP64, or FP32
 * / bfloat16 (products FP32, every sum FP64: the slice, the partial slices and their reduction). */
#define SPX_CSB_RANKED 6

typedef int32_t spx_dtype;
#define SPX_F64 0
#define SPX_F32 1  /* stored values only: products take FP32 x and y (spx_spmv_f32)      */
#define SPX_BF16 2 /* bfloat16 stored values (round to nearest even); FP32 x and y        */

/* Layout of the dense n x k (X) and m x k (Y) operands of spx_spmm. */
typedef int32_t spx_layout;
#define SPX_COL_MAJOR 0 /* element (i, c) at base[i + c * ld], ld >= rows (BLAS layout)  */
#define SPX_ROW_MAJOR 1 /* element (i, c) at base[i * ld + c], ld >= k                   */

/* ------------------------------------------------------------------ inputs */
/* Triplet format (Section 2): entry i is (row[i], col[i], val[i]).  Entries may come in any order
 * and may repeat a coordinate; repeats are summed in increasing i by default.  Explicit zeros are
 * kept as stored entries. */
typedef struct {
    int32_t m;          /* rows,    >= 0                                   */
    int32_t n;          /* columns, >= 0                                   */
    int64_t nnz;        /* number of triplets, 0 <= nnz < 2^31             */
    const int32_t* row; /* device, nnz entries (may be NULL when nnz == 0) */
    const int32_t* col; /* device, nnz entries                             */
    const void* val;    /* device, nnz values of type val_type             */
    spx_dtype val_type; /* SPX_F64                                         */
} spx_coo_desc;

typedef struct {
    int32_t sum_duplicates; /* 1: sum repeated coordinates (default); 0: keep each as an entry  */
    int32_t log2_beta;      /* CSB/CSBH/BCOHC/BCOHCH block side 2^log2_beta; 0 = block-size
                             * rule (Section 3.1)                                            */
    int32_t validate;       /* indices are always checked (fused into the key build); 0 or 1  */
    int32_t tile_items;     /* work per tile/unit; 0 = default for the format                  */
    int32_t hot_columns;    /* CRS formats: at most this many of the most frequent columns get a
                             * compact copy of their x values per product (x_hot); -1 = automatic
                             * (up to 2^19 when n >= 2^19), 0 = off.  y is unchanged by it.      */
    spx_dtype value_type;   /* stored value type: SPX_F64 (default), or SPX_F32 / SPX_BF16
                             * (repeats are summed in FP64, then rounded once)                 */
} spx_convert_opts;

typedef struct {
    float convert_ms;  /* device time of the whole conversion, events on `stream`      */
    int64_t nnz_out;   /* stored entries after repeats were summed                      */
    int64_t bytes;     /* device bytes held by the handle                               */
    int32_t log2_beta; /* CSBH block side used (0 for CRS formats)                      */
    int32_t parts;     /* work units of the format (tiles, row blocks, block-row chunks)*/
    int64_t sort_split_keys; /* keys moved by the sort's global split levels, summed      */
    int32_t sort_levels;     /* global split levels the sort ran                          */
    int32_t sort_first_fused; /* 1: the first level read the triplets (keys built there) */
} spx_convert_report;

typedef struct spx_matrix_s* spx_matrix;

typedef struct {
    int32_t m, n;
    int64_t nnz;       /* stored entries                        */
    spx_format format;
    int32_t log2_beta; /* CSBH only                             */
    int64_t bytes;     /* device bytes held by the handle       */
    int64_t parts;     /* work units                            */
    spx_dtype value_type;
} spx_matrix_info;

/* Arrays of a converted matrix that spx_matrix_export can copy out. */
typedef int32_t spx_array;
#define SPX_ARRAY_ROW_PTR 0 /* CRS formats: int32[m+1]                                      */
#define SPX_ARRAY_COL_IND 1 /* CRS formats: int32[nnz], ascending inside a row              */
#define SPX_ARRAY_VALUES 2  /* all formats: values[nnz] in storage order, of the stored type */
#define SPX_ARRAY_BLK_PTR 3 /* CSB/CSBH: int32[nbr*nbc+1], blocks in row-wise order;
                             * CSBR: int32[panels*segments+1], block (panel, rank segment) at
                             * panel * segments + segment;
                             * BCOHC/BCOHCH: int32[blocks+1], first entry of each stored block */
#define SPX_ARRAY_PACKED 4  /* CSB/CSBH: uint32[nnz], (local_row << 16) | local_col, in the
                             * block's Hilbert (CSBH) or Z-Morton (CSB) order; CSBR:
                             * (column rank mod 2^18) << 14 | (row rank mod 2^14), column-major
                             * in a block */
#define SPX_ARRAY_PARTS 5   /* format's work-unit table, int32 (layout is internal; BCOHC /
                             * BCOHCH: P+1 partition first rows, then P+1 first blocks)     */
#define SPX_ARRAY_BLK_COORD 6 /* BCOHC/BCOHCH: uint32[blocks], (block_row << 16) | block_col */
#define SPX_ARRAY_COL_ORDER 7 /* CSBR: int32[ranked columns], the column of each rank          */
#define SPX_ARRAY_ROW_ORDER 8 /* CSBR: int32[ranked rows], the row of each row rank             */

/* Optional device allocator: alloc returns NULL on failure; free accepts what alloc returned. */
typedef void* (*spx_alloc_fn)(size_t bytes, void* stream, void* ctx);
typedef void (*spx_free_fn)(void* ptr, void* stream, void* ctx);

/* ------------------------------------------------------------------ entry points */

/* Fill *opts with the defaults: sum_duplicates=1, log2_beta=0, validate=1, tile_items=0,
 * hot_columns=-1, value_type=SPX_F64. */
spx_status spx_convert_opts_default(spx_convert_opts* opts);

/*
 * Convert triplets to `fmt` (Section 5.1: sort the entries into the format's order, then fill and
 * compress the arrays).  The sort is a stable device radix sort on the format's key:
 *   CRS:  (row, col);
 *   CSBH: (block row, block column, Hilbert index of the local (row, col) in the block);
 *   CSB:  the same with the Z-Morton index;
 *   CSBR: (panel, column rank, row rank), after counts of the raw triplets per row and per
 *         column (with the first and last panel each column meets) and sorts of the rows and the
 *         columns by those counts.
 * Repeated coordinates become one entry whose value is the sum in increasing triplet index.
 * The work-unit table the product uses is built here as well, and counted in the conversion.
 *
 * coo:  host pointer to the descriptor; its arrays are device memory owned by the caller and
 *       only read.
 * opts: host, may be NULL for defaults.
 * out:  host; receives a new handle on success, NULL on any error.
 * rep:  host, may be NULL.  convert_ms covers all device work of the call.
 * The call returns after the device work is complete (it reads back the entry count).
 * Errors: INVALID_ARG, RANGE (m, n or nnz beyond int32, a CSB / BCOHC key beyond 64 bits, or
 * more than 2^26 rows or columns for CSBR), INDEX (an index out of range; indices are always
 * checked), UNSUPPORTED (sum_duplicates=0 for BCOHC / BCOHCH), NOMEM, HIP, DEVICE (a device-side
 * list of the sort outgrew its bound; not expected).  On error every temporary is freed.
 */
spx_status spx_convert(const spx_coo_desc* coo, spx_format fmt, const spx_convert_opts* opts,
                       void* stream, spx_matrix* out, spx_convert_report* rep);

/*
 * y = A x (Algorithm 1's result; y is overwritten, rows without entries give +0).
 * x: device, n doubles.  y: device, m doubles.  x and y must not overlap (SPX_ERR_ALIAS).
 * Asynchronous on `stream`.  A handle holds per-product scratch, so at most one product per
 * handle may be in flight at a time; products on different handles may overlap freely.
 * Summation order: fixed for the CRS formats (repeated products are bitwise identical); the block
 * formats (CSB, CSBH, CSBR, BCOHC, BCOHCH) add products into an on-chip slice of y with float atomics,
 * so their last bits may differ from run to run (always within the row-scaled 1e-12 bound).
 */
spx_status spx_spmv(spx_matrix A, const double* x, double* y, void* stream);

/*
 * Reduced-precision product y = A x for a matrix stored in FP32 or bfloat16 (value_type at
 * conversion): x (n floats) and y (m floats) are device FP32.  CRS formats: products and sums
 * inside a merge tile or row block are FP32, sums that cross tiles and rows longer than a row
 * block are FP64.  Block formats (CSB, CSBH, BCOHC, BCOHCH, CSBR): products FP32, every sum FP64
 * (the on-chip slice of y); y rounded to FP32 once.
 * Otherwise as spx_spmv.  Errors: UNSUPPORTED for an FP64 matrix (use spx_spmv), and spx_spmv
 * returns UNSUPPORTED for a reduced-precision matrix.
 */
spx_status spx_spmv_f32(spx_matrix A, const float* x, float* y, void* stream);

/*
 * Product with k right-hand sides, Y = A X: column c of Y is the product of Section 2 with column
 * c of X, for c = 0 .. k-1, and the k products share one pass over the matrix.  X is n x k and Y
 * is m x k, device memory, both in `layout` with leading dimensions ldx and ldy (see spx_layout);
 * their element type is that of the matrix's products: double for FP64 matrices, float for FP32 and
 * bfloat16 ones (accumulation as in spx_spmv / spx_spmv_f32).  Y is overwritten; X is only read.
 * Any k >= 1 (columns are processed in chunks of 64).  CRS formats only.
 * Scratch (row-major copies of column-major X and Y chunks, compact hot rows, tile carries) is held by
 * the handle, grown on demand and freed by spx_matrix_destroy; as for spx_spmv, one product call
 * per handle may be in flight at a time.
 * Errors: INVALID_ARG for k < 1, an unknown layout, a leading dimension below its minimum or a
 * NULL operand; ALIAS when the spans of X and Y overlap; UNSUPPORTED for the block formats (CSB,
 * CSBH, BCOHC, BCOHCH, CSBR); RANGE
 * when a span does not fit in 64 bits; NOMEM when scratch cannot be allocated.
 */
spx_status spx_spmm(spx_matrix A, int32_t k, const void* X, int64_t ldx, void* Y, int64_t ldy,
                    spx_layout layout, void* stream);

/*
 * Y = A X exactly as spx_spmm (same arguments, results and errors), for callers that cannot
 * allocate device memory: code under HIP graph capture, tight serving loops, harnesses that forbid
 * hipMalloc.  It makes no device allocation and calls no allocating routine.  Its scratch (the
 * staging of column-major X and Y chunks, the hot rows of X, the merge tiles' carries and, for
 * row-split matrices, the merge tile starts) lives in a static device array of 32 MiB that each
 * GPU the library runs on holds until the process ends; a product needing more is refused with
 * SPX_ERR_RANGE before any device work.  All calls on one GPU share that array, which keeps the
 * last call's contents: calls that overlap on one GPU (other streams or threads) race, and the
 * caller must serialise them.  The current device must be the matrix's (SPX_ERR_INVALID_ARG).
 * Additional errors: HIP when the array's device address cannot be obtained.
 */
spx_status spx_spmm_noalloc(spx_matrix A, int32_t k, const void* X, int64_t ldx, void* Y,
                            int64_t ldy, spx_layout layout, void* stream);

/* Sizes and format of a handle.  info: host. */
spx_status spx_matrix_get_info(spx_matrix A, spx_matrix_info* info);

/*
 * Copy one array of the handle into caller memory `dst` (device, `bytes` long) on `stream`,
 * asynchronously.  Errors: INVALID_ARG when the array does not exist for the format or when
 * `bytes` is smaller than the array (the required size is written to *needed if not NULL).
 */
spx_status spx_matrix_export(spx_matrix A, spx_array which, void* dst, int64_t bytes,
                             int64_t* needed, void* stream);

/* Wait for the handle's device work, then free everything it holds.  NULL is accepted. */
spx_status spx_matrix_destroy(spx_matrix A);

/*
 * Number of products after which `fmt` pays for its longer conversion against the reference CRS
 * path: the N where conv_fmt + N * spmv_fmt = conv_ref + N * spmv_ref (Section 7 reports such
 * counts).  Returns +infinity when spmv_fmt >= spmv_ref, and 0 when the format multiplies faster
 * and converts no slower (it is ahead from the first product).  Times in any one unit.
 */
double spx_break_even(double conv_fmt, double conv_ref, double spmv_ref, double spmv_fmt);

/* Route the library's device allocations through caller functions (both NULL = hipMalloc and
 * hipFree).  Affects allocations made after the call; not thread-safe against running calls. */
spx_status spx_set_allocator(spx_alloc_fn alloc, spx_free_fn free_fn, void* ctx);

/*
 * Per-kernel timing (measurement aid; the paper reports minimum times over repeated runs,
 * Section 5.2).  While enabled, every kernel the library launches is bracketed by HIP events on
 * its launch stream.  spx_profile_enable clears the statistics; spx_profile_collect waits for the
 * recorded events and returns one record per kernel name (sorted by name).
 */
typedef struct {
    char name[48];     /* kernel name                        */
    int64_t launches;  /* launches recorded since enabling   */
    double total_ms;   /* summed event-to-event durations    */
    double min_ms;
    double max_ms;
} spx_kernel_stat;

spx_status spx_profile_enable(int32_t enable);
/* out: host array of `max` records (may be NULL when max == 0); *count receives the number of
 * kernels recorded, which may exceed max. */
spx_status spx_profile_collect(spx_kernel_stat* out, int32_t max, int32_t* count);

/*
 * Memory-system probe (measurement aid): `n` random 8-byte loads from the first `window` doubles
 * of x (device; window a power of two, 1 <= window <= x's length), each thread summing its loads
 * into out (device, spx_probe_out_len() doubles, overwritten).  Timed by the caller on `stream`.
 * With a window far beyond the L2 every load fills one 128-byte line (the rate that bounds the x
 * gathers of a product); inside the L2 it measures the L2 request rate.
 * Errors: INVALID_ARG for a NULL pointer, a window that is not a power of two, or n < 0.
 */
spx_status spx_probe_gather(const double* x, int64_t window, int64_t n, double* out, void* stream);
int64_t spx_probe_out_len(void);

/* Static text for a status code. */
const char* spx_status_string(spx_status s);

/* Details of the last error on the calling thread ("" when none). */
const char* spx_last_error_message(void);

/* Library version as "major.minor.patch". */
const char* spx_version(void);

#ifdef __cplusplus
}
#endif
#endif /* SPX_H */
