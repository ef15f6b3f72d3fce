/*
 * spx_batch.h -- one launch for the products of many matrices (part of libspx).
 *
 * A batch holds a set of converted CRS matrices (handles from spx_convert, FP32 or bfloat16
 * values) and computes y_i = A_i x_i for all of them with one product launch over the work items
 * of every matrix, followed by one small launch that adds the merge tiles' carries.  Each matrix
 * is cut into work items by its own plan:
 *   - merge tiles: 256 * ipt consecutive items of the merge of row ends and entries (Section
 *     3.3), ipt in {4, 8, 16}; the values a tile leaves open are added in tile order by the
 *     fix-up launch;
 *   - row tiles: `rows` consecutive whole rows, each row reduced by a group of lanes sized to the
 *     tile's average row length (for matrices whose rows are all at most 1024 entries long).
 * The workgroups of the product launch take the work items of all matrices in a fixed stride
 * (persistent workgroups when the grid is smaller than the item count), so small and large
 * matrices share the device without one launch per matrix.
 *
 * The plan of each matrix is chosen by an autotuner at creation (unless fixed by the caller): it
 * times every candidate (merge tiles with ipt 4, 8, 16; row tiles of 512 or 2048 entries when the
 * rows allow) on the matrix alone, its tiles repeated to at least 8192 work items so that the
 * device is as full as inside a batch, and keeps the cheapest per pass.  It then times the whole
 * batch with one workgroup per item and with persistent grids of 4096 and 1024 workgroups, for
 * those plans, with 16-item merge tiles turned into 8-item ones (the largest tile sets the
 * launch's LDS size, hence the occupancy of every workgroup), and with each single plan for all
 * matrices, and keeps the fastest: the tuned batch is never slower than one fixed plan for all,
 * to the precision of the timing.
 *
 * A product is two kernel launches with no allocation, no host synchronisation and no memset, so
 * it can be captured in a HIP graph and replayed.
 * Results are deterministic; they equal each matrix's product within the FP32 dot-product error
 * bound (integer-valued inputs: exactly).
 */
#ifndef SPX_BATCH_H
#define SPX_BATCH_H

#include "spx.h"

#ifdef __cplusplus
extern "C" {
#endif

typedef struct spx_batch_s* spx_batch;

#define SPX_PLAN_AUTO 0       /* autotune                                              */
#define SPX_PLAN_MERGE_4 1    /* merge tiles of 256 * 4 items                           */
#define SPX_PLAN_MERGE_8 2    /* merge tiles of 256 * 8 items                           */
#define SPX_PLAN_MERGE_16 3   /* merge tiles of 256 * 16 items                          */
#define SPX_PLAN_ROWS_512 4   /* row tiles of about 512 entries (rows <= 1024 entries)  */
#define SPX_PLAN_ROWS_2048 5  /* row tiles of about 2048 entries                        */

/*
 * Build a batch over `count` handles (CRS, FP32 or bfloat16 values; a handle may appear only
 * once; the handles must outlive the batch and are not modified).  plans: NULL (autotune all) or
 * `count` SPX_PLAN_* values; chosen (nullable): receives the plan used per matrix.  Autotuning
 * runs products on `stream` with scratch vectors and synchronises it.
 * Errors: INVALID_ARG (NULL, count < 1, a repeated handle, an unknown plan, a row-tile plan for a
 * matrix with a row longer than 1024 entries), UNSUPPORTED (a CSB handle or FP64 values), NOMEM.
 */
spx_status spx_batch_create(const spx_matrix* mats, int32_t count, const int32_t* plans,
                            void* stream, spx_batch* out, int32_t* chosen);

/* Bind the vectors: xs[i] (n_i floats) and ys[i] (m_i floats) are device pointers, given in a
 * host array; y_i must not overlap any x_j or other y_j.  Copies the table to the device and
 * synchronises `stream`.  Products use the bound vectors until the next bind. */
spx_status spx_batch_bind(spx_batch B, const float* const* xs, float* const* ys, void* stream);

/* y_i = A_i x_i for every matrix of the batch: one kernel launch on `stream`. */
spx_status spx_batch_spmv(spx_batch B, void* stream);

/* Work items and workgroups of the launch. */
spx_status spx_batch_get_info(spx_batch B, int64_t* items, int32_t* workgroups);

spx_status spx_batch_destroy(spx_batch B);

#ifdef __cplusplus
}
#endif
#endif
