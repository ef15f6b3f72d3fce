// k_partition.hip -- work-unit tables built at conversion time (gfx950).
//
//   merge-path CRS : start point of every tile on the merge path of (row ends, entry indices)
//                    (Section 3.3): tile t starts on diagonal t * MP_TILE.
//   row-split CRS  : row blocks with a bounded entry count, plus the list of long rows and their
//                    chunk pointers (rows are never shared between blocks).
//   CSBH           : chunks of at most `unit_nnz` entries inside one block row (Section 3.1 splits
//                    heavy block rows into several tasks with temporary output vectors).
#include "dev_scan.h"
#include "spx_internal.h"

// ------------------------------------------------------------------ merge path

// Point (i, j) on diagonal d: i row ends and j entries consumed, ties consuming the row end
// first.  Binary search for the number of row ends i: A[p] = row_ptr[p+1] precedes B[d-p-1] =
// d-p-1 exactly when row_ptr[p+1] <= d-p-1.
__global__ void k_merge_coords(const int32_t* __restrict__ row_ptr, int32_t m, int64_t nnz,
                               int2* __restrict__ coords, int32_t tiles, int32_t tile_items) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t > tiles) return;
    const int64_t total = (int64_t)m + nnz;
    int64_t d = t * tile_items;
    if (d > total) d = total;
    int64_t lo = d - nnz > 0 ? d - nnz : 0;
    int64_t hi = d < m ? d : m;
    while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if ((int64_t)row_ptr[mid + 1] <= d - mid - 1) lo = mid + 1;
        else hi = mid;
    }
    coords[t] = make_int2((int)lo, (int)(d - lo));
}

hipError_t launch_merge_coords(const int32_t* row_ptr, int32_t m, int64_t nnz, int2* coords,
                               int32_t tiles, hipStream_t s, int32_t tile_items) {
    const unsigned g = spx_div_up((int64_t)tiles + 1, 256);
    SPX_LAUNCH("merge_coords", k_merge_coords, dim3(g), dim3(256), 0, s, row_ptr, m, nnz, coords,
               tiles, tile_items);
    return hipGetLastError();
}

// ------------------------------------------------------------------ row split
//
// A row block starts at row r when r is 0 or m, r is a multiple of RS_ROWS, row r or row r-1 is
// long (more than RS_LONG entries), or row r starts in a different bucket of RS_NNZ - RS_LONG
// entries than row r-1.  A block without long rows then holds at most
// (RS_NNZ - RS_LONG - 1) + RS_LONG < RS_NNZ entries; a long row is a block on its own.

#define RS_BUCKET (RS_NNZ - RS_LONG)

struct LoadRsBoundary {
    const int32_t* rp;
    int32_t m;
    __device__ uint32_t operator()(int64_t r) const {
        if (r == 0 || r == m || (r % RS_ROWS) == 0) return 1u;
        const int32_t a = rp[r - 1], b = rp[r], c = rp[r + 1];
        if (b - a > RS_LONG || c - b > RS_LONG) return 1u;
        return (b / RS_BUCKET) != (a / RS_BUCKET) ? 1u : 0u;
    }
};
struct StoreRsBoundary {
    int32_t* blocks;
    __device__ void operator()(int64_t r, uint32_t incl, uint32_t item) const {
        if (item) blocks[incl - 1] = (int32_t)r;
    }
};
struct LoadRsLong {
    const int32_t* rp;
    __device__ uint32_t operator()(int64_t r) const {
        return rp[r + 1] - rp[r] > RS_LONG ? 1u : 0u;
    }
};
struct StoreRsLong {
    int32_t* rows;
    __device__ void operator()(int64_t r, uint32_t incl, uint32_t item) const {
        if (item) rows[incl - 1] = (int32_t)r;
    }
};

hipError_t rowsplit_count(const int32_t* row_ptr, int32_t m, uint32_t* tile_sums_a,
                          uint32_t* tile_sums_b, uint32_t* totals, hipStream_t s) {
    hipError_t e = scan_phase12<uint32_t, OpSum<uint32_t>>(LoadRsBoundary{row_ptr, m},
                                                           (int64_t)m + 1, tile_sums_a, totals, s);
    if (e != hipSuccess) return e;
    return scan_phase12<uint32_t, OpSum<uint32_t>>(LoadRsLong{row_ptr}, (int64_t)m, tile_sums_b,
                                                   totals + 1, s);
}

hipError_t rowsplit_fill(const int32_t* row_ptr, int32_t m, const uint32_t* tile_sums_a,
                         const uint32_t* tile_sums_b, int32_t* blocks, int32_t* long_rows,
                         hipStream_t s) {
    hipError_t e = scan_phase3<uint32_t, OpSum<uint32_t>>(
        LoadRsBoundary{row_ptr, m}, StoreRsBoundary{blocks}, (int64_t)m + 1, tile_sums_a, s);
    if (e != hipSuccess || long_rows == nullptr) return e;
    return scan_phase3<uint32_t, OpSum<uint32_t>>(LoadRsLong{row_ptr}, StoreRsLong{long_rows},
                                                  (int64_t)m, tile_sums_b, s);
}

struct LoadRsChunks {
    const int32_t* rp;
    const int32_t* rows;
    __device__ uint32_t operator()(int64_t j) const {
        const int32_t r = rows[j];
        return (uint32_t)((rp[r + 1] - rp[r] + RS_CHUNK - 1) / RS_CHUNK);
    }
};
struct StoreRsChunks {
    int32_t* ptr;
    int64_t n;
    __device__ void operator()(int64_t j, uint32_t incl, uint32_t item) const {
        ptr[j] = (int32_t)(incl - item);
        if (j == n - 1) ptr[n] = (int32_t)incl;
    }
};

hipError_t rowsplit_chunks(const int32_t* row_ptr, const int32_t* long_rows, int32_t nlong,
                           int32_t* chunk_ptr, uint32_t* tile_sums, uint32_t* total,
                           hipStream_t s) {
    if (nlong <= 0) return hipSuccess;
    hipError_t e = scan_phase12<uint32_t, OpSum<uint32_t>>(LoadRsChunks{row_ptr, long_rows}, nlong,
                                                           tile_sums, total, s);
    if (e != hipSuccess) return e;
    return scan_phase3<uint32_t, OpSum<uint32_t>>(LoadRsChunks{row_ptr, long_rows},
                                                  StoreRsChunks{chunk_ptr, nlong}, nlong,
                                                  tile_sums, s);
}

// ------------------------------------------------------------------ CSBH units

// One workgroup: per block row br, units = max(1, ceil(entries / unit_nnz)); rows with more than
// one unit get that many partial-output slots and one entry in the split list.  Exclusive
// prefixes of the three counts are written per block row; totals[0..2] get the sums.
__global__ __launch_bounds__(256) void k_csbh_plan(const int32_t* __restrict__ blk_ptr,
                                                   int64_t nbr, int64_t nbc, int64_t unit_nnz,
                                                   int32_t* unit_ptr, int32_t* slot_ptr,
                                                   int32_t* split_ptr, uint32_t* totals) {
    __shared__ uint32_t stmp[4];
    uint32_t cu = 0, cs = 0, cp = 0;
    for (int64_t base = 0; base < nbr; base += 256) {
        const int64_t br = base + threadIdx.x;
        uint32_t nu = 0, ns = 0, np = 0;
        if (br < nbr) {
            const int64_t z = (int64_t)blk_ptr[(br + 1) * nbc] - blk_ptr[br * nbc];
            nu = z <= unit_nnz ? 1u : (uint32_t)((z + unit_nnz - 1) / unit_nnz);
            ns = nu > 1 ? nu : 0u;
            np = nu > 1 ? 1u : 0u;
        }
        uint32_t tu, ts, tp;
        const uint32_t eu = block_excl_scan<256, uint32_t, OpSum<uint32_t>>(nu, stmp, &tu);
        const uint32_t es = block_excl_scan<256, uint32_t, OpSum<uint32_t>>(ns, stmp, &ts);
        const uint32_t ep = block_excl_scan<256, uint32_t, OpSum<uint32_t>>(np, stmp, &tp);
        if (br < nbr) {
            unit_ptr[br] = (int32_t)(cu + eu);
            slot_ptr[br] = (int32_t)(cs + es);
            split_ptr[br] = (int32_t)(cp + ep);
        }
        cu += tu;
        cs += ts;
        cp += tp;
    }
    if (threadIdx.x == 0) {
        totals[0] = cu;
        totals[1] = cs;
        totals[2] = cp;
    }
}

hipError_t csbh_plan(const int32_t* blk_ptr, int64_t nbr, int64_t nbc, int64_t unit_nnz,
                     int32_t* unit_ptr, int32_t* slot_ptr, int32_t* split_ptr, uint32_t* totals,
                     hipStream_t s) {
    SPX_LAUNCH("csbh_plan", k_csbh_plan, dim3(1), dim3(256), 0, s, blk_ptr, nbr, nbc, unit_nnz,
                       unit_ptr, slot_ptr, split_ptr, totals);
    return hipGetLastError();
}

__global__ void k_csbh_units(const int32_t* __restrict__ blk_ptr, int64_t nbr, int64_t nbc,
                             int64_t unit_nnz, const int32_t* __restrict__ unit_ptr,
                             const int32_t* __restrict__ slot_ptr,
                             const int32_t* __restrict__ split_ptr, int4* __restrict__ units,
                             int4* __restrict__ split) {
    const int64_t br = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (br >= nbr) return;
    const int64_t a = blk_ptr[br * nbc], b = blk_ptr[(br + 1) * nbc];
    const int64_t z = b - a;
    const int64_t nu = z <= unit_nnz ? 1 : (z + unit_nnz - 1) / unit_nnz;
    const int32_t u0 = unit_ptr[br], s0 = slot_ptr[br];
    for (int64_t i = 0; i < nu; ++i) {
        const int64_t k0 = a + i * unit_nnz;
        const int64_t k1 = k0 + unit_nnz < b ? k0 + unit_nnz : b;
        units[u0 + i] = make_int4((int)br, (int)k0, (int)k1, nu > 1 ? s0 + (int)i : -1);
    }
    if (nu > 1) split[split_ptr[br]] = make_int4((int)br, s0, (int)nu, 0);
}

hipError_t csbh_units(const int32_t* blk_ptr, int64_t nbr, int64_t nbc, int64_t unit_nnz,
                      const int32_t* unit_ptr, const int32_t* slot_ptr, const int32_t* split_ptr,
                      int4* units, int4* split, hipStream_t s) {
    SPX_LAUNCH("csbh_units", k_csbh_units, dim3(spx_div_up(nbr, 256)), dim3(256), 0, s, blk_ptr, nbr,
                       nbc, unit_nnz, unit_ptr, slot_ptr, split_ptr, units, split);
    return hipGetLastError();
}
