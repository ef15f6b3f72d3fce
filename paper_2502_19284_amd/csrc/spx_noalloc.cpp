// spx_noalloc.cpp -- Y = A X for callers that cannot allocate device memory.
//
// Same products as spx_spmm (the same kernels and plan), with every scratch buffer carved from
// one static device array of this file instead of handle-held allocations: the row-major copy of
// a column-major X chunk, the row-major results of a chunk for a column-major Y, the hot rows of
// X, the merge tiles' carries and, for row-split matrices, the merge tile starts.  No buffer needs
// to start at zero: every launch writes what the next one reads.  Each GPU holds its own copy of
// the array; its address is obtained once per device, with that device current, and only that
// address is passed to kernels.  Calls that overlap on one GPU share the array and race.
#include <hip/hip_runtime.h>

#include <cstdio>
#include <mutex>

#include "spx_internal.h"

#define SPX_NOALLOC_BYTES ((size_t)32 << 20)
#define SPX_NOALLOC_MAX_DEVICES 64

static __device__ __align__(256) unsigned char scratch[SPX_NOALLOC_BYTES];

static std::mutex g_scratch_mu;
static void* g_scratch_ptr[SPX_NOALLOC_MAX_DEVICES];

spx_status spmm_check(spx_matrix A, int32_t k, const void* x, int64_t ldx, const void* y,
                      int64_t ldy, spx_layout layout);

static spx_status noalloc_fail(spx_status s, const char* fmt, size_t a, size_t b) {
    char msg[256];
    snprintf(msg, sizeof msg, fmt, a, b);
    return spx_fail(s, msg);
}

// Device address of this GPU's scratch array (looked up on the first call on the device).
static spx_status scratch_address(int dev, unsigned char** out) {
    if (dev < 0 || dev >= SPX_NOALLOC_MAX_DEVICES)
        return noalloc_fail(SPX_ERR_UNSUPPORTED, "device %zu beyond the %zu supported", (size_t)dev,
                            (size_t)SPX_NOALLOC_MAX_DEVICES);
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void* p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return noalloc_fail(SPX_ERR_HIP, "hipGetSymbolAddress of the scratch array failed "
                                "(error %zu, device %zu)", (size_t)e, (size_t)dev);
        g_scratch_ptr[dev] = p;
    }
    *out = (unsigned char*)g_scratch_ptr[dev];
    return SPX_OK;
}

static size_t align256(size_t b) { return (b + 255) & ~(size_t)255; }

extern "C" spx_status spx_spmm_noalloc(spx_matrix A, int32_t k, const void* x, int64_t ldx,
                                       void* y, int64_t ldy, spx_layout layout, void* stream) {
    spx_status st = spmm_check(A, k, x, ldx, y, ldy, layout);
    if (st != SPX_OK) return st;
    const int64_t m = A->m, n = A->n;
    if (m == 0) return SPX_OK;
    const size_t es = A->value_type == SPX_F64 ? 8 : 4;
    const bool row_major = layout == SPX_ROW_MAJOR;
    const bool merge = A->fmt == SPX_CSR_MERGE;
    const int64_t tiles = merge ? A->mp_tiles : ((int64_t)m + A->nnz + MP_TILE - 1) / MP_TILE;
    const size_t kc = (size_t)spmm_chunk_cols(k);
    // scratch layout: [coords][carry rows][carries][X copy][Y results][hot rows]
    const size_t b_coords = merge ? 0 : align256(((size_t)tiles + 1) * sizeof(int2));
    const size_t b_crow = align256(((size_t)tiles + 1) * 4);
    const size_t b_carry = align256(((size_t)tiles + 1) * kc * 8);
    const size_t b_z = (!row_major && n > 0) ? align256((size_t)n * kc * es) : 0;
    const size_t b_w = !row_major ? align256((size_t)m * kc * es) : 0;
    const size_t b_h = A->nhot > 0 ? align256((size_t)A->nhot * kc * es) : 0;
    const size_t need = b_coords + b_crow + b_carry + b_z + b_w + b_h;
    if (need > SPX_NOALLOC_BYTES)
        return noalloc_fail(SPX_ERR_RANGE, "this product needs %zu bytes of scratch; the static "
                            "scratch holds %zu (use spx_spmm)", need, SPX_NOALLOC_BYTES);
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return spx_fail(SPX_ERR_HIP, "hipGetDevice failed");
    if (dev != A->device)
        return noalloc_fail(SPX_ERR_INVALID_ARG, "current device %zu is not the matrix's (%zu)",
                            (size_t)dev, (size_t)A->device);
    unsigned char* base = nullptr;
    st = scratch_address(dev, &base);
    if (st != SPX_OK) return st;
    hipStream_t s = (hipStream_t)stream;
    SpmmPlan P;
    size_t off = 0;
    if (merge) {
        P.coords = A->mp_coords;
    } else {
        int2* c = (int2*)(base + off);
        off += b_coords;
        if (tiles > 0) {
            const hipError_t e = launch_merge_coords(A->row_ptr, A->m, A->nnz, c, (int32_t)tiles, s);
            if (e != hipSuccess) return spx_fail(SPX_ERR_HIP, hipGetErrorString(e));
        }
        P.coords = c;
    }
    P.tiles = (int32_t)tiles;
    P.carry_row = (int32_t*)(base + off);
    off += b_crow;
    P.carry_val = (double*)(base + off);
    off += b_carry;
    P.z = b_z ? (void*)(base + off) : nullptr;
    off += b_z;
    P.w = b_w ? (void*)(base + off) : nullptr;
    off += b_w;
    P.h = b_h ? (void*)(base + off) : nullptr;
    A->last_stream = s;
    const hipError_t e = spmm_crs(A, P, k, x, ldx, y, ldy, row_major ? 1 : 0, s);
    if (e != hipSuccess) return spx_fail(SPX_ERR_HIP, hipGetErrorString(e));
    return SPX_OK;
}
