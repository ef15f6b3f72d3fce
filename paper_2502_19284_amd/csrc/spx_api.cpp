// spx_api.cpp -- C ABI of libspx: argument checks, conversion orchestration, product dispatch.
//
// Every argument check runs on the host before any HIP call, so invalid requests fail without
// touching a device.  Device work is enqueued on the caller's stream; conversion reads back a few
// counters (index errors, entry count, work-unit counts) and therefore synchronises the stream.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <limits>
#include <new>
#include <string>
#include <vector>

#include "spx_internal.h"

// ------------------------------------------------------------------ errors

static thread_local std::string g_last_error;

static spx_status fail(spx_status s, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
static spx_status fail(spx_status s, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return s;
}

#define HIP_TRY(expr)                                                                           \
    do {                                                                                        \
        hipError_t e_ = (expr);                                                                 \
        if (e_ != hipSuccess)                                                                   \
            return fail(SPX_ERR_HIP, "%s failed: %s (%s:%d)", #expr, hipGetErrorString(e_),    \
                        __FILE__, __LINE__);                                                    \
    } while (0)

extern "C" const char* spx_status_string(spx_status s) {
    switch (s) {
        case SPX_OK: return "SPX_OK";
        case SPX_ERR_INVALID_ARG: return "SPX_ERR_INVALID_ARG";
        case SPX_ERR_INDEX: return "SPX_ERR_INDEX";
        case SPX_ERR_RANGE: return "SPX_ERR_RANGE";
        case SPX_ERR_ALIAS: return "SPX_ERR_ALIAS";
        case SPX_ERR_NOMEM: return "SPX_ERR_NOMEM";
        case SPX_ERR_HIP: return "SPX_ERR_HIP";
        case SPX_ERR_UNSUPPORTED: return "SPX_ERR_UNSUPPORTED";
        case SPX_ERR_DEVICE: return "SPX_ERR_DEVICE";
        default: return "SPX_ERR_UNKNOWN";
    }
}

// the same, for the other host sources of the library (spx_serve.cpp)
spx_status spx_fail(spx_status s, const char* msg) { return fail(s, "%s", msg); }

extern "C" const char* spx_last_error_message(void) { return g_last_error.c_str(); }

extern "C" const char* spx_version(void) { return "0.1.0"; }

// ------------------------------------------------------------------ allocation

static spx_alloc_fn g_alloc = nullptr;
static spx_free_fn g_free = nullptr;
static void* g_alloc_ctx = nullptr;

extern "C" spx_status spx_set_allocator(spx_alloc_fn alloc, spx_free_fn free_fn, void* ctx) {
    if ((alloc == nullptr) != (free_fn == nullptr))
        return fail(SPX_ERR_INVALID_ARG, "spx_set_allocator: give both functions or neither");
    g_alloc = alloc;
    g_free = free_fn;
    g_alloc_ctx = ctx;
    return SPX_OK;
}

void* spx_dev_alloc(size_t bytes, hipStream_t s) {
    if (bytes == 0) return nullptr;
    if (g_alloc) return g_alloc(bytes, (void*)s, g_alloc_ctx);
    void* p = nullptr;
    if (hipMalloc(&p, bytes) != hipSuccess) {
        (void)hipGetLastError();
        return nullptr;
    }
    return p;
}

void spx_dev_free(void* p, hipStream_t s) {
    if (!p) return;
    if (g_free) g_free(p, (void*)s, g_alloc_ctx);
    else (void)hipFree(p);
}

// Allocations of one call; freed on scope exit unless released to a handle.
struct AllocSet {
    hipStream_t s;
    std::vector<void*> ptrs;
    size_t bytes = 0;
    explicit AllocSet(hipStream_t st) : s(st) {}
    ~AllocSet() {
        for (void* p : ptrs) spx_dev_free(p, s);
    }
    template <typename T>
    spx_status get(T** out, size_t count, const char* what) {
        *out = nullptr;
        if (count == 0) return SPX_OK;
        void* p = spx_dev_alloc(count * sizeof(T), s);
        if (!p) return fail(SPX_ERR_NOMEM, "device allocation of %zu bytes for %s failed",
                            count * sizeof(T), what);
        ptrs.push_back(p);
        bytes += count * sizeof(T);
        *out = (T*)p;
        return SPX_OK;
    }
};

#define SPX_TRY(expr)                  \
    do {                               \
        spx_status st_ = (expr);       \
        if (st_ != SPX_OK) return st_; \
    } while (0)

// ------------------------------------------------------------------ helpers

static int ceil_log2_u64(uint64_t v) {  // smallest b with 2^b >= v (v >= 1)
    int b = 0;
    while (b < 64 && (1ull << b) < v) ++b;
    return b;
}

// Block size rule of Section 3.1 (equation eq:CSB-BlockSize): start at 3 + ceil(log2 sqrt n),
// lower while beta > 2^16 or the beta-entry output slice (doubles) exceeds the LDS budget.
static int csbh_default_log2_beta(int64_t m, int64_t n) {
    const int64_t d = m > n ? m : n;
    int t = 0;
    while (t < 32 && (int64_t)1 << (2 * t) < d) ++t;  // 4^t >= d
    int k = t + 3;
    while (k > 0 && ((1ll << k) > (1ll << 16) || (1ll << k) * 8 > CB_LDS_BUDGET)) --k;
    return k;
}

static bool ranges_overlap(const void* a, size_t na, const void* b, size_t nb) {
    const uintptr_t a0 = (uintptr_t)a, b0 = (uintptr_t)b;
    return na > 0 && nb > 0 && a0 < b0 + nb && b0 < a0 + na;
}

extern "C" spx_status spx_convert_opts_default(spx_convert_opts* opts) {
    if (!opts) return fail(SPX_ERR_INVALID_ARG, "opts is NULL");
    opts->sum_duplicates = 1;
    opts->log2_beta = 0;
    opts->validate = 1;
    opts->tile_items = 0;
    opts->hot_columns = -1;
    opts->value_type = SPX_F64;
    return SPX_OK;
}

extern "C" double spx_break_even(double conv_fmt, double conv_ref, double spmv_ref,
                                 double spmv_fmt) {
    const double gain = spmv_ref - spmv_fmt;
    if (!(gain > 0)) return std::numeric_limits<double>::infinity();
    // a format that converts no slower and multiplies faster is ahead from the first product
    return conv_fmt <= conv_ref ? 0.0 : (conv_fmt - conv_ref) / gain;
}

// ------------------------------------------------------------------ conversion

static spx_status sync_read(void* host, const void* dev, size_t bytes, hipStream_t s) {
    HIP_TRY(hipMemcpyAsync(host, dev, bytes, hipMemcpyDeviceToHost, s));
    HIP_TRY(hipStreamSynchronize(s));
    return SPX_OK;
}

// Sort and count runs of equal keys.  Produces sorted keys and values, nnz_out, and (when
// repeats are summed) the scanned tile counts of run heads that the fused gather consumes.
struct SortedEntries {
    const uint64_t* keys = nullptr;
    const double* vals = nullptr;
    const uint32_t* head_tiles = nullptr;  // null when repeats are kept
    int64_t nnz_out = 0;
    MsdStats sort;
};

static spx_status build_keys_and_sort(const spx_coo_desc* coo, spx_format fmt, int k, int64_t nbc,
                                      int cbits, const int32_t* part_of, int K2, uint64_t* k0,
                                      uint64_t* v0, uint64_t* k1, uint64_t* v1,
                                      const MsdScratch& sc, Readback* rb_dev, hipStream_t s,
                                      SortedEntries* out, const uint64_t** vs, int* failed,
                                      uint32_t* head_tiles, int* heads,
                                      const int32_t* row_map);

// part_of / K2: BCOH partitions and Hilbert level, or CSBR column ranks and rank width; row_map:
// CSBR row rank of every triplet.
static spx_status sort_and_dedup(AllocSet& tmp, const spx_coo_desc* coo, spx_format fmt, int k,
                                 int64_t nbc, int cbits, int sum_dup, hipStream_t s,
                                 SortedEntries* out, const int32_t* part_of = nullptr,
                                 int K2 = 0, const int32_t* row_map = nullptr) {
    const int64_t E = coo->nnz;
    uint64_t *k0, *k1, *v0, *v1;
    uint32_t* tsums;
    Readback* rb_dev;
    SPX_TRY(tmp.get(&k0, E, "sort keys"));
    SPX_TRY(tmp.get(&k1, E, "sort keys"));
    SPX_TRY(tmp.get(&v0, E, "sort values"));
    SPX_TRY(tmp.get(&v1, E, "sort values"));
    SPX_TRY(tmp.get(&tsums, scan_tile_count(E), "scan tile sums"));
    SPX_TRY(tmp.get(&rb_dev, 1, "readback"));
    MsdScratch sc;
    sc.z = msd_sizes(E);
    for (int i = 0; i < 2; ++i) {
        SPX_TRY(tmp.get(&sc.seg_start[i], (size_t)sc.z.cap_big, "sort segments"));
        SPX_TRY(tmp.get(&sc.seg_len[i], (size_t)sc.z.cap_big, "sort segments"));
    }
    SPX_TRY(tmp.get(&sc.tbase, (size_t)sc.z.cap_big + 1, "sort segment tiles"));
    SPX_TRY(tmp.get(&sc.tile_seg, (size_t)sc.z.cap_tiles, "sort tile segments"));
    SPX_TRY(tmp.get(&sc.hist, (size_t)sc.z.hist, "radix histogram"));
    SPX_TRY(tmp.get(&sc.tile_sums, (size_t)sc.z.tile_sums, "scan tile sums"));
    SPX_TRY(tmp.get(&sc.chunks, (size_t)sc.z.cap_chunks, "sort chunks"));
    uint32_t* ctr;
    SPX_TRY(tmp.get(&ctr, 16, "sort counters"));
    sc.counters = ctr;

    HIP_TRY(launch_init_readback(rb_dev, s));
    const uint64_t* vs = nullptr;
    int failed = 0, heads = 0;
    if (!spx_is_bcoh(fmt) && fmt != SPX_CSB_RANKED && E > RS_LOCAL_MAX) {
        // CRS and CSB: the sort's first level builds the keys from the triplets (and checks
        // them)
        const int order = !spx_is_csb(fmt) ? 0 : fmt == SPX_CSB_HILBERT ? 1 : 2;
        const MsdTripletSource src{coo->row, coo->col, coo->m, coo->n, order, cbits, k, nbc};
        HIP_TRY(radix_sort_msd(k0, v0, k1, v1, (const uint64_t*)coo->val, E, 0, sc, s,
                               &out->keys, &vs, &failed, &out->sort, &src,
                               sum_dup ? tsums : nullptr, &heads));
    } else {
        SPX_TRY(build_keys_and_sort(coo, fmt, k, nbc, cbits, part_of, K2, k0, v0, k1, v1, sc,
                                    rb_dev, s, out, &vs, &failed, sum_dup ? tsums : nullptr,
                                    &heads, row_map));
    }
    if (failed == 2)
        return fail(SPX_ERR_INDEX, "a triplet index lies outside [0,%d) x [0,%d)", coo->m, coo->n);
    if (failed) return fail(SPX_ERR_DEVICE, "radix sort: a device-side list overflowed");
    out->vals = (const double*)vs;
    if (!sum_dup) {
        out->head_tiles = nullptr;
        out->nnz_out = E;
        return SPX_OK;
    }
    Readback rb;
    if (heads)  // run heads were counted per tile inside the sort
        HIP_TRY(launch_head_tiles_scan(tsums, E, &rb_dev->totals[0], s));
    else
        HIP_TRY(launch_dedup_count(out->keys, E, tsums, &rb_dev->totals[0], s));
    SPX_TRY(sync_read(&rb, rb_dev, sizeof rb, s));
    out->nnz_out = rb.totals[0];
    out->head_tiles = tsums;
    return SPX_OK;
}

// Keys by the format's key function (keys kernel, index check), then the sort.
static spx_status build_keys_and_sort(const spx_coo_desc* coo, spx_format fmt, int k, int64_t nbc,
                                      int cbits, const int32_t* part_of, int K2, uint64_t* k0,
                                      uint64_t* v0, uint64_t* k1, uint64_t* v1,
                                      const MsdScratch& sc, Readback* rb_dev, hipStream_t s,
                                      SortedEntries* out, const uint64_t** vs, int* failed,
                                      uint32_t* head_tiles, int* heads,
                                      const int32_t* row_map) {
    const int64_t E = coo->nnz;
    if (spx_is_bcoh(fmt))
        HIP_TRY(launch_keys_bcoh(coo->row, coo->col, E, coo->m, coo->n, part_of, k, K2,
                                 fmt == SPX_BCOHCH, k0, &rb_dev->err, rb_dev->masks, s));
    else if (fmt == SPX_CSB_RANKED)  // part_of: column ranks, row_map: triplets' row ranks,
                                     // K2: rank width
        HIP_TRY(launch_keys_csbr(row_map, coo->col, E, coo->m, coo->n, part_of, K2, k0,
                                 &rb_dev->err, rb_dev->masks, s));
    else if (spx_is_csb(fmt))
        HIP_TRY(launch_keys_csb(coo->row, coo->col, E, coo->m, coo->n, k, nbc,
                                fmt == SPX_CSB_HILBERT, k0, &rb_dev->err, rb_dev->masks, s));
    else
        HIP_TRY(launch_keys_csr(coo->row, coo->col, E, coo->m, coo->n, cbits, k0, &rb_dev->err,
                                rb_dev->masks, s));
    Readback rb;
    SPX_TRY(sync_read(&rb, rb_dev, sizeof rb, s));
    if (rb.err) {
        *failed = 2;
        return SPX_OK;
    }
    const uint64_t vary = rb.masks[0] ^ rb.masks[1];
    HIP_TRY(radix_sort_msd(k0, v0, k1, v1, (const uint64_t*)coo->val, E, vary, sc, s, &out->keys,
                           vs, failed, &out->sort, nullptr, head_tiles, heads));
    return SPX_OK;
}

// Moves an allocation of `tmp` to the handle, which frees it in spx_matrix_destroy.
static void keep(AllocSet& tmp, spx_matrix_s* A, void* p) {
    if (!p) return;
    for (auto& q : tmp.ptrs)
        if (q == p) {
            q = nullptr;
            A->owned.push_back(p);
            return;
        }
}

// The stored values, once val_out holds the FP64 sums of every run: FP64 values are kept by the
// handle; reduced-precision ones are rounded once into a buffer of their own, and val_out is left
// to be released with the other temporaries.
static spx_status finish_values(AllocSet& tmp, spx_matrix_s* A, double* val_out, int64_t nnz,
                                spx_dtype vt, hipStream_t s) {
    A->value_type = vt;
    if (vt == SPX_F64) {
        keep(tmp, A, val_out);
        A->val = val_out;
        return SPX_OK;
    }
    void* lp = nullptr;
    if (vt == SPX_F32) {
        float* f;
        SPX_TRY(tmp.get(&f, (size_t)std::max<int64_t>(nnz, 1), "FP32 values"));
        lp = f;
    } else {
        uint16_t* h;
        SPX_TRY(tmp.get(&h, (size_t)std::max<int64_t>(nnz, 1), "bfloat16 values"));
        lp = h;
    }
    keep(tmp, A, lp);
    A->val_lp = lp;
    HIP_TRY(launch_round_values(val_out, nnz, vt, lp, s));
    return SPX_OK;
}

// Hot-column compaction: the (at most hot_max) columns with the largest sampled entry counts get
// dense ranks, and their entries will store ~rank.  Counts are sampled from the sorted keys
// (repeats included).  The threshold is the smallest sampled count whose column set fits in
// hot_max, found by bisection on device-side counts.  On return *hm describes the set (bitmap +
// word prefixes, conversion temporaries) and the handle owns hot_cols and the x_hot scratch.
static spx_status select_hot_columns(AllocSet& tmp, spx_matrix_s* A, int32_t hot_opt,
                                     const uint64_t* keys, int64_t E, uint64_t cmask,
                                     Readback* rb_dev, hipStream_t s, HotMap* hm) {
    const int64_t n = A->n;
    *hm = HotMap{};
    int64_t hot_max = hot_opt;
    if (hot_opt < 0) hot_max = n >= HOT_AUTO_MIN_N ? HOT_AUTO_MAX : 0;
    if (hot_max > n) hot_max = n;
    if (hot_max <= 0 || E <= 0) return SPX_OK;
    uint32_t *freq, *tsums, *pre;
    uint64_t* bits;
    const int64_t nwords = (n + 63) / 64;
    SPX_TRY(tmp.get(&freq, (size_t)n, "column counts"));
    SPX_TRY(tmp.get(&tsums, scan_tile_count(n), "scan tile sums"));
    SPX_TRY(tmp.get(&bits, (size_t)nwords, "hot bitmap"));
    SPX_TRY(tmp.get(&pre, (size_t)nwords, "hot word prefixes"));
    HIP_TRY(hipMemsetAsync(freq, 0, (size_t)n * 4, s));
    // samples: runs of HOT_RUN consecutive keys, one run per HOT_RUN * stride keys
    const int64_t stride = E > HOT_MAX_SAMPLES ? (E + HOT_MAX_SAMPLES - 1) / HOT_MAX_SAMPLES : 1;
    int64_t ns = E;
    if (stride > 1) {
        const int64_t span = HOT_RUN * stride, runs = (E + span - 1) / span;
        const int64_t last = E - (runs - 1) * span;
        ns = (runs - 1) * HOT_RUN + (last < HOT_RUN ? last : HOT_RUN);
    }
    {
        uint64_t *s0, *s1, *p0, *p1;
        uint32_t *shist, *stsums;
        SPX_TRY(tmp.get(&s0, (size_t)ns, "column samples"));
        SPX_TRY(tmp.get(&s1, (size_t)ns, "column samples"));
        SPX_TRY(tmp.get(&p0, (size_t)ns, "column samples"));
        SPX_TRY(tmp.get(&p1, (size_t)ns, "column samples"));
        const size_t hn = radix_hist_elems(ns);
        SPX_TRY(tmp.get(&shist, hn, "radix histogram"));
        SPX_TRY(tmp.get(&stsums, scan_tile_count((int64_t)hn), "scan tile sums"));
        HIP_TRY(launch_hot_sample(keys, stride, ns, cmask, s0, s));
        const uint64_t *sorted, *unused;
        HIP_TRY(radix_sort_pairs(s0, p0, s1, p1, s0, ns, cmask, shist, stsums, s, &sorted,
                                 &unused));
        HIP_TRY(launch_hot_count_sorted(sorted, ns, freq, s));
    }
    Readback rb;
    auto count_ge = [&](uint32_t tau, uint32_t* out) -> spx_status {
        HIP_TRY(launch_hot_count_ge(freq, n, tau, tsums, &rb_dev->totals[3], s));
        SPX_TRY(sync_read(&rb, rb_dev, sizeof rb, s));
        *out = rb.totals[3];
        return SPX_OK;
    };
    // smallest tau >= 1 with count_ge(tau) <= hot_max; count_ge is non-increasing in tau.  A
    // histogram of the counts answers every tau below HOT_HIST_BINS - 1 with one readback;
    // larger thresholds fall back to bisection with device-side counts.
    uint32_t* fh;
    SPX_TRY(tmp.get(&fh, HOT_HIST_BINS, "count histogram"));
    HIP_TRY(hipMemsetAsync(fh, 0, HOT_HIST_BINS * 4, s));
    HIP_TRY(launch_hot_freq_hist(freq, n, fh, s));
    std::vector<uint32_t> hh(HOT_HIST_BINS);
    SPX_TRY(sync_read(hh.data(), fh, HOT_HIST_BINS * 4, s));
    uint64_t suffix = 0;  // count_ge(t) for t = HOT_HIST_BINS - 1 down to 1
    uint32_t tau = 0;
    uint64_t nhot_hist = 0;  // count_ge(tau) when tau comes from the histogram
    for (int t = HOT_HIST_BINS - 1; t >= 1; --t) {
        suffix += hh[t];
        if (suffix > (uint64_t)hot_max) break;
        tau = (uint32_t)t;
        nhot_hist = suffix;
    }
    if (tau == 0) {  // even count_ge(HOT_HIST_BINS - 1) exceeds hot_max
        uint64_t lo = HOT_HIST_BINS, hi = (uint64_t)ns + 1;  // no column has more than ns
        if (hi < lo) hi = lo;  // count_ge(hi) == 0
        while (lo < hi) {
            const uint64_t mid = (lo + hi) / 2;
            uint32_t c;
            SPX_TRY(count_ge((uint32_t)mid, &c));
            if (c <= (uint64_t)hot_max) hi = mid;
            else lo = mid + 1;
        }
        tau = (uint32_t)lo;
    }
    // the last bin holds every count >= HOT_HIST_BINS - 1, so for a threshold taken from the
    // histogram the suffix sum is the exact column count (no second readback)
    uint32_t nhot = (uint32_t)nhot_hist;
    if (tau >= HOT_HIST_BINS) SPX_TRY(count_ge(tau, &nhot));
    if (nhot == 0) return SPX_OK;
    int32_t* hot_cols;
    double* x_hot;
    SPX_TRY(tmp.get(&hot_cols, nhot, "hot columns"));
    SPX_TRY(tmp.get(&x_hot, nhot, "hot x"));
    keep(tmp, A, hot_cols);
    keep(tmp, A, x_hot);
    uint4* words;
    SPX_TRY(tmp.get(&words, (size_t)nwords, "hot words"));
    HIP_TRY(launch_hot_set(freq, n, tau, bits, pre, hot_cols, tsums, s));
    HIP_TRY(launch_hot_pack(bits, pre, nwords, words, s));
    A->hot_cols = hot_cols;
    A->x_hot = x_hot;
    A->nhot = (int32_t)nhot;
    hm->words = words;
    return SPX_OK;
}

// BCOHC / BCOHCH: partitions of whole rows with about equal raw entry counts (at most
// BH_WINDOW rows each), then one sort by (partition, Hilbert block index, position in block),
// the fused repeat-sum + populate step, and the block and partition tables.
static spx_status convert_bcoh(const spx_coo_desc* coo, spx_format fmt, int k, int K2,
                               spx_dtype vt, hipStream_t s, spx_matrix_s* A, AllocSet& tmp) {
    HIP_TRY(bcoh_prepare_kernel());
    const int64_t E = coo->nnz;
    const int32_t m = coo->m;
    Readback* rb_dev;
    Readback rb;
    SPX_TRY(tmp.get(&rb_dev, 1, "readback"));
    HIP_TRY(launch_init_readback(rb_dev, s));
    uint32_t *counts, *cum, *tsums;
    int32_t *part_of, *part_row;
    // more than 2^26 rows need at least 8192 partitions and 27 Hilbert levels: 68 key bits
    const int wbits = bcoh_row_bucket_bits(m);
    if (wbits < 0) return fail(SPX_ERR_RANGE, "BCOHC sort key exceeds 64 bits (m = %d)", m);
    SPX_TRY(tmp.get(&counts, (size_t)m + 1, "row counts"));
    SPX_TRY(tmp.get(&cum, (size_t)m + 1, "row count scan"));
    SPX_TRY(tmp.get(&part_of, (size_t)m + 1, "row partitions"));
    SPX_TRY(tmp.get(&part_row, (size_t)m + 2, "partition rows"));
    size_t tsn = scan_tile_count((int64_t)m + 2);
    if (scan_tile_count(E + 1) > tsn) tsn = scan_tile_count(E + 1);
    const size_t rhn = bcoh_rows_hist_elems(m, E, wbits);
    if (scan_tile_count((int64_t)rhn) > tsn) tsn = scan_tile_count((int64_t)rhn);
    SPX_TRY(tmp.get(&tsums, tsn, "scan tile sums"));
    HIP_TRY(launch_fill_i32((int32_t*)counts, (int64_t)m + 1, 0, s));
    uint32_t *rhist, *rtotal;
    int32_t* rows_out;
    SPX_TRY(tmp.get(&rhist, rhn > 0 ? rhn : 1, "row bucket histogram"));
    SPX_TRY(tmp.get(&rows_out, (size_t)(E > 0 ? E : 1), "rows by bucket"));
    SPX_TRY(tmp.get(&rtotal, 1, "row bucket total"));
    HIP_TRY(launch_bcoh_rows_bucketed(coo->row, coo->col, E, m, coo->n, wbits, rhist, rows_out,
                                      tsums, rtotal, counts, &rb_dev->err, s));
    HIP_TRY(launch_excl_scan_u32(counts, cum, m, tsums, &rb_dev->totals[1], s));
    const int64_t target64 = (E + BH_PARTS_TARGET - 1) / BH_PARTS_TARGET;
    const uint32_t target = (uint32_t)(target64 > (1 << 16) ? target64 : (1 << 16));
    HIP_TRY(launch_bcoh_partitions(cum, m, target, part_of, part_row, tsums, &rb_dev->totals[0],
                                   s));
    SPX_TRY(sync_read(&rb, rb_dev, sizeof rb, s));
    if (rb.err) return fail(SPX_ERR_INDEX, "a triplet index lies outside [0,%d) x [0,%d)", coo->m,
                            coo->n);
    const int32_t P = (int32_t)rb.totals[0];
    HIP_TRY(launch_fill_i32(part_row + P, 1, m, s));
    const int pbits = ceil_log2_u64((uint64_t)(P > 1 ? P : 1));
    if (pbits + 2 * (K2 + k) > 64) return fail(SPX_ERR_RANGE, "BCOHC sort key exceeds 64 bits");

    SortedEntries se;
    if (E > 0) SPX_TRY(sort_and_dedup(tmp, coo, fmt, k, 0, 0, 1, s, &se, part_of, K2));
    A->sort = se.sort;
    const int64_t nnz = se.nnz_out;
    A->nnz = nnz;
    double* val_out;
    uint32_t *packed, *flags;
    uint64_t* majors;
    SPX_TRY(tmp.get(&val_out, (size_t)nnz, "values"));
    SPX_TRY(tmp.get(&packed, (size_t)nnz, "packed indices"));
    SPX_TRY(tmp.get(&flags, (size_t)nnz, "block flags"));
    SPX_TRY(tmp.get(&majors, (size_t)nnz, "block keys"));
    keep(tmp, A, packed);
    A->packed = packed;
    int64_t nb = 0;
    if (nnz > 0) {
        HIP_TRY(launch_dedup_gather(se.keys, se.vals, E, se.head_tiles,
                                    fmt == SPX_BCOHC ? 3 : 4, 2 * k, HotMap{}, (int32_t*)packed,
                                    val_out, (int32_t*)flags, s, K2 + k, majors));
        if (scan_tile_count(nnz) > tsn) {
            SPX_TRY(tmp.get(&tsums, scan_tile_count(nnz), "scan tile sums"));
            tsn = scan_tile_count(nnz);
        }
        HIP_TRY(launch_incl_scan_u32(flags, nnz, tsums, &rb_dev->totals[2], s));
        SPX_TRY(sync_read(&rb, rb_dev, sizeof rb, s));
        nb = rb.totals[2];
    }
    SPX_TRY(finish_values(tmp, A, val_out, nnz, vt, s));
    int32_t *bptr, *bpart, *parts;
    uint32_t* bcoord;
    SPX_TRY(tmp.get(&bptr, (size_t)nb + 1, "block pointers"));
    SPX_TRY(tmp.get(&bcoord, (size_t)nb + 1, "block coordinates"));
    SPX_TRY(tmp.get(&bpart, (size_t)nb + 1, "block partitions"));
    SPX_TRY(tmp.get(&parts, 2 * ((size_t)P + 1), "partition table"));
    keep(tmp, A, bptr);
    keep(tmp, A, bcoord);
    keep(tmp, A, parts);
    HIP_TRY(launch_bcoh_blocks(flags, majors, nnz, K2, bptr, bcoord, bpart, s));
    HIP_TRY(launch_fill_i32(bptr + nb, 1, (int32_t)nnz, s));
    HIP_TRY(hipMemcpyAsync(parts, part_row, ((size_t)P + 1) * 4, hipMemcpyDeviceToDevice, s));
    HIP_TRY(launch_bcoh_part_blk(bpart, nb, P, parts + P + 1, s));
    A->bh_part_row = parts;
    A->bh_part_blk = parts + P + 1;
    A->bh_nparts = P;
    A->bh_blk_ptr = bptr;
    A->bh_blk_coord = bcoord;
    A->bh_nblocks = nb;
    A->parts = P;
    HIP_TRY(hipStreamSynchronize(s));
    return SPX_OK;
}

// Ranks by a stable device sort of (2^eb - 1 - count, first panel, last panel) with the index as
// payload (first / last NULL: by count alone): order[i] = index of rank i for the counted indices,
// rank_of[c] for all, *nranked_dev (device word) = their number.
static spx_status rank_by_counts(AllocSet& tmp, const uint32_t* counts, const uint32_t* first,
                                 const uint32_t* last, int32_t n, int eb, int pbits,
                                 int32_t* order, int32_t* rank_of, uint32_t* nranked_dev,
                                 hipStream_t s) {
    if (n <= 0) return SPX_OK;
    uint64_t *rk0, *rk1, *rv0, *rv1, *ridx;
    SPX_TRY(tmp.get(&ridx, (size_t)n, "rank payload"));
    SPX_TRY(tmp.get(&rk0, (size_t)n, "rank keys"));
    SPX_TRY(tmp.get(&rk1, (size_t)n, "rank keys"));
    SPX_TRY(tmp.get(&rv0, (size_t)n, "rank payload"));
    SPX_TRY(tmp.get(&rv1, (size_t)n, "rank payload"));
    MsdScratch sc;
    sc.z = msd_sizes(n);
    for (int i = 0; i < 2; ++i) {
        SPX_TRY(tmp.get(&sc.seg_start[i], (size_t)sc.z.cap_big, "sort segments"));
        SPX_TRY(tmp.get(&sc.seg_len[i], (size_t)sc.z.cap_big, "sort segments"));
    }
    SPX_TRY(tmp.get(&sc.tbase, (size_t)sc.z.cap_big + 1, "sort segment tiles"));
    SPX_TRY(tmp.get(&sc.tile_seg, (size_t)sc.z.cap_tiles, "sort tile segments"));
    SPX_TRY(tmp.get(&sc.hist, (size_t)sc.z.hist, "radix histogram"));
    SPX_TRY(tmp.get(&sc.tile_sums, (size_t)sc.z.tile_sums, "scan tile sums"));
    SPX_TRY(tmp.get(&sc.chunks, (size_t)sc.z.cap_chunks, "sort chunks"));
    uint32_t* ctr;
    SPX_TRY(tmp.get(&ctr, 16, "sort counters"));
    sc.counters = ctr;
    // the high bits of the index fill what the key has left: equal keys only among indices
    // that share them (a sort finishes long runs of equal keys by copying them, one workgroup
    // per run)
    const int cb = ceil_log2_u64((uint64_t)n);
    const int ib = std::max(0, std::min(cb, 64 - eb - 2 * pbits));
    HIP_TRY(launch_rank_keys(counts, first, last, n, eb, pbits, ib, cb - ib, rk0, ridx, s));
    const int kb = eb + 2 * pbits + ib;  // bits that can vary
    const uint64_t vary = kb >= 64 ? ~0ull : ((1ull << kb) - 1ull);
    const uint64_t *sorted, *vs;
    int failed = 0;
    MsdStats st;
    HIP_TRY(radix_sort_msd(rk0, rv0, rk1, rv1, ridx, n, vary, sc, s, &sorted, &vs, &failed, &st));
    if (failed) return fail(SPX_ERR_DEVICE, "radix sort: a device-side list overflowed");
    HIP_TRY(launch_rank_scatter(sorted, vs, n, eb, 2 * pbits + ib, order, rank_of, nranked_dev,
                                s));
    return SPX_OK;
}

// CSBR: raw triplets per row (bucketed count, checking every index) and the row ranking; raw
// triplets per column with the first and last panel each column meets, and the column ranking;
// triplets sorted by (panel, column rank, row rank) with repeats summed, block pointers over
// (panel, rank segment), then the CSBH work-unit tables over panels.
static spx_status convert_csbr(const spx_coo_desc* coo, const spx_convert_opts* o, hipStream_t s,
                               spx_matrix_s* A, AllocSet& tmp) {
    HIP_TRY(csbr_prepare_kernel());
    HIP_TRY(rowc_extent_prepare_kernel());
    const int64_t E = coo->nnz;
    const int32_t m = coo->m, n = coo->n;
    const int wbr = bcoh_row_bucket_bits(m);
    if (wbr < 0) return fail(SPX_ERR_RANGE, "CSBR: %d rows, more than 2^26", m);
    const int wbc = bcoh_row_bucket_bits(n);
    if (wbc < 0) return fail(SPX_ERR_RANGE, "CSBR: %d columns, more than 2^26", n);
    const int eb = ceil_log2_u64((uint64_t)E + 1);  // bits of a count
    Readback* rb_dev;
    SPX_TRY(tmp.get(&rb_dev, 1, "readback"));
    HIP_TRY(launch_init_readback(rb_dev, s));
    // scratch of both bucketed counts
    uint32_t *hist, *btotal, *tsums;
    int32_t* bucketed;
    const size_t hn = std::max(bcoh_rows_hist_elems(m, E, wbr), bcoh_rows_hist_elems(n, E, wbc));
    SPX_TRY(tmp.get(&hist, hn > 0 ? hn : 1, "bucket histogram"));
    SPX_TRY(tmp.get(&bucketed, (size_t)(E > 0 ? E : 1), "indices by bucket"));
    SPX_TRY(tmp.get(&btotal, 1, "bucket total"));
    size_t tsn = std::max(scan_tile_count(hn > 0 ? (int64_t)hn : 1),
                          scan_tile_count((int64_t)std::max(m, n) + 2));
    SPX_TRY(tmp.get(&tsums, tsn, "scan tile sums"));
    // 1. raw triplets per row, then the row ranks
    uint32_t* rcounts;
    int32_t *row_order, *row_rank;
    SPX_TRY(tmp.get(&rcounts, (size_t)m + 1, "row counts"));
    SPX_TRY(tmp.get(&row_order, (size_t)std::max<int32_t>(m, 1), "row order"));
    SPX_TRY(tmp.get(&row_rank, (size_t)std::max<int32_t>(m, 1), "row ranks"));
    HIP_TRY(launch_fill_u32(rcounts, (int64_t)m + 1, 0u, s));
    HIP_TRY(launch_bcoh_rows_bucketed(coo->row, coo->col, E, m, n, wbr, hist, bucketed, tsums,
                                      btotal, rcounts, &rb_dev->err, s));
    Readback rb;
    SPX_TRY(sync_read(&rb, rb_dev, sizeof rb, s));
    if (rb.err)
        return fail(SPX_ERR_INDEX, "a triplet index lies outside [0,%d) x [0,%d)", m, n);
    SPX_TRY(rank_by_counts(tmp, rcounts, nullptr, nullptr, m, eb, 0, row_order, row_rank,
                           &rb_dev->totals[2], s));
    SPX_TRY(sync_read(&rb, rb_dev, sizeof rb, s));
    const int32_t nrows = (int32_t)rb.totals[2];
    const int64_t npan = std::max<int64_t>(1, ((int64_t)nrows + (1 << CR_PB) - 1) >> CR_PB);
    const int pbits = ceil_log2_u64((uint64_t)npan);  // bits of a panel
    if (eb + 2 * pbits > 64)
        return fail(SPX_ERR_RANGE, "CSBR: ranking key of %d bits exceeds 64", eb + 2 * pbits);
    // 2. raw triplets per column, with the first and last panel each column meets, then the
    //    column ranks.  Rows and columns trade places in the bucketed count, and a triplet's
    //    panel (row rank >> CR_PB, below 2^17) rides along in the bits above the column's place
    //    in its bucket.
    uint32_t *counts, *first, *last;
    SPX_TRY(tmp.get(&counts, (size_t)n + 1, "column counts"));
    SPX_TRY(tmp.get(&first, (size_t)std::max<int32_t>(n, 1), "first panel of each column"));
    SPX_TRY(tmp.get(&last, (size_t)std::max<int32_t>(n, 1), "last panel of each column"));
    HIP_TRY(launch_fill_u32(counts, (int64_t)n + 1, 0u, s));
    HIP_TRY(launch_fill_u32(first, n, 0xFFFFFFFFu, s));
    HIP_TRY(launch_fill_u32(last, n, 0u, s));
    int32_t* trank;  // row rank of every triplet, for the sort keys
    SPX_TRY(tmp.get(&trank, (size_t)(E > 0 ? E : 1), "row rank of each triplet"));
    HIP_TRY(launch_bcoh_rows_bucketed(coo->col, coo->row, E, n, m, wbc, hist, bucketed, tsums,
                                      btotal, counts, &rb_dev->err, s, CR_PB, first, last,
                                      row_rank, trank));
    int32_t *order, *rank_of;
    SPX_TRY(tmp.get(&order, (size_t)std::max<int32_t>(n, 1), "column order"));
    SPX_TRY(tmp.get(&rank_of, (size_t)std::max<int32_t>(n, 1), "column ranks"));
    SPX_TRY(rank_by_counts(tmp, counts, first, last, n, eb, pbits, order, rank_of,
                           &rb_dev->totals[3], s));
    SPX_TRY(sync_read(&rb, rb_dev, sizeof rb, s));
    const int32_t nranked = (int32_t)rb.totals[3];
    const int rbits = std::max(CR_RB, ceil_log2_u64((uint64_t)std::max<int32_t>(nranked, 1)));
    const int64_t nseg = (int64_t)1 << (rbits - CR_RB);
    if (ceil_log2_u64((uint64_t)npan) + rbits + CR_PB > 64)
        return fail(SPX_ERR_RANGE, "CSBR sort key exceeds 64 bits");
    if ((double)npan * (double)nseg >= 2147483647.0)
        return fail(SPX_ERR_RANGE, "CSBR: %lld x %lld blocks exceed the int32 block pointer range",
                    (long long)npan, (long long)nseg);
    keep(tmp, A, order);
    keep(tmp, A, row_order);
    keep(tmp, A, row_rank);
    A->cr_order = order;
    A->cr_nranked = nranked;
    A->cr_row_order = row_order;
    A->cr_row_rank = row_rank;
    A->cr_nrows = nrows;
    A->log2_beta = CR_PB;
    A->nbr = npan;
    A->nbc = nseg;
    // 3. sort by (panel, column rank, row rank), sum repeats, populate
    SortedEntries se;
    if (E > 0)
        SPX_TRY(sort_and_dedup(tmp, coo, SPX_CSB_RANKED, 0, nseg, 0, o->sum_duplicates, s, &se,
                               rank_of, rbits, trank));
    A->sort = se.sort;
    const int64_t nnz = se.nnz_out;
    A->nnz = nnz;
    double* val_out;
    uint32_t* packed;
    int32_t* bp;
    const int64_t nblk = npan * nseg;
    SPX_TRY(tmp.get(&val_out, (size_t)nnz, "values"));
    SPX_TRY(tmp.get(&packed, (size_t)nnz, "packed indices"));
    SPX_TRY(tmp.get(&bp, (size_t)nblk + 1, "blk_ptr"));
    keep(tmp, A, packed);
    keep(tmp, A, bp);
    A->packed = packed;
    A->blk_ptr = bp;
    HIP_TRY(launch_fill_i32(bp, nblk + 1, 0, s));
    if (se.head_tiles)
        HIP_TRY(launch_dedup_gather(se.keys, se.vals, E, se.head_tiles, 5, 32, HotMap{},
                                    (int32_t*)packed, val_out, bp + 1, s));
    else
        HIP_TRY(launch_gather_csbr(se.keys, se.vals, nullptr, E, nnz, packed, val_out, bp + 1, s));
    if (scan_tile_count(nblk) > tsn) {
        SPX_TRY(tmp.get(&tsums, scan_tile_count(nblk), "scan tile sums"));
        tsn = scan_tile_count(nblk);
    }
    HIP_TRY(launch_max_scan_i32(bp + 1, nblk, tsums, s));
    SPX_TRY(finish_values(tmp, A, val_out, nnz, o->value_type, s));
    // 4. work units over panels (heaviest first in launch order)
    const int64_t unit = o->tile_items > 0 ? o->tile_items : CR_UNIT_DEFAULT;
    int32_t *unit_ptr, *slot_ptr, *split_ptr;
    SPX_TRY(tmp.get(&unit_ptr, (size_t)npan, "unit ptr"));
    SPX_TRY(tmp.get(&slot_ptr, (size_t)npan, "slot ptr"));
    SPX_TRY(tmp.get(&split_ptr, (size_t)npan, "split ptr"));
    HIP_TRY(csbh_plan(bp, npan, nseg, unit, unit_ptr, slot_ptr, split_ptr, rb_dev->totals, s));
    SPX_TRY(sync_read(&rb, rb_dev, sizeof rb, s));
    A->cb_nunits = (int32_t)rb.totals[0];
    A->cb_nslots = (int32_t)rb.totals[1];
    A->cb_nsplit = (int32_t)rb.totals[2];
    int4 *units, *split;
    double *partials, *xr;
    SPX_TRY(tmp.get(&units, (size_t)A->cb_nunits, "units"));
    SPX_TRY(tmp.get(&split, (size_t)std::max<int32_t>(A->cb_nsplit, 1), "split panels"));
    SPX_TRY(tmp.get(&partials, (size_t)std::max<int32_t>(A->cb_nslots, 1) << CR_PB,
                    "partial slices"));
    double* yr;
    SPX_TRY(tmp.get(&xr, (size_t)std::max<int32_t>(nranked, 1), "ranked x"));
    SPX_TRY(tmp.get(&yr, (size_t)std::max<int32_t>(nrows, 1), "ranked y"));
    keep(tmp, A, units);
    keep(tmp, A, split);
    keep(tmp, A, partials);
    keep(tmp, A, xr);
    keep(tmp, A, yr);
    A->cb_units = units;
    A->cb_split = split;
    A->cb_partials = partials;
    A->cr_xr = xr;
    A->cr_yr = yr;
    HIP_TRY(csbh_units(bp, npan, nseg, unit, unit_ptr, slot_ptr, split_ptr, units, split, s));
    if (A->cb_nunits > 1) {
        // a unit's run time grows with its entries: launching the largest first keeps one large
        // unit from starting last (stable order among equal sizes)
        std::vector<int4> hu((size_t)A->cb_nunits);
        SPX_TRY(sync_read(hu.data(), units, hu.size() * sizeof(int4), s));
        std::stable_sort(hu.begin(), hu.end(),
                         [](const int4& a, const int4& b) { return a.z - a.y > b.z - b.y; });
        HIP_TRY(hipMemcpyAsync(units, hu.data(), hu.size() * sizeof(int4), hipMemcpyHostToDevice,
                               s));
        HIP_TRY(hipStreamSynchronize(s));
    }
    A->parts = A->cb_nunits;
    return SPX_OK;
}

static spx_status convert_impl(const spx_coo_desc* coo, spx_format fmt,
                               const spx_convert_opts* o, hipStream_t s, spx_matrix_s* A,
                               AllocSet& tmp) {
    const int64_t E = coo->nnz;
    const int32_t m = coo->m, n = coo->n;
    A->m = m;
    A->n = n;
    A->fmt = fmt;
    const int cbits = ceil_log2_u64((uint64_t)(n > 1 ? n : 1));
    const int rbits = ceil_log2_u64((uint64_t)(m > 1 ? m : 1));
    int k = 0;
    int64_t nbr = 0, nbc = 0;
    if (fmt == SPX_CSB_RANKED) return convert_csbr(coo, o, s, A, tmp);
    if (spx_is_bcoh(fmt)) {
        k = o->log2_beta > 0 ? o->log2_beta : csbh_default_log2_beta(m, n);
        if (k < 1 || k > 16)
            return fail(SPX_ERR_INVALID_ARG, "log2_beta %d outside [1,16]", k);
        nbr = ((int64_t)m + (1 << k) - 1) >> k;
        nbc = ((int64_t)n + (1 << k) - 1) >> k;
        const int K2 = ceil_log2_u64((uint64_t)std::max<int64_t>(1, std::max(nbr, nbc)));
        if (K2 + k > 31) return fail(SPX_ERR_RANGE, "matrix too large for the Hilbert order");
        A->log2_beta = k;
        A->nbr = nbr;
        A->nbc = nbc;
        return convert_bcoh(coo, fmt, k, K2, o->value_type, s, A, tmp);
    }
    if (spx_is_csb(fmt)) {
        k = o->log2_beta > 0 ? o->log2_beta : csbh_default_log2_beta(m, n);
        if (k < 1 || k > 16)
            return fail(SPX_ERR_INVALID_ARG, "log2_beta %d outside [1,16]", k);
        if (((int64_t)1 << k) * 8 > 160 * 1024 - 16)
            return fail(SPX_ERR_UNSUPPORTED, "log2_beta %d: output slice exceeds LDS", k);
        nbr = ((int64_t)m + (1 << k) - 1) >> k;
        nbc = ((int64_t)n + (1 << k) - 1) >> k;
        if (nbr < 1) nbr = 1;
        if (nbc < 1) nbc = 1;
        if ((double)nbr * (double)nbc >= 2147483647.0)
            return fail(SPX_ERR_RANGE, "%lld x %lld blocks exceed the int32 block pointer range",
                        (long long)nbr, (long long)nbc);
        const int kb = ceil_log2_u64((uint64_t)(nbr * nbc));
        if (kb + 2 * k > 64) return fail(SPX_ERR_RANGE, "CSBH sort key exceeds 64 bits");
        A->log2_beta = k;
        A->nbr = nbr;
        A->nbc = nbc;
    } else if (rbits + cbits > 64) {
        return fail(SPX_ERR_RANGE, "CRS sort key exceeds 64 bits");
    }

    SortedEntries se;
    if (E > 0) SPX_TRY(sort_and_dedup(tmp, coo, fmt, k, nbc, cbits, o->sum_duplicates, s, &se));
    A->sort = se.sort;
    const int64_t nnz = se.nnz_out;
    A->nnz = nnz;

    uint32_t* tsums;
    Readback* rb_dev;
    size_t tsn = scan_tile_count((int64_t)m + 2);
    SPX_TRY(tmp.get(&rb_dev, 1, "readback"));
    HIP_TRY(launch_init_readback(rb_dev, s));

    double* val_out;  // FP64 run sums (finish_values keeps or rounds them)
    SPX_TRY(tmp.get(&val_out, (size_t)nnz, "values"));

    if (spx_is_csb(fmt)) {
        const int64_t nblk = nbr * nbc;
        int32_t *bp;
        uint32_t* packed;
        SPX_TRY(tmp.get(&bp, (size_t)nblk + 1, "blk_ptr"));
        SPX_TRY(tmp.get(&packed, (size_t)nnz, "packed indices"));
        keep(tmp, A, bp);
        keep(tmp, A, packed);
        A->blk_ptr = bp;
        A->packed = packed;
        HIP_TRY(launch_fill_i32(bp, nblk + 1, 0, s));
        if (se.head_tiles)
            HIP_TRY(launch_dedup_gather(se.keys, se.vals, E, se.head_tiles,
                                        fmt == SPX_CSB_HILBERT ? 1 : 2, 2 * k, HotMap{},
                                        (int32_t*)packed, val_out, bp + 1, s));
        else
            HIP_TRY(launch_gather_csb(se.keys, se.vals, nullptr, E, nnz, k,
                                      fmt == SPX_CSB_HILBERT, packed, val_out, bp + 1, s));
        if (scan_tile_count(nblk) > tsn) tsn = scan_tile_count(nblk);
        SPX_TRY(tmp.get(&tsums, tsn, "scan tile sums"));
        HIP_TRY(launch_max_scan_i32(bp + 1, nblk, tsums, s));
        SPX_TRY(finish_values(tmp, A, val_out, nnz, o->value_type, s));
        // work units
        int64_t unit = o->tile_items > 0 ? o->tile_items : CB_UNIT_DEFAULT;
        int32_t *unit_ptr, *slot_ptr, *split_ptr;
        SPX_TRY(tmp.get(&unit_ptr, (size_t)nbr, "unit ptr"));
        SPX_TRY(tmp.get(&slot_ptr, (size_t)nbr, "slot ptr"));
        SPX_TRY(tmp.get(&split_ptr, (size_t)nbr, "split ptr"));
        HIP_TRY(csbh_plan(bp, nbr, nbc, unit, unit_ptr, slot_ptr, split_ptr, rb_dev->totals, s));
        Readback rb;
        SPX_TRY(sync_read(&rb, rb_dev, sizeof rb, s));
        A->cb_nunits = (int32_t)rb.totals[0];
        A->cb_nslots = (int32_t)rb.totals[1];
        A->cb_nsplit = (int32_t)rb.totals[2];
        int4 *units, *split;
        double* partials;
        SPX_TRY(tmp.get(&units, (size_t)A->cb_nunits, "units"));
        SPX_TRY(tmp.get(&split, (size_t)A->cb_nsplit, "split rows"));
        SPX_TRY(tmp.get(&partials, (size_t)A->cb_nslots << k, "partial slices"));
        keep(tmp, A, units);
        keep(tmp, A, split);
        keep(tmp, A, partials);
        A->cb_units = units;
        A->cb_split = split;
        A->cb_partials = partials;
        HIP_TRY(csbh_units(bp, nbr, nbc, unit, unit_ptr, slot_ptr, split_ptr, units, split, s));
        A->parts = A->cb_nunits;
        return SPX_OK;
    }

    // CRS formats
    int32_t *rp, *col;
    SPX_TRY(tmp.get(&rp, (size_t)m + 1, "row_ptr"));
    SPX_TRY(tmp.get(&col, (size_t)nnz, "col_ind"));
    keep(tmp, A, rp);
    keep(tmp, A, col);
    A->row_ptr = rp;
    A->col = col;
    HIP_TRY(launch_fill_i32(rp, (int64_t)m + 1, 0, s));
    HotMap hm;
    SPX_TRY(select_hot_columns(tmp, A, o->hot_columns, se.keys, E,
                               cbits >= 64 ? ~0ull : ((1ull << cbits) - 1ull), rb_dev, s, &hm));
    if (se.head_tiles)
        HIP_TRY(launch_dedup_gather(se.keys, se.vals, E, se.head_tiles, 0, cbits, hm, col,
                                    val_out, rp + 1, s));
    else
        HIP_TRY(launch_gather_csr(se.keys, se.vals, nullptr, E, nnz, cbits, hm, col, val_out,
                              rp + 1, s));
    SPX_TRY(tmp.get(&tsums, tsn, "scan tile sums"));
    HIP_TRY(launch_max_scan_i32(rp + 1, m, tsums, s));
    // (reduced precision: the hot x copy holds FP32 values, the buffer is large enough)
    SPX_TRY(finish_values(tmp, A, val_out, nnz, o->value_type, s));

    if (fmt == SPX_CSR_MERGE) {
        const int64_t total = (int64_t)m + nnz;
        const int64_t tiles = (total + MP_TILE - 1) / MP_TILE;
        if (tiles >= INT32_MAX) return fail(SPX_ERR_RANGE, "too many merge tiles");
        A->mp_tiles = (int32_t)tiles;
        int2* coords;
        int32_t* crow;
        double* cval;
        SPX_TRY(tmp.get(&coords, (size_t)tiles + 1, "merge coordinates"));
        SPX_TRY(tmp.get(&crow, (size_t)tiles, "carry rows"));
        SPX_TRY(tmp.get(&cval, (size_t)tiles, "carry values"));
        keep(tmp, A, coords);
        keep(tmp, A, crow);
        keep(tmp, A, cval);
        A->mp_coords = coords;
        A->mp_carry_row = crow;
        A->mp_carry_val = cval;
        if (tiles > 0) HIP_TRY(launch_merge_coords(rp, m, nnz, coords, (int32_t)tiles, s));
        A->parts = tiles;
        HIP_TRY(hipStreamSynchronize(s));
        return SPX_OK;
    }

    // row split
    uint32_t* tsb;
    SPX_TRY(tmp.get(&tsb, tsn, "scan tile sums"));
    HIP_TRY(rowsplit_count(rp, m, tsums, tsb, rb_dev->totals, s));
    Readback rb;
    SPX_TRY(sync_read(&rb, rb_dev, sizeof rb, s));
    const int32_t nflags = (int32_t)rb.totals[0];  // blocks + sentinel
    const int32_t nlong = (int32_t)rb.totals[1];
    A->rs_nb = nflags - 1;
    A->rs_nlong = nlong;
    int32_t *blocks, *long_rows = nullptr, *chunk_ptr = nullptr;
    SPX_TRY(tmp.get(&blocks, (size_t)nflags, "row blocks"));
    keep(tmp, A, blocks);
    A->rs_blocks = blocks;
    if (nlong > 0) {
        SPX_TRY(tmp.get(&long_rows, (size_t)nlong, "long rows"));
        SPX_TRY(tmp.get(&chunk_ptr, (size_t)nlong + 1, "chunk pointers"));
        keep(tmp, A, long_rows);
        keep(tmp, A, chunk_ptr);
    }
    A->rs_long_rows = long_rows;
    A->rs_chunk_ptr = chunk_ptr;
    HIP_TRY(rowsplit_fill(rp, m, tsums, tsb, blocks, long_rows, s));
    if (nlong > 0) {
        HIP_TRY(rowsplit_chunks(rp, long_rows, nlong, chunk_ptr, tsums, &rb_dev->totals[2], s));
        SPX_TRY(sync_read(&rb, rb_dev, sizeof rb, s));
        A->rs_nchunks = (int32_t)rb.totals[2];
        double* partials;
        SPX_TRY(tmp.get(&partials, (size_t)A->rs_nchunks, "chunk partials"));
        keep(tmp, A, partials);
        A->rs_partials = partials;
    }
    A->parts = A->rs_nb;
    HIP_TRY(hipStreamSynchronize(s));
    return SPX_OK;
}

static int64_t sum_owned_bytes(const spx_matrix_s* A) {
    int64_t b = 0;
    b += (A->row_ptr ? ((int64_t)A->m + 1) * 4 : 0);
    b += (A->col ? A->nnz * 4 : 0);
    b += (A->val ? A->nnz * 8 : 0);
    b += (A->val_lp ? A->nnz * (A->value_type == SPX_F32 ? 4 : 2) : 0);
    b += (A->blk_ptr ? (A->nbr * A->nbc + 1) * 4 : 0);
    b += (A->packed ? A->nnz * 4 : 0);
    b += (A->bh_blk_ptr ? (A->bh_nblocks + 1) * 8 + 8 * ((int64_t)A->bh_nparts + 1) : 0);
    b += (A->mp_coords ? ((int64_t)A->mp_tiles + 1) * 8 + (int64_t)A->mp_tiles * 12 : 0);
    b += (A->rs_blocks ? ((int64_t)A->rs_nb + 1) * 4 : 0);
    b += (A->rs_long_rows ? (int64_t)A->rs_nlong * 8 + 4 + (int64_t)A->rs_nchunks * 8 : 0);
    b += (A->cb_units ? (int64_t)A->cb_nunits * 16 + (int64_t)A->cb_nsplit * 16 : 0);
    b += (A->cb_partials ? ((int64_t)A->cb_nslots << A->log2_beta) * 8 : 0);
    b += (int64_t)A->nhot * 12;
    // CSBR: column order and ranked x, row order and ranked y, rank of every row
    b += ((int64_t)A->cr_nranked * 12 + (int64_t)A->cr_nrows * 12 +
          (A->cr_row_rank ? (int64_t)A->m * 4 : 0));
    return b;
}

extern "C" spx_status spx_convert(const spx_coo_desc* coo, spx_format fmt,
                                  const spx_convert_opts* opts, void* stream, spx_matrix* out,
                                  spx_convert_report* rep) {
    g_last_error.clear();
    if (!out) return fail(SPX_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    if (!coo) return fail(SPX_ERR_INVALID_ARG, "coo is NULL");
    if (!spx_is_crs(fmt) && !spx_is_csb(fmt) && !spx_is_bcoh(fmt) && fmt != SPX_CSB_RANKED)
        return fail(SPX_ERR_INVALID_ARG, "unknown format %d", (int)fmt);
    if (coo->m < 0 || coo->n < 0 || coo->nnz < 0)
        return fail(SPX_ERR_INVALID_ARG, "negative size (m=%d n=%d nnz=%lld)", coo->m, coo->n,
                    (long long)coo->nnz);
    if (coo->nnz >= 2147483647LL)
        return fail(SPX_ERR_RANGE, "nnz %lld does not fit the int32 index range",
                    (long long)coo->nnz);
    if (coo->val_type != SPX_F64)
        return fail(SPX_ERR_UNSUPPORTED, "value type %d (only SPX_F64)", (int)coo->val_type);
    if (coo->nnz > 0 && (!coo->row || !coo->col || !coo->val))
        return fail(SPX_ERR_INVALID_ARG, "null triplet array with nnz > 0");
    if (coo->nnz > 0 && (coo->m == 0 || coo->n == 0))
        return fail(SPX_ERR_INDEX, "entries given for an empty (%d x %d) matrix", coo->m, coo->n);
    spx_convert_opts o;
    spx_convert_opts_default(&o);
    if (opts) o = *opts;
    if (o.sum_duplicates != 0 && o.sum_duplicates != 1)
        return fail(SPX_ERR_INVALID_ARG, "sum_duplicates must be 0 or 1");
    if (o.log2_beta < 0 || o.log2_beta > 16)
        return fail(SPX_ERR_INVALID_ARG, "log2_beta %d outside [0,16]", o.log2_beta);
    if (o.tile_items < 0) return fail(SPX_ERR_INVALID_ARG, "tile_items < 0");
    if (o.hot_columns < -1) return fail(SPX_ERR_INVALID_ARG, "hot_columns < -1");
    if (o.value_type != SPX_F64 && o.value_type != SPX_F32 && o.value_type != SPX_BF16)
        return fail(SPX_ERR_INVALID_ARG, "unknown value_type %d", (int)o.value_type);
    if (fmt == SPX_CSB_RANKED && o.log2_beta != 0 && o.log2_beta != CR_PB)
        return fail(SPX_ERR_UNSUPPORTED, "CSBR panels are 2^%d rows (log2_beta 0 or %d)", CR_PB,
                    CR_PB);
    if (spx_is_bcoh(fmt) && !o.sum_duplicates)
        return fail(SPX_ERR_UNSUPPORTED, "BCOHC/BCOHCH are built with repeats summed");
    if (!spx_is_csb(fmt) && fmt != SPX_CSB_RANKED && o.tile_items != 0)
        return fail(SPX_ERR_UNSUPPORTED, "tile_items is only adjustable for CSB/CSBH/CSBR");

    hipStream_t s = (hipStream_t)stream;
    int device = 0;
    HIP_TRY(hipGetDevice(&device));
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    if (rep) {
        HIP_TRY(hipEventCreate(&ev0));
        if (hipEventCreate(&ev1) != hipSuccess) {
            (void)hipEventDestroy(ev0);
            return fail(SPX_ERR_HIP, "hipEventCreate failed");
        }
        (void)hipEventRecord(ev0, s);
    }
    spx_matrix_s* A = new (std::nothrow) spx_matrix_s();
    if (!A) return fail(SPX_ERR_NOMEM, "host allocation failed");
    A->device = device;
    spx_status st;
    {
        AllocSet tmp(s);
        st = convert_impl(coo, fmt, &o, s, A, tmp);
        if (st == SPX_OK) {
            hipError_t e = hipStreamSynchronize(s);
            if (e != hipSuccess)
                st = fail(SPX_ERR_HIP, "conversion failed on the device: %s",
                          hipGetErrorString(e));
        } else {
            (void)hipStreamSynchronize(s);
        }
    }  // temporaries freed here
    if (st != SPX_OK) {
        for (void* p : A->owned) spx_dev_free(p, s);
        delete A;
        if (ev0) (void)hipEventDestroy(ev0);
        if (ev1) (void)hipEventDestroy(ev1);
        return st;
    }
    A->bytes = sum_owned_bytes(A);
    A->last_stream = s;
    if (rep) {
        (void)hipEventRecord(ev1, s);
        (void)hipEventSynchronize(ev1);
        float ms = 0.f;
        (void)hipEventElapsedTime(&ms, ev0, ev1);
        rep->convert_ms = ms;
        rep->nnz_out = A->nnz;
        rep->bytes = A->bytes;
        rep->log2_beta = A->log2_beta;
        rep->parts = (int32_t)A->parts;
        rep->sort_split_keys = A->sort.split_keys;
        rep->sort_levels = A->sort.levels;
        rep->sort_first_fused = A->sort.first_fused;
        (void)hipEventDestroy(ev0);
        (void)hipEventDestroy(ev1);
    }
    *out = A;
    return SPX_OK;
}

// ------------------------------------------------------------------ product and handle

extern "C" spx_status spx_spmv_f32(spx_matrix A, const float* x, float* y, void* stream) {
    if (!A) return fail(SPX_ERR_INVALID_ARG, "matrix handle is NULL");
    if (A->value_type == SPX_F64)
        return fail(SPX_ERR_UNSUPPORTED, "FP64 matrix: use spx_spmv");
    if (A->m > 0 && !y) return fail(SPX_ERR_INVALID_ARG, "y is NULL");
    if (A->n > 0 && !x) return fail(SPX_ERR_INVALID_ARG, "x is NULL");
    if (ranges_overlap(x, (size_t)A->n * 4, y, (size_t)A->m * 4))
        return fail(SPX_ERR_ALIAS, "x and y overlap");
    if (A->m == 0) return SPX_OK;
    hipStream_t s = (hipStream_t)stream;
    A->last_stream = s;
    switch (A->fmt) {
        case SPX_CSR_MERGE:
        case SPX_CSR_ROWSPLIT: HIP_TRY(spmv_crs_f32(A, x, y, s)); break;
        case SPX_CSB_HILBERT:
        case SPX_CSB_ZMORTON: HIP_TRY(spmv_csbh_f32(A, x, y, s)); break;
        case SPX_BCOHC:
        case SPX_BCOHCH: HIP_TRY(spmv_bcoh_f32(A, x, y, s)); break;
        case SPX_CSB_RANKED: HIP_TRY(spmv_csbr_f32(A, x, y, s)); break;
        default: return fail(SPX_ERR_INVALID_ARG, "corrupt handle");
    }
    return SPX_OK;
}

extern "C" spx_status spx_spmv(spx_matrix A, const double* x, double* y, void* stream) {
    if (!A) return fail(SPX_ERR_INVALID_ARG, "matrix handle is NULL");
    if (A->value_type != SPX_F64)
        return fail(SPX_ERR_UNSUPPORTED, "reduced-precision matrix: use spx_spmv_f32");
    if (A->m > 0 && !y) return fail(SPX_ERR_INVALID_ARG, "y is NULL");
    if (A->n > 0 && !x) return fail(SPX_ERR_INVALID_ARG, "x is NULL");
    if (ranges_overlap(x, (size_t)A->n * 8, y, (size_t)A->m * 8))
        return fail(SPX_ERR_ALIAS, "x and y overlap");
    if (A->m == 0) return SPX_OK;
    hipStream_t s = (hipStream_t)stream;
    A->last_stream = s;
    switch (A->fmt) {
        case SPX_CSR_MERGE: HIP_TRY(spmv_merge(A, x, y, s)); break;
        case SPX_CSR_ROWSPLIT: HIP_TRY(spmv_rowsplit(A, x, y, s)); break;
        case SPX_CSB_HILBERT:
        case SPX_CSB_ZMORTON: HIP_TRY(spmv_csbh(A, x, y, s)); break;
        case SPX_BCOHC:
        case SPX_BCOHCH: HIP_TRY(spmv_bcoh(A, x, y, s)); break;
        case SPX_CSB_RANKED: HIP_TRY(spmv_csbr(A, x, y, s)); break;
        default: return fail(SPX_ERR_INVALID_ARG, "corrupt handle");
    }
    return SPX_OK;
}

// Grows a handle-held scratch buffer to at least `need` bytes.  The previous buffer may still be
// read by the handle's last product, so that stream is drained before the buffer is released.
static spx_status grow_scratch(spx_matrix_s* A, void** p, size_t* have, size_t need,
                               hipStream_t s, const char* what) {
    if (need <= *have) return SPX_OK;
    if (*p) {
        HIP_TRY(hipStreamSynchronize(A->last_stream));
        spx_dev_free(*p, A->last_stream);
        *p = nullptr;
        *have = 0;
    }
    *p = spx_dev_alloc(need, s);
    if (!*p) return fail(SPX_ERR_NOMEM, "device allocation of %zu bytes for %s failed", need, what);
    *have = need;
    return SPX_OK;
}

// Argument checks shared by spx_spmm and spx_spmm_noalloc (reported before any device work).
spx_status spmm_check(spx_matrix A, int32_t k, const void* x, int64_t ldx, const void* y,
                      int64_t ldy, spx_layout layout) {
    if (!A) return fail(SPX_ERR_INVALID_ARG, "matrix handle is NULL");
    if (!spx_is_crs(A->fmt))
        return fail(SPX_ERR_UNSUPPORTED, "products with several right-hand sides are provided for "
                                         "the CRS formats");
    if (k < 1) return fail(SPX_ERR_INVALID_ARG, "k = %d, must be >= 1", k);
    if (layout != SPX_COL_MAJOR && layout != SPX_ROW_MAJOR)
        return fail(SPX_ERR_INVALID_ARG, "unknown layout %d", layout);
    const int64_t m = A->m, n = A->n;
    const int64_t es = A->value_type == SPX_F64 ? 8 : 4;
    // spans in elements: last element + 1
    int64_t xlen = 0, ylen = 0;
    const int64_t big = INT64_MAX / 16;
    if (layout == SPX_COL_MAJOR) {
        if (ldx < (n > 1 ? n : 1) || ldy < (m > 1 ? m : 1))
            return fail(SPX_ERR_INVALID_ARG, "column-major leading dimensions must be >= n (x) "
                                             "and >= m (y)");
        if (ldx > big / k || ldy > big / k) return fail(SPX_ERR_RANGE, "operand span too large");
        xlen = n > 0 ? ldx * (k - 1) + n : 0;
        ylen = m > 0 ? ldy * (k - 1) + m : 0;
    } else {
        if (ldx < k || ldy < k)
            return fail(SPX_ERR_INVALID_ARG, "row-major leading dimensions must be >= k");
        if ((n > 0 && ldx > big / n) || (m > 0 && ldy > big / m))
            return fail(SPX_ERR_RANGE, "operand span too large");
        xlen = n > 0 ? ldx * (n - 1) + k : 0;
        ylen = m > 0 ? ldy * (m - 1) + k : 0;
    }
    if (m > 0 && !y) return fail(SPX_ERR_INVALID_ARG, "Y is NULL");
    if (n > 0 && !x) return fail(SPX_ERR_INVALID_ARG, "X is NULL");
    if (ranges_overlap(x, (size_t)(xlen * es), y, (size_t)(ylen * es)))
        return fail(SPX_ERR_ALIAS, "X and Y overlap");
    return SPX_OK;
}

extern "C" spx_status spx_spmm(spx_matrix A, int32_t k, const void* x, int64_t ldx, void* y,
                               int64_t ldy, spx_layout layout, void* stream) {
    SPX_TRY(spmm_check(A, k, x, ldx, y, ldy, layout));
    const int64_t m = A->m, n = A->n;
    const int64_t es = A->value_type == SPX_F64 ? 8 : 4;
    if (m == 0) return SPX_OK;
    hipStream_t s = (hipStream_t)stream;

    SpmmPlan P;
    if (A->fmt == SPX_CSR_MERGE) {
        P.coords = A->mp_coords;
        P.tiles = A->mp_tiles;
    } else {
        if (!A->mm_coords) {
            const int64_t tiles = ((int64_t)m + A->nnz + MP_TILE - 1) / MP_TILE;
            void* p = spx_dev_alloc(((size_t)tiles + 1) * sizeof(int2), s);
            if (!p) return fail(SPX_ERR_NOMEM, "device allocation for merge coordinates failed");
            if (tiles > 0) {
                const hipError_t e = launch_merge_coords(A->row_ptr, A->m, A->nnz, (int2*)p,
                                                         (int32_t)tiles, s);
                if (e != hipSuccess) {
                    spx_dev_free(p, s);
                    return fail(SPX_ERR_HIP, "merge coordinates: %s", hipGetErrorString(e));
                }
            }
            A->mm_coords = (int2*)p;
            A->mm_tiles = (int32_t)tiles;
        }
        P.coords = A->mm_coords;
        P.tiles = A->mm_tiles;
    }
    const int64_t kc = spmm_chunk_cols(k);
    if (!A->mm_carry_row) {  // one per tile; the tiling of a handle never changes
        A->mm_carry_row = (int32_t*)spx_dev_alloc(((size_t)P.tiles + 1) * 4, s);
        if (!A->mm_carry_row) return fail(SPX_ERR_NOMEM, "device allocation for carry rows failed");
    }
    SPX_TRY(grow_scratch(A, &A->mm_carry, &A->mm_carry_bytes, ((size_t)P.tiles + 1) * kc * 8, s,
                         "SpMM carries"));
    if (layout == SPX_COL_MAJOR && n > 0)
        SPX_TRY(grow_scratch(A, &A->mm_z, &A->mm_z_bytes, (size_t)(n * kc * es), s,
                             "row-major X copy"));
    if (layout == SPX_COL_MAJOR)
        SPX_TRY(grow_scratch(A, &A->mm_w, &A->mm_w_bytes, (size_t)(m * kc * es), s,
                             "row-major Y scratch"));
    if (A->nhot > 0)
        SPX_TRY(grow_scratch(A, &A->mm_h, &A->mm_h_bytes, (size_t)(A->nhot * kc * es), s,
                             "hot X rows"));
    P.carry_row = A->mm_carry_row;
    P.carry_val = (double*)A->mm_carry;
    P.z = A->mm_z;
    P.h = A->mm_h;
    P.w = A->mm_w;
    A->last_stream = s;
    HIP_TRY(spmm_crs(A, P, k, x, ldx, y, ldy, layout == SPX_ROW_MAJOR, s));
    return SPX_OK;
}

extern "C" spx_status spx_matrix_get_info(spx_matrix A, spx_matrix_info* info) {
    if (!A || !info) return fail(SPX_ERR_INVALID_ARG, "NULL argument");
    info->m = A->m;
    info->n = A->n;
    info->nnz = A->nnz;
    info->format = A->fmt;
    info->log2_beta = A->log2_beta;
    info->bytes = A->bytes;
    info->parts = A->parts;
    info->value_type = A->value_type;
    return SPX_OK;
}

extern "C" spx_status spx_matrix_export(spx_matrix A, spx_array which, void* dst, int64_t bytes,
                                        int64_t* needed, void* stream) {
    if (!A) return fail(SPX_ERR_INVALID_ARG, "matrix handle is NULL");
    const void* src = nullptr;
    int64_t len = 0;
    bool exists = false;
    const bool bcoh = spx_is_bcoh(A->fmt);
    const bool crs = spx_is_crs(A->fmt);
    switch (which) {
        case SPX_ARRAY_ROW_PTR:
            exists = crs;
            src = A->row_ptr;
            len = ((int64_t)A->m + 1) * 4;
            break;
        case SPX_ARRAY_COL_IND:
            exists = crs;
            src = A->col;
            len = A->nnz * 4;
            break;
        case SPX_ARRAY_VALUES:
            exists = true;
            src = A->value_type == SPX_F64 ? (const void*)A->val : (const void*)A->val_lp;
            len = A->nnz * (A->value_type == SPX_F64 ? 8 : A->value_type == SPX_F32 ? 4 : 2);
            break;
        case SPX_ARRAY_BLK_PTR:
            exists = !crs;
            src = bcoh ? A->bh_blk_ptr : A->blk_ptr;
            len = bcoh ? (A->bh_nblocks + 1) * 4 : (A->nbr * A->nbc + 1) * 4;
            break;
        case SPX_ARRAY_COL_ORDER:
            exists = A->fmt == SPX_CSB_RANKED;
            src = A->cr_order;
            len = (int64_t)A->cr_nranked * 4;
            break;
        case SPX_ARRAY_ROW_ORDER:
            exists = A->fmt == SPX_CSB_RANKED;
            src = A->cr_row_order;
            len = (int64_t)A->cr_nrows * 4;
            break;
        case SPX_ARRAY_BLK_COORD:
            exists = bcoh;
            src = A->bh_blk_coord;
            len = A->bh_nblocks * 4;
            break;
        case SPX_ARRAY_PACKED:
            exists = !crs;
            src = A->packed;
            len = A->nnz * 4;
            break;
        case SPX_ARRAY_PARTS:
            exists = true;
            if (A->fmt == SPX_CSR_MERGE) {
                src = A->mp_coords;
                len = ((int64_t)A->mp_tiles + 1) * 8;
            } else if (A->fmt == SPX_CSR_ROWSPLIT) {
                src = A->rs_blocks;
                len = A->rs_blocks ? ((int64_t)A->rs_nb + 1) * 4 : 0;
            } else if (bcoh) {
                src = A->bh_part_row;
                len = 8 * ((int64_t)A->bh_nparts + 1);
            } else {
                src = A->cb_units;
                len = (int64_t)A->cb_nunits * 16;
            }
            break;
        default: return fail(SPX_ERR_INVALID_ARG, "unknown array %d", (int)which);
    }
    if (!exists)
        return fail(SPX_ERR_INVALID_ARG, "array %d does not exist for format %d", (int)which,
                    (int)A->fmt);
    if (src == nullptr) len = 0;
    if (needed) *needed = len;
    if (bytes < len)
        return fail(SPX_ERR_INVALID_ARG, "destination holds %lld of %lld bytes",
                    (long long)bytes, (long long)len);
    if (len == 0) return SPX_OK;
    if (!dst) return fail(SPX_ERR_INVALID_ARG, "dst is NULL");
    if (which == SPX_ARRAY_COL_IND && A->nhot > 0) {  // hot entries back to their columns
        HIP_TRY(launch_hot_unmap(A->col, A->nnz, A->hot_cols, (int32_t*)dst, (hipStream_t)stream));
        return SPX_OK;
    }
    HIP_TRY(hipMemcpyAsync(dst, src, (size_t)len, hipMemcpyDeviceToDevice, (hipStream_t)stream));
    return SPX_OK;
}

extern "C" spx_status spx_matrix_destroy(spx_matrix A) {
    if (!A) return SPX_OK;
    (void)hipStreamSynchronize(A->last_stream);
    for (void* p : A->owned) spx_dev_free(p, A->last_stream);
    for (void* p : {(void*)A->mm_coords, (void*)A->mm_carry_row, A->mm_carry, A->mm_z, A->mm_h,
                    A->mm_w})
        spx_dev_free(p, A->last_stream);
    delete A;
    return SPX_OK;
}

// ------------------------------------------------------------------ memory probe

extern "C" int64_t spx_probe_out_len(void) { return probe_out_len(); }

extern "C" spx_status spx_probe_gather(const double* x, int64_t window, int64_t n, double* out,
                                       void* stream) {
    if (!x || !out) return fail(SPX_ERR_INVALID_ARG, "NULL pointer");
    if (window < 1 || (window & (window - 1)) != 0)
        return fail(SPX_ERR_INVALID_ARG, "window %lld is not a power of two", (long long)window);
    if (n < 0) return fail(SPX_ERR_INVALID_ARG, "n < 0");
    HIP_TRY(launch_probe_gather(x, window, n, out, (hipStream_t)stream));
    return SPX_OK;
}
