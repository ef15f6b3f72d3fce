// spx_batch.cpp -- batches of matrices multiplied by one persistent launch, and the per-matrix
// plan autotuner.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <new>
#include <unordered_set>
#include <utility>
#include <vector>

#include "../../include/spx_batch.h"
#include "spx_internal.h"

namespace {

constexpr int kRowPlanMaxRow = 1024;  // row tiles only when no row is longer (FP32 sums)
constexpr int kCandidates[] = {SPX_PLAN_MERGE_4, SPX_PLAN_MERGE_8, SPX_PLAN_MERGE_16,
                               SPX_PLAN_ROWS_512, SPX_PLAN_ROWS_2048};
constexpr int kTuneWarm = 2, kTuneReps = 8;
// A candidate is timed on at least this many work items (the matrix's tiles repeated), so that
// it is measured at full occupancy, the condition it will run under inside a batch.
constexpr int64_t kTuneItems = 8192;

bool is_merge(int plan) { return plan >= SPX_PLAN_MERGE_4 && plan <= SPX_PLAN_MERGE_16; }
int plan_ipt(int plan) {
    return plan == SPX_PLAN_MERGE_4 ? 4 : plan == SPX_PLAN_MERGE_8 ? 8 : 16;
}

struct Dev {  // device allocations of one batch, freed together
    std::vector<void*> ptrs;
    hipStream_t s = nullptr;
    template <typename T>
    T* get(size_t count) {
        if (count == 0) count = 1;
        void* p = spx_dev_alloc(count * sizeof(T), s);
        if (p) ptrs.push_back(p);
        return (T*)p;
    }
    void release() {
        for (void* p : ptrs) spx_dev_free(p, s);
        ptrs.clear();
    }
};

}  // namespace

struct spx_batch_s {
    int32_t count = 0;
    std::vector<BatchMat> host;  // per matrix
    std::vector<spx_matrix> handles;
    BatchMat* mats = nullptr;
    int2* items = nullptr;
    int64_t nitems = 0;
    int32_t grid = 0;
    int32_t max_tile = 256;
    const float** xs = nullptr;  // device tables
    float** ys = nullptr;
    bool bound = false;
    Dev dev;
};

static spx_status herr(hipError_t e, const char* what) {
    char buf[256];
    snprintf(buf, sizeof buf, "%s: %s", what, hipGetErrorString(e));
    return spx_fail(SPX_ERR_HIP, buf);
}

// Fills the plan fields of M (coords and carries must already be sized for the plan).
static hipError_t apply_plan(BatchMat& M, int plan, int64_t nnz, hipStream_t s) {
    M.plan = plan;
    if (is_merge(plan)) {
        const int64_t tile = 256LL * plan_ipt(plan);
        M.tiles = (int32_t)(((int64_t)M.m + nnz + tile - 1) / tile);
        M.rows_per_tile = 0;
        if (M.tiles > 0)
            return launch_merge_coords(M.row_ptr, M.m, nnz, (int2*)M.coords, M.tiles, s,
                                       (int32_t)tile);
        return hipSuccess;
    }
    const int64_t target = plan == SPX_PLAN_ROWS_512 ? 512 : 2048;
    const int64_t avg = M.m > 0 ? std::max<int64_t>(1, (nnz + M.m - 1) / M.m) : 1;
    M.rows_per_tile = (int32_t)std::max<int64_t>(1, std::min<int64_t>(target / avg, 4096));
    M.tiles = (int32_t)((M.m + M.rows_per_tile - 1) / M.rows_per_tile);
    return hipSuccess;
}

// Upper bound of the work items of a batch under any plans.
static int64_t items_bound(const spx_matrix* mats, int32_t count) {
    int64_t b = 0;
    for (int32_t i = 0; i < count; ++i)
        b += std::max<int64_t>(mats[i]->m, ((int64_t)mats[i]->m + mats[i]->nnz) / 1024 + 2);
    return std::max<int64_t>(b, 1);
}

// Applies `plan`, rebuilds the item list (matrices in order, tiles in order) and the device
// tables, sets max_tile and a default grid (one workgroup per item).
static hipError_t build_tables(spx_batch_s* B, const std::vector<int32_t>& plan, hipStream_t s) {
    std::vector<int2> items;
    B->max_tile = 256;
    for (int32_t i = 0; i < B->count; ++i) {
        const hipError_t e = apply_plan(B->host[i], plan[i], B->handles[i]->nnz, s);
        if (e != hipSuccess) return e;
        for (int32_t t = 0; t < B->host[i].tiles; ++t) items.push_back(make_int2(i, t));
        if (is_merge(plan[i])) B->max_tile = std::max(B->max_tile, 256 * plan_ipt(plan[i]));
    }
    B->nitems = (int64_t)items.size();
    B->grid = (int32_t)std::min<int64_t>(std::max<int64_t>(B->nitems, 1), 1 << 20);
    hipError_t e = hipSuccess;
    if (!items.empty())
        e = hipMemcpyAsync(B->items, items.data(), items.size() * sizeof(int2),
                           hipMemcpyHostToDevice, s);
    if (e == hipSuccess)
        e = hipMemcpyAsync(B->mats, B->host.data(), B->count * sizeof(BatchMat),
                           hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    return e;
}

// Times the whole batch (zero x shared by all matrices, a scratch y per matrix) for the plans as
// tuned, with 16-item merge tiles replaced by 8-item ones, and with every single plan for all
// matrices (row tiles only where the rows allow, merge tiles of 8 items elsewhere), each with
// one workgroup per item and with persistent grids of 4096 and 1024 workgroups; keeps the
// fastest, so the result is never slower (to the timing's precision) than one plan for all.
static hipError_t tune_batch(spx_batch_s* B, const std::vector<int32_t>& plan,
                             const std::vector<uint32_t>& maxlen, int64_t max_n, hipStream_t s) {
    Dev tmp;
    tmp.s = s;
    int64_t total_m = 0;
    for (const BatchMat& M : B->host) total_m += M.m;
    float* xt = tmp.get<float>(max_n);
    float* yt = tmp.get<float>(total_m);
    if (!xt || !yt) {
        tmp.release();
        return hipErrorOutOfMemory;
    }
    std::vector<const float*> hx(B->count, xt);
    std::vector<float*> hy(B->count);
    int64_t off = 0;
    for (int32_t i = 0; i < B->count; ++i) {
        hy[i] = yt + off;
        off += B->host[i].m;
    }
    hipEvent_t e0 = nullptr, e1 = nullptr;
    hipError_t e = hipMemsetAsync(xt, 0, max_n * 4, s);
    if (e == hipSuccess)
        e = hipMemcpyAsync(B->xs, hx.data(), B->count * sizeof(void*), hipMemcpyHostToDevice, s);
    if (e == hipSuccess)
        e = hipMemcpyAsync(B->ys, hy.data(), B->count * sizeof(void*), hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    std::vector<std::vector<int32_t>> variants{plan};
    if (std::count(plan.begin(), plan.end(), SPX_PLAN_MERGE_16) > 0) {
        std::vector<int32_t> v = plan;
        for (int32_t& p : v)
            if (p == SPX_PLAN_MERGE_16) p = SPX_PLAN_MERGE_8;
        variants.push_back(v);
    }
    for (int cand : kCandidates) {
        std::vector<int32_t> v(plan.size());
        for (size_t i = 0; i < v.size(); ++i)
            v[i] = (cand >= SPX_PLAN_ROWS_512 && maxlen[i] > (uint32_t)kRowPlanMaxRow)
                       ? SPX_PLAN_MERGE_8
                       : cand;
        if (std::find(variants.begin(), variants.end(), v) == variants.end()) variants.push_back(v);
    }
    float best = 0;
    size_t best_v = 0;
    int32_t best_g = B->grid;
    for (size_t vi = 0; vi < variants.size() && e == hipSuccess; ++vi) {
        e = build_tables(B, variants[vi], s);
        const int64_t all = B->grid;
        for (int64_t g : {all, (int64_t)4096, (int64_t)1024}) {
            if (e != hipSuccess) break;
            if (g != all && g >= all) continue;  // a persistent grid only when it is smaller
            for (int r = 0; r < kTuneWarm && e == hipSuccess; ++r)
                e = launch_batch_spmv(B->mats, B->items, (int32_t)B->nitems, (int32_t)g,
                                      B->max_tile, B->xs, B->ys, s);
            if (e == hipSuccess) e = hipEventRecord(e0, s);
            for (int r = 0; r < 3 && e == hipSuccess; ++r)
                e = launch_batch_spmv(B->mats, B->items, (int32_t)B->nitems, (int32_t)g,
                                      B->max_tile, B->xs, B->ys, s);
            if (e == hipSuccess) e = hipEventRecord(e1, s);
            if (e == hipSuccess) e = hipEventSynchronize(e1);
            float ms = 0;
            if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
            if (e == hipSuccess && (best == 0 || ms < best)) {
                best = ms;
                best_v = vi;
                best_g = (int32_t)g;
            }
        }
    }
    if (e == hipSuccess) {
        e = build_tables(B, variants[best_v], s);
        B->grid = best_g;
    }
    if (e0) (void)hipEventDestroy(e0);
    if (e1) (void)hipEventDestroy(e1);
    (void)hipStreamSynchronize(s);
    tmp.release();
    return e;
}

extern "C" spx_status spx_batch_create(const spx_matrix* mats, int32_t count,
                                       const int32_t* plans, void* stream, spx_batch* out,
                                       int32_t* chosen) {
    if (!out) return spx_fail(SPX_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    if (!mats || count < 1) return spx_fail(SPX_ERR_INVALID_ARG, "no matrices");
    std::unordered_set<const void*> seen;
    for (int32_t i = 0; i < count; ++i) {
        const spx_matrix A = mats[i];
        if (!A) return spx_fail(SPX_ERR_INVALID_ARG, "NULL handle");
        if (!seen.insert(A).second) return spx_fail(SPX_ERR_INVALID_ARG, "repeated handle");
        if (A->fmt != SPX_CSR_ROWSPLIT && A->fmt != SPX_CSR_MERGE)
            return spx_fail(SPX_ERR_UNSUPPORTED, "batches hold CRS matrices");
        if (A->value_type != SPX_F32 && A->value_type != SPX_BF16)
            return spx_fail(SPX_ERR_UNSUPPORTED, "batches hold FP32 or bfloat16 matrices");
        if (plans && (plans[i] < SPX_PLAN_AUTO || plans[i] > SPX_PLAN_ROWS_2048))
            return spx_fail(SPX_ERR_INVALID_ARG, "unknown plan");
    }
    hipStream_t s = (hipStream_t)stream;
    spx_batch_s* B = new (std::nothrow) spx_batch_s;
    if (!B) return spx_fail(SPX_ERR_NOMEM, "host allocation failed");
    B->count = count;
    B->dev.s = s;
    auto bail = [&](spx_status st) {
        (void)hipStreamSynchronize(s);
        B->dev.release();
        delete B;
        return st;
    };

    // longest row of every matrix
    uint32_t* maxlen_d = B->dev.get<uint32_t>(count);
    if (!maxlen_d) return bail(spx_fail(SPX_ERR_NOMEM, "device allocation failed"));
    hipError_t e = launch_fill_u32(maxlen_d, count, 0u, s);
    for (int32_t i = 0; i < count && e == hipSuccess; ++i)
        e = launch_batch_maxlen(mats[i]->row_ptr, mats[i]->m, maxlen_d + i, s);
    std::vector<uint32_t> maxlen(count);
    if (e == hipSuccess)
        e = hipMemcpyAsync(maxlen.data(), maxlen_d, count * 4, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return bail(herr(e, "row lengths"));

    // per matrix: static fields, coords / carries sized for the finest merge tiles
    B->host.resize(count);
    B->handles.assign(mats, mats + count);
    int64_t max_m = 1, max_n = 1;
    for (int32_t i = 0; i < count; ++i) {
        const spx_matrix A = mats[i];
        BatchMat& M = B->host[i];
        M = BatchMat{};
        M.row_ptr = A->row_ptr;
        M.col = A->col;
        M.val = A->val_lp;
        M.hot_cols = A->hot_cols;
        M.m = A->m;
        M.n = A->n;
        M.bf16 = A->value_type == SPX_BF16;
        const int64_t tiles_max = ((int64_t)A->m + A->nnz) / 1024 + 2;
        M.coords = B->dev.get<int2>(tiles_max + 1);
        M.carry_row = B->dev.get<int32_t>(tiles_max);
        M.carry_val = B->dev.get<double>(tiles_max);
        if (!M.coords || !M.carry_row || !M.carry_val)
            return bail(spx_fail(SPX_ERR_NOMEM, "device allocation failed"));
        if (plans && plans[i] >= SPX_PLAN_ROWS_512 && maxlen[i] > (uint32_t)kRowPlanMaxRow)
            return bail(spx_fail(SPX_ERR_INVALID_ARG, "row-tile plan for a matrix with a row "
                                                      "longer than 1024 entries"));
        max_m = std::max<int64_t>(max_m, A->m);
        max_n = std::max<int64_t>(max_n, A->n);
    }

    // autotune: time each candidate plan on the matrix alone
    std::vector<int32_t> plan(count);
    bool tune = false;
    for (int32_t i = 0; i < count; ++i) {
        plan[i] = plans ? plans[i] : SPX_PLAN_AUTO;
        tune = tune || plan[i] == SPX_PLAN_AUTO;
    }
    BatchMat* one = B->dev.get<BatchMat>(1);
    const float** xs = (const float**)B->dev.get<void*>(count);
    float** ys = (float**)B->dev.get<void*>(count);
    if (!one || !xs || !ys) return bail(spx_fail(SPX_ERR_NOMEM, "device allocation failed"));
    if (tune) {
        Dev tmp;
        tmp.s = s;
        float* xt = tmp.get<float>(max_n);
        float* yt = tmp.get<float>(max_m);
        // work items of one matrix under any candidate: merge tiles of 1024 items or row tiles
        int64_t it_cap = 1;
        for (int32_t i = 0; i < count; ++i)
            it_cap = std::max<int64_t>(it_cap, std::max<int64_t>(mats[i]->m,
                                                                 ((int64_t)mats[i]->m + mats[i]->nnz) / 1024 + 2));
        it_cap += kTuneItems;
        int2* it = tmp.get<int2>(it_cap);
        const float** xst = (const float**)tmp.get<void*>(1);
        float** yst = (float**)tmp.get<void*>(1);
        hipEvent_t e0 = nullptr, e1 = nullptr;
        if (!xt || !yt || !it || !xst || !yst) {
            tmp.release();
            return bail(spx_fail(SPX_ERR_NOMEM, "device allocation failed"));
        }
        e = hipMemsetAsync(xt, 0, max_n * 4, s);
        if (e == hipSuccess) e = hipMemcpyAsync(xst, &xt, sizeof(void*), hipMemcpyHostToDevice, s);
        if (e == hipSuccess) e = hipMemcpyAsync(yst, &yt, sizeof(void*), hipMemcpyHostToDevice, s);
        if (e == hipSuccess) e = hipEventCreate(&e0);
        if (e == hipSuccess) e = hipEventCreate(&e1);
        std::vector<int2> hit;
        for (int32_t i = 0; i < count && e == hipSuccess; ++i) {
            if (plan[i] != SPX_PLAN_AUTO) continue;
            const spx_matrix A = mats[i];
            float best_ms = 0;
            int best = SPX_PLAN_MERGE_8;
            for (int cand : kCandidates) {
                if (cand >= SPX_PLAN_ROWS_512 && maxlen[i] > (uint32_t)kRowPlanMaxRow) continue;
                BatchMat M = B->host[i];
                e = apply_plan(M, cand, A->nnz, s);
                if (e != hipSuccess) break;
                if (M.tiles == 0) {
                    best = cand;
                    break;
                }
                // the tiles repeated up to kTuneItems items; repeats rewrite the same outputs of
                // the scratch y, whose values are not used
                const int64_t reps = (kTuneItems + M.tiles - 1) / M.tiles;
                const int32_t nit = (int32_t)(reps * M.tiles);
                hit.resize(nit);
                for (int32_t q = 0; q < nit; ++q) hit[q] = make_int2(0, q % M.tiles);
                e = hipMemcpyAsync(it, hit.data(), nit * sizeof(int2), hipMemcpyHostToDevice, s);
                if (e == hipSuccess)
                    e = hipMemcpyAsync(one, &M, sizeof(BatchMat), hipMemcpyHostToDevice, s);
                const int32_t mt = is_merge(cand) ? 256 * plan_ipt(cand) : 256;
                for (int r = 0; r < kTuneWarm && e == hipSuccess; ++r)
                    e = launch_batch_spmv(one, it, nit, nit, mt, xst, yst, s);
                if (e == hipSuccess) e = hipEventRecord(e0, s);
                for (int r = 0; r < kTuneReps && e == hipSuccess; ++r)
                    e = launch_batch_spmv(one, it, nit, nit, mt, xst, yst, s);
                if (e == hipSuccess) e = hipEventRecord(e1, s);
                if (e == hipSuccess) e = hipEventSynchronize(e1);
                float ms = 0;
                if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
                if (e != hipSuccess) break;
                ms /= (float)reps;  // cost of one pass over the matrix
                if (best_ms == 0 || ms < best_ms) {
                    best_ms = ms;
                    best = cand;
                }
            }
            plan[i] = best;
        }
        if (e0) (void)hipEventDestroy(e0);
        if (e1) (void)hipEventDestroy(e1);
        (void)hipStreamSynchronize(s);
        tmp.release();
        if (e != hipSuccess) return bail(herr(e, "autotuning"));
    }

    // final plans and the item list
    B->xs = xs;
    B->ys = ys;
    B->items = B->dev.get<int2>(items_bound(mats, count));
    B->mats = B->dev.get<BatchMat>(count);
    if (!B->items || !B->mats) return bail(spx_fail(SPX_ERR_NOMEM, "device allocation failed"));
    e = build_tables(B, plan, s);
    if (e == hipSuccess && B->nitems >= INT32_MAX)
        return bail(spx_fail(SPX_ERR_RANGE, "too many work items"));
    if (e == hipSuccess && tune && B->nitems > 1024) {
        // whole-batch choices: the launch shape, and whether merge tiles of 16 items per thread
        // (which set the launch's LDS size for every workgroup) beat 8 items per thread
        e = tune_batch(B, plan, maxlen, max_n, s);
    }
    if (e != hipSuccess) return bail(herr(e, "plans"));
    if (chosen)
        for (int32_t i = 0; i < count; ++i) chosen[i] = B->host[i].plan;
    *out = B;
    return SPX_OK;
}

extern "C" spx_status spx_batch_bind(spx_batch B, const float* const* xs, float* const* ys,
                                     void* stream) {
    if (!B || !xs || !ys) return spx_fail(SPX_ERR_INVALID_ARG, "NULL argument");
    // intervals of every vector; a y may not overlap anything else
    struct Iv {
        uintptr_t a, b;
        bool out;
    };
    std::vector<Iv> iv;
    for (int32_t i = 0; i < B->count; ++i) {
        const BatchMat& M = B->host[i];
        if ((M.n > 0 && !xs[i]) || (M.m > 0 && !ys[i]))
            return spx_fail(SPX_ERR_INVALID_ARG, "NULL vector");
        if (M.n > 0) iv.push_back({(uintptr_t)xs[i], (uintptr_t)xs[i] + (uintptr_t)M.n * 4, false});
        if (M.m > 0) iv.push_back({(uintptr_t)ys[i], (uintptr_t)ys[i] + (uintptr_t)M.m * 4, true});
    }
    std::sort(iv.begin(), iv.end(), [](const Iv& p, const Iv& q) { return p.a < q.a; });
    uintptr_t end_any = 0, end_out = 0;
    for (const Iv& v : iv) {
        if (v.out && v.a < end_any) return spx_fail(SPX_ERR_ALIAS, "an output overlaps a vector");
        if (!v.out && v.a < end_out) return spx_fail(SPX_ERR_ALIAS, "an input overlaps an output");
        end_any = std::max(end_any, v.b);
        if (v.out) end_out = std::max(end_out, v.b);
    }
    hipStream_t s = (hipStream_t)stream;
    hipError_t e = hipMemcpyAsync(B->xs, xs, B->count * sizeof(void*), hipMemcpyHostToDevice, s);
    if (e == hipSuccess)
        e = hipMemcpyAsync(B->ys, ys, B->count * sizeof(void*), hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return herr(e, "bind");
    B->bound = true;
    return SPX_OK;
}

extern "C" spx_status spx_batch_spmv(spx_batch B, void* stream) {
    if (!B) return spx_fail(SPX_ERR_INVALID_ARG, "batch is NULL");
    if (!B->bound) return spx_fail(SPX_ERR_INVALID_ARG, "no vectors bound");
    const hipError_t e = launch_batch_spmv(B->mats, B->items, (int32_t)B->nitems, B->grid,
                                           B->max_tile, B->xs, B->ys, (hipStream_t)stream);
    if (e != hipSuccess) return herr(e, "batch product");
    return SPX_OK;
}

extern "C" spx_status spx_batch_get_info(spx_batch B, int64_t* items, int32_t* workgroups) {
    if (!B) return spx_fail(SPX_ERR_INVALID_ARG, "batch is NULL");
    if (items) *items = B->nitems;
    if (workgroups) *workgroups = B->grid;
    return SPX_OK;
}

extern "C" spx_status spx_batch_destroy(spx_batch B) {
    if (!B) return SPX_OK;
    (void)hipDeviceSynchronize();
    B->dev.release();
    delete B;
    return SPX_OK;
}
