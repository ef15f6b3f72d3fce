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
    uint32_t* done = nullptr;
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
    uint32_t* done = B->dev.get<uint32_t>(count);
    const float** xs = (const float**)B->dev.get<void*>(count);
    float** ys = (float**)B->dev.get<void*>(count);
    if (!one || !done || !xs || !ys)
        return bail(spx_fail(SPX_ERR_NOMEM, "device allocation failed"));
    e = launch_fill_u32(done, count, 0u, s);
    if (e != hipSuccess) return bail(herr(e, "counters"));
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
                hit.resize(M.tiles);
                for (int32_t t = 0; t < M.tiles; ++t) hit[t] = make_int2(0, t);
                e = hipMemcpyAsync(it, hit.data(), M.tiles * sizeof(int2), hipMemcpyHostToDevice, s);
                if (e == hipSuccess)
                    e = hipMemcpyAsync(one, &M, sizeof(BatchMat), hipMemcpyHostToDevice, s);
                const int32_t grid = (int32_t)std::min<int64_t>(M.tiles, 1024);
                for (int r = 0; r < kTuneWarm && e == hipSuccess; ++r)
                    e = launch_batch_spmv(one, it, M.tiles, grid, xst, yst, done, s);
                if (e == hipSuccess) e = hipEventRecord(e0, s);
                for (int r = 0; r < kTuneReps && e == hipSuccess; ++r)
                    e = launch_batch_spmv(one, it, M.tiles, grid, xst, yst, done, s);
                if (e == hipSuccess) e = hipEventRecord(e1, s);
                if (e == hipSuccess) e = hipEventSynchronize(e1);
                float ms = 0;
                if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
                if (e != hipSuccess) break;
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

    // final plans and the item list (matrices in order, tiles in order)
    std::vector<int2> items;
    for (int32_t i = 0; i < count; ++i) {
        e = apply_plan(B->host[i], plan[i], mats[i]->nnz, s);
        if (e != hipSuccess) return bail(herr(e, "plans"));
        for (int32_t t = 0; t < B->host[i].tiles; ++t) items.push_back(make_int2(i, t));
        if (chosen) chosen[i] = plan[i];
    }
    B->nitems = (int64_t)items.size();
    if (B->nitems >= INT32_MAX) return bail(spx_fail(SPX_ERR_RANGE, "too many work items"));
    B->items = B->dev.get<int2>(items.size());
    B->mats = B->dev.get<BatchMat>(count);
    if (!B->items || !B->mats) return bail(spx_fail(SPX_ERR_NOMEM, "device allocation failed"));
    e = hipMemcpyAsync(B->items, items.data(), items.size() * sizeof(int2),
                       hipMemcpyHostToDevice, s);
    if (e == hipSuccess)
        e = hipMemcpyAsync(B->mats, B->host.data(), count * sizeof(BatchMat),
                           hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return bail(herr(e, "tables"));
    B->grid = (int32_t)std::min<int64_t>(B->nitems, 1024);
    B->done = done;
    B->xs = xs;
    B->ys = ys;
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
    const hipError_t e = launch_batch_spmv(B->mats, B->items, (int32_t)B->nitems, B->grid, B->xs,
                                           B->ys, B->done, (hipStream_t)stream);
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
