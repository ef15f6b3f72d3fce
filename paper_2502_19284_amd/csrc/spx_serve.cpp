// spx_serve.cpp -- serving loop: resident matrices, request queues, continuous batching.
//
// One scheduler thread per server does all device work after admission.  Requests are queued per
// matrix under one mutex; the scheduler polls its in-flight batches (one HIP event per slot),
// retires the finished ones, and fills free slots with the matrix whose oldest waiting request is
// oldest, coalescing up to max_batch of its waiting requests into one product.  Product scratch
// (carries, hot rows, staging of X and Y) belongs to the slot, not to the matrix, so a popular
// matrix can have batches on several slots at once.  Admission and conversion run on the
// caller's thread; the scheduler only allocates to grow its slot buffers.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <mutex>
#include <new>
#include <thread>
#include <unordered_map>
#include <vector>

#include "../../include/spx_serve.h"
#include "spx_internal.h"

namespace {

using clock_type = std::chrono::steady_clock;

struct Req {
    spx_request r{};
    hipEvent_t ready = nullptr;  // recorded on r.stream at submission (null: x complete)
    uint64_t ticket = 0;
    double t_submit = 0, t_done = 0;
    bool done = false;
    spx_status status = SPX_OK;
};

struct Mat {
    spx_matrix A = nullptr;
    int32_t id = 0, m = 0, n = 0;
    int64_t bytes = 0;
    std::deque<Req*> waiting;
    int32_t in_flight = 0;  // batches of this matrix on the device
    int64_t outstanding = 0;
    const int2* coords = nullptr;  // merge tiles of the product (the handle's)
    int32_t tiles = 0, nhot = 0;
};

struct Slot {
    hipStream_t stream = nullptr;
    hipEvent_t done = nullptr;
    bool busy = false;
    Mat* mat = nullptr;
    std::vector<Req*> batch;
    float* X = nullptr;  // n x k, row-major
    float* Y = nullptr;  // m x k, row-major
    size_t xcap = 0, ycap = 0;
    // product scratch owned by the slot, so that one matrix may have batches on several slots
    int32_t* crow = nullptr;  // tile carry rows
    double* cval = nullptr;   // tile carries, tiles x k
    float* H = nullptr;       // hot rows of X, nhot x k
    size_t crow_cap = 0, cval_cap = 0, hcap = 0;
    void* dtab = nullptr;  // device: k x pointers, k y pointers, k alphas, k betas
    void* htab = nullptr;  // pinned host mirror
};

constexpr int kMaxBatch = 64;
constexpr size_t kTabBytes = kMaxBatch * (2 * sizeof(void*) + 2 * sizeof(float));

}  // namespace

struct spx_server_s {
    spx_server_opts o{};
    int device = 0;
    std::mutex mu;
    std::condition_variable cv_sched, cv_done;
    std::unordered_map<int32_t, Mat*> mats;
    std::unordered_map<uint64_t, Req*> reqs;
    int32_t next_id = 1;
    uint64_t next_ticket = 1;
    std::vector<Slot> slots;
    std::thread th;
    bool stop = false;
    int64_t used = 0, staging = 0;
    int64_t stage_max = 0;               // largest per-slot staging bound of an admitted matrix
    std::vector<hipEvent_t> ev_pool;     // recycled request events
    int64_t n_done = 0, n_batches = 0, widest = 0;
    int32_t in_flight = 0;
    int64_t waiting_total = 0;
    clock_type::time_point epoch = clock_type::now();

    double now_us() const {
        return std::chrono::duration<double, std::micro>(clock_type::now() - epoch).count();
    }
    void run();
    void retire(Slot& sl, double t, spx_status st);
    spx_status launch(Slot& sl);
};

static spx_status hip_fail(hipError_t e, const char* what) {
    char buf[256];
    snprintf(buf, sizeof buf, "%s: %s", what, hipGetErrorString(e));
    return spx_fail(SPX_ERR_HIP, buf);
}

extern "C" spx_status spx_server_opts_default(spx_server_opts* o) {
    if (!o) return spx_fail(SPX_ERR_INVALID_ARG, "opts is NULL");
    o->memory_budget = (int64_t)64 << 30;
    o->slots = 4;
    o->max_batch = 32;
    o->coalesce = 1;
    o->poll_us = 0;
    return SPX_OK;
}

// Upper bound of what a resident matrix holds: stored arrays for nnz <= E entries, both
// partitions' tables, the hot-column tables, and the product scratch of max_batch columns that
// its batches occupy in the slots.
static int64_t footprint_bound(const spx_coo_desc* c, int32_t vt, int32_t max_batch) {
    const int64_t m = c->m, n = c->n, E = c->nnz;
    const int64_t vs = vt == SPX_F32 ? 4 : 2;
    const int64_t tiles = (m + E) / MP_TILE + 2;
    const int64_t hot = std::min<int64_t>(n, HOT_AUTO_MAX);
    int64_t b = 4 * (m + 1) + (4 + vs) * E;              // row_ptr, col_ind, values
    b += 20 * tiles;                                     // merge tile starts and carries
    b += 4 * (m + 2) + 16 * (E / RS_LONG + 2) + 8 * (E / RS_CHUNK + 2);  // row-split tables
    b += 20 * hot + 4 * hot * max_batch;                 // hot set, hot x copy, hot X rows
    b += (12 + 8 * (int64_t)max_batch) * tiles;          // product tiles, carry rows and values
    return b;
}

// Upper bound of one slot's staging for a batch of max_batch requests on a matrix: the x and y
// columns (row-major X and Y), the hot rows of X and the tile carries (rows and values).
static int64_t staging_bound(const spx_coo_desc* c, int32_t max_batch) {
    const int64_t m = c->m, n = c->n, E = c->nnz;
    const int64_t tiles = (m + E) / MP_TILE + 2;
    const int64_t hot = std::min<int64_t>(n, HOT_AUTO_MAX);
    return 4 * (m + n) * max_batch + 4 * hot * max_batch + (4 + 8 * (int64_t)max_batch) * tiles;
}

extern "C" spx_status spx_server_create(const spx_server_opts* opts, spx_server* out) {
    if (!out) return spx_fail(SPX_ERR_INVALID_ARG, "out is NULL");
    *out = nullptr;
    spx_server_opts o;
    spx_server_opts_default(&o);
    if (opts) o = *opts;
    if (o.memory_budget <= 0) return spx_fail(SPX_ERR_INVALID_ARG, "memory_budget must be > 0");
    if (o.slots < 1 || o.slots > 16) return spx_fail(SPX_ERR_INVALID_ARG, "slots must be 1..16");
    if (o.max_batch < 1 || o.max_batch > kMaxBatch)
        return spx_fail(SPX_ERR_INVALID_ARG, "max_batch must be 1..64");
    if (o.poll_us < 0 || o.poll_us > 1000)
        return spx_fail(SPX_ERR_INVALID_ARG, "poll_us must be 0..1000");
    if (!o.coalesce) {  // the plain path: one request per launch, in arrival order
        o.slots = 1;
        o.max_batch = 1;
    }
    spx_server_s* S = new (std::nothrow) spx_server_s;
    if (!S) return spx_fail(SPX_ERR_NOMEM, "host allocation failed");
    S->o = o;
    hipError_t e = hipGetDevice(&S->device);
    S->slots.resize(o.slots);
    for (auto& sl : S->slots) {
        if (e == hipSuccess) e = hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&sl.done, hipEventDisableTiming);
        if (e == hipSuccess) e = hipMalloc(&sl.dtab, kTabBytes);
        if (e == hipSuccess) e = hipHostMalloc(&sl.htab, kTabBytes, hipHostMallocDefault);
    }
    if (e != hipSuccess) {
        const spx_status st = hip_fail(e, "server streams and tables");
        for (auto& sl : S->slots) {
            if (sl.htab) (void)hipHostFree(sl.htab);
            if (sl.dtab) (void)hipFree(sl.dtab);
            if (sl.done) (void)hipEventDestroy(sl.done);
            if (sl.stream) (void)hipStreamDestroy(sl.stream);
        }
        delete S;
        return st;
    }
    S->th = std::thread([S] { S->run(); });
    *out = S;
    return SPX_OK;
}

// Marks a finished batch's requests done (caller holds the lock).
void spx_server_s::retire(Slot& sl, double t, spx_status st) {
    for (Req* q : sl.batch) {
        q->t_done = t;
        q->status = st;
        q->done = true;
        if (q->ready) {
            ev_pool.push_back(q->ready);
            q->ready = nullptr;
        }
    }
    n_done += (int64_t)sl.batch.size();
    sl.mat->outstanding -= (int64_t)sl.batch.size();
    --sl.mat->in_flight;
    sl.mat = nullptr;
    sl.batch.clear();
    sl.busy = false;
    --in_flight;
    cv_done.notify_all();
}

// Grows an idle slot's buffer to `need` elements (hipFree waits for the device).
template <typename T>
static hipError_t grow(T** p, size_t* cap, size_t need) {
    if (need <= *cap) return hipSuccess;
    if (*p) (void)hipFree(*p);
    *p = nullptr;
    *cap = 0;
    hipError_t e = hipMalloc((void**)p, need * sizeof(T));
    if (e == hipSuccess) *cap = need;
    return e;
}

// Enqueues the slot's batch (lock not held; the slot is reserved).  The plain path runs the
// single-vector product on the handle; the coalescing path runs the product with k right-hand
// sides (k = 1 included) on the slot's own scratch, so batches of one matrix may overlap.
spx_status spx_server_s::launch(Slot& sl) {
    Mat* M = sl.mat;
    const int k = (int)sl.batch.size();
    hipStream_t s = sl.stream;
    hipError_t e;
    const spx_request& r0 = sl.batch[0]->r;
    const float beta0 = (1.0f - r0.damping) / (float)M->n;
    for (Req* q : sl.batch)  // x of each request is produced on the submitter's stream
        if (q->ready) {
            e = hipStreamWaitEvent(s, q->ready, 0);
            if (e != hipSuccess) return hip_fail(e, "waiting for a request's input");
        }
    if (!o.coalesce) {
        spx_status st = spx_spmv_f32(M->A, r0.x, r0.y, s);
        if (st != SPX_OK) return st;
        if (r0.kind == SPX_REQ_PAGERANK) {
            e = launch_serve_axpb(r0.y, M->m, r0.damping, beta0, s);
            if (e != hipSuccess) return hip_fail(e, "epilogue");
        }
        e = hipEventRecord(sl.done, s);
        return e == hipSuccess ? SPX_OK : hip_fail(e, "event");
    }
    const size_t before = (sl.xcap + sl.ycap + sl.hcap) * 4 + sl.crow_cap * 4 + sl.cval_cap * 8;
    e = grow(&sl.crow, &sl.crow_cap, (size_t)M->tiles + 1);
    if (e == hipSuccess) e = grow(&sl.cval, &sl.cval_cap, ((size_t)M->tiles + 1) * k);
    if (e == hipSuccess) e = grow(&sl.H, &sl.hcap, (size_t)M->nhot * k);
    if (e == hipSuccess && k > 1) e = grow(&sl.X, &sl.xcap, (size_t)M->n * k);
    if (e == hipSuccess && k > 1) e = grow(&sl.Y, &sl.ycap, (size_t)M->m * k);
    if (e != hipSuccess) return hip_fail(e, "slot buffers");
    {
        const size_t after = (sl.xcap + sl.ycap + sl.hcap) * 4 + sl.crow_cap * 4 + sl.cval_cap * 8;
        std::lock_guard<std::mutex> g(mu);
        staging += (int64_t)(after - before);
    }
    SpmmPlan P;
    P.coords = M->coords;
    P.tiles = M->tiles;
    P.carry_row = sl.crow;
    P.carry_val = sl.cval;
    P.h = sl.H;
    if (k == 1) {  // x and y are already a 1-column row-major X and Y
        e = spmm_crs(M->A, P, 1, r0.x, 1, r0.y, 1, 1, s);
        if (e == hipSuccess && r0.kind == SPX_REQ_PAGERANK)
            e = launch_serve_axpb(r0.y, M->m, r0.damping, beta0, s);
        if (e != hipSuccess) return hip_fail(e, "product");
    } else {
        char* h = (char*)sl.htab;
        const float** xs = (const float**)h;
        float** ys = (float**)(h + kMaxBatch * sizeof(void*));
        float* al = (float*)(h + 2 * kMaxBatch * sizeof(void*));
        float* be = al + kMaxBatch;
        for (int c = 0; c < k; ++c) {
            const spx_request& r = sl.batch[c]->r;
            xs[c] = r.x;
            ys[c] = r.y;
            const bool pr = r.kind == SPX_REQ_PAGERANK;
            al[c] = pr ? r.damping : 1.0f;
            be[c] = pr ? (1.0f - r.damping) / (float)M->n : 0.0f;
        }
        e = hipMemcpyAsync(sl.dtab, sl.htab, kTabBytes, hipMemcpyHostToDevice, s);
        if (e != hipSuccess) return hip_fail(e, "request table");
        char* d = (char*)sl.dtab;
        e = launch_serve_gather((const float* const*)d, k, M->n, sl.X, s);
        if (e == hipSuccess) e = spmm_crs(M->A, P, k, sl.X, k, sl.Y, k, 1, s);
        float* dal = (float*)(d + 2 * kMaxBatch * sizeof(void*));
        if (e == hipSuccess)
            e = launch_serve_scatter(sl.Y, k, M->m,
                                     (float* const*)(d + kMaxBatch * sizeof(void*)), dal,
                                     dal + kMaxBatch, s);
        if (e != hipSuccess) return hip_fail(e, "batched product");
    }
    e = hipEventRecord(sl.done, s);
    if (e != hipSuccess) return hip_fail(e, "event");
    return SPX_OK;
}

void spx_server_s::run() {
    (void)hipSetDevice(device);
    std::unique_lock<std::mutex> lk(mu);
    for (;;) {
        // retire finished batches
        for (auto& sl : slots) {
            if (!sl.busy) continue;
            const hipError_t q = hipEventQuery(sl.done);
            if (q == hipSuccess) retire(sl, now_us(), SPX_OK);
            else if (q != hipErrorNotReady) retire(sl, now_us(), SPX_ERR_HIP);
        }
        // fill free slots: oldest waiting request first, its matrix's waiting requests coalesced
        for (auto& sl : slots) {
            if (sl.busy) continue;
            Mat* best = nullptr;
            for (auto& kv : mats) {
                Mat* M = kv.second;
                if (M->waiting.empty()) continue;
                if (!best || M->waiting.front()->t_submit < best->waiting.front()->t_submit)
                    best = M;
            }
            if (!best) break;
            const int k = (int)std::min<size_t>(best->waiting.size(), (size_t)o.max_batch);
            for (int c = 0; c < k; ++c) {
                sl.batch.push_back(best->waiting.front());
                best->waiting.pop_front();
            }
            waiting_total -= k;
            ++best->in_flight;
            sl.mat = best;
            sl.busy = true;
            ++in_flight;
            ++n_batches;
            widest = std::max<int64_t>(widest, k);
            lk.unlock();
            const spx_status st = launch(sl);
            lk.lock();
            if (st != SPX_OK) {
                (void)hipStreamSynchronize(sl.stream);
                retire(sl, now_us(), st);
            }
        }
        if (stop && in_flight == 0 && waiting_total == 0) break;
        if (in_flight > 0) {
            lk.unlock();
            if (o.poll_us > 0) std::this_thread::sleep_for(std::chrono::microseconds(o.poll_us));
            else std::this_thread::yield();
            lk.lock();
        } else {
            cv_sched.wait(lk, [&] { return stop || waiting_total > 0; });
        }
    }
}

extern "C" spx_status spx_server_destroy(spx_server S) {
    if (!S) return SPX_OK;
    {
        std::lock_guard<std::mutex> g(S->mu);
        S->stop = true;
    }
    S->cv_sched.notify_all();
    S->th.join();
    for (auto& kv : S->reqs) {
        if (kv.second->ready) (void)hipEventDestroy(kv.second->ready);
        delete kv.second;
    }
    for (hipEvent_t ev : S->ev_pool) (void)hipEventDestroy(ev);
    for (auto& kv : S->mats) {
        spx_matrix_destroy(kv.second->A);
        delete kv.second;
    }
    for (auto& sl : S->slots) {
        (void)hipStreamSynchronize(sl.stream);
        for (void* p : {(void*)sl.X, (void*)sl.Y, (void*)sl.crow, (void*)sl.cval, (void*)sl.H})
            if (p) (void)hipFree(p);
        (void)hipHostFree(sl.htab);
        (void)hipFree(sl.dtab);
        (void)hipEventDestroy(sl.done);
        (void)hipStreamDestroy(sl.stream);
    }
    delete S;
    return SPX_OK;
}

extern "C" spx_status spx_server_add_matrix(spx_server S, const spx_coo_desc* coo,
                                            spx_format fmt, const spx_convert_opts* opts,
                                            void* stream, int32_t* id, int64_t* bytes) {
    if (!S || !coo || !opts || !id) return spx_fail(SPX_ERR_INVALID_ARG, "NULL argument");
    if (fmt != SPX_CSR_ROWSPLIT && fmt != SPX_CSR_MERGE)
        return spx_fail(SPX_ERR_UNSUPPORTED, "served matrices must be CRS (row-split or merge)");
    if (opts->value_type != SPX_F32 && opts->value_type != SPX_BF16)
        return spx_fail(SPX_ERR_UNSUPPORTED, "served matrices store FP32 or bfloat16 values");
    if (coo->m < 0 || coo->n < 0 || coo->nnz < 0)
        return spx_fail(SPX_ERR_INVALID_ARG, "negative size");
    const int64_t need = footprint_bound(coo, opts->value_type, S->o.max_batch);
    const int64_t stage = staging_bound(coo, S->o.max_batch);
    {
        std::lock_guard<std::mutex> g(S->mu);
        const int64_t stage_all = (int64_t)S->o.slots * std::max(S->stage_max, stage);
        if (S->used + need + stage_all > S->o.memory_budget) {
            char buf[200];
            snprintf(buf, sizeof buf, "admission: %lld bytes needed and %lld for slot staging, "
                     "%lld of %lld free", (long long)need, (long long)stage_all,
                     (long long)(S->o.memory_budget - S->used), (long long)S->o.memory_budget);
            return spx_fail(SPX_ERR_NOMEM, buf);
        }
        S->used += need;  // reserved while converting
        S->stage_max = std::max(S->stage_max, stage);
    }
    auto unreserve = [&] {
        std::lock_guard<std::mutex> g(S->mu);
        S->used -= need;
    };
    spx_matrix A = nullptr;
    spx_status st = spx_convert(coo, fmt, opts, stream, &A, nullptr);
    if (st != SPX_OK) {
        unreserve();
        return st;
    }
    // a row-split handle gets its merge tiles for products with several right-hand sides here,
    // through one product, so the scheduler never allocates on a handle
    const int2* coords = A->mp_coords;
    int32_t tiles = A->mp_tiles;
    if (S->o.coalesce && A->fmt == SPX_CSR_ROWSPLIT && coo->m > 0) {
        float *X = nullptr, *Y = nullptr;
        hipError_t e = hipMalloc((void**)&X, (size_t)std::max(coo->n, 1) * 4);
        if (e == hipSuccess) e = hipMalloc((void**)&Y, (size_t)coo->m * 4);
        if (e == hipSuccess)
            e = hipMemsetAsync(X, 0, (size_t)std::max(coo->n, 1) * 4, (hipStream_t)stream);
        if (e == hipSuccess) {
            st = spx_spmm(A, 1, X, 1, Y, 1, SPX_ROW_MAJOR, stream);
            e = hipStreamSynchronize((hipStream_t)stream);
        }
        if (X) (void)hipFree(X);
        if (Y) (void)hipFree(Y);
        if (st == SPX_OK && e != hipSuccess) st = hip_fail(e, "merge tiles");
        if (st != SPX_OK) {
            spx_matrix_destroy(A);
            unreserve();
            return st;
        }
        coords = A->mm_coords;
        tiles = A->mm_tiles;
    }
    Mat* M = new (std::nothrow) Mat;
    if (!M) {
        spx_matrix_destroy(A);
        unreserve();
        return spx_fail(SPX_ERR_NOMEM, "host allocation failed");
    }
    M->A = A;
    M->m = coo->m;
    M->n = coo->n;
    M->bytes = need;
    M->coords = coords;
    M->tiles = tiles;
    M->nhot = A->nhot;
    {
        std::lock_guard<std::mutex> g(S->mu);
        M->id = S->next_id++;
        S->mats[M->id] = M;
    }
    *id = M->id;
    if (bytes) *bytes = need;
    return SPX_OK;
}

extern "C" spx_status spx_server_remove_matrix(spx_server S, int32_t id) {
    if (!S) return spx_fail(SPX_ERR_INVALID_ARG, "server is NULL");
    std::unique_lock<std::mutex> lk(S->mu);
    auto it = S->mats.find(id);
    if (it == S->mats.end()) return spx_fail(SPX_ERR_INVALID_ARG, "unknown matrix id");
    Mat* M = it->second;
    S->cv_done.wait(lk, [&] { return M->outstanding == 0; });
    S->mats.erase(it);
    S->used -= M->bytes;
    lk.unlock();
    spx_matrix_destroy(M->A);
    delete M;
    return SPX_OK;
}

static bool overlap(const void* a, size_t na, const void* b, size_t nb) {
    const uintptr_t a0 = (uintptr_t)a, b0 = (uintptr_t)b;
    return na > 0 && nb > 0 && a0 < b0 + nb && b0 < a0 + na;
}

// Checks and queues one request (caller holds the lock).
static spx_status submit_locked(spx_server S, const spx_request* r, uint64_t* ticket) {
    auto it = S->mats.find(r->matrix);
    if (it == S->mats.end()) return spx_fail(SPX_ERR_INVALID_ARG, "unknown matrix id");
    Mat* M = it->second;
    if (r->kind != SPX_REQ_SPMV && r->kind != SPX_REQ_PAGERANK)
        return spx_fail(SPX_ERR_INVALID_ARG, "unknown request kind");
    if (r->kind == SPX_REQ_PAGERANK && !(r->damping >= 0.0f && r->damping <= 1.0f))
        return spx_fail(SPX_ERR_INVALID_ARG, "damping must be in [0, 1]");
    if ((M->m > 0 && !r->y) || (M->n > 0 && !r->x))
        return spx_fail(SPX_ERR_INVALID_ARG, "x or y is NULL");
    if (overlap(r->x, (size_t)M->n * 4, r->y, (size_t)M->m * 4))
        return spx_fail(SPX_ERR_ALIAS, "x and y overlap");
    hipEvent_t ev = nullptr;
    if (r->stream && M->m > 0) {
        hipError_t e = hipSuccess;
        if (!S->ev_pool.empty()) {
            ev = S->ev_pool.back();
            S->ev_pool.pop_back();
        } else {
            e = hipEventCreateWithFlags(&ev, hipEventDisableTiming);
        }
        if (e == hipSuccess) e = hipEventRecord(ev, (hipStream_t)r->stream);
        if (e != hipSuccess) {
            if (ev) S->ev_pool.push_back(ev);
            return hip_fail(e, "recording the request's input event");
        }
    }
    Req* q = new (std::nothrow) Req;
    if (!q) {
        if (ev) S->ev_pool.push_back(ev);
        return spx_fail(SPX_ERR_NOMEM, "host allocation failed");
    }
    q->r = *r;
    q->ready = ev;
    q->ticket = S->next_ticket++;
    q->t_submit = S->now_us();
    if (M->m == 0) {  // nothing to compute
        q->t_done = q->t_submit;
        q->done = true;
        ++S->n_done;
    } else {
        M->waiting.push_back(q);
        ++M->outstanding;
        ++S->waiting_total;
    }
    S->reqs[q->ticket] = q;
    *ticket = q->ticket;
    return SPX_OK;
}

extern "C" spx_status spx_server_submit(spx_server S, const spx_request* req, uint64_t* ticket) {
    if (!S || !req || !ticket) return spx_fail(SPX_ERR_INVALID_ARG, "NULL argument");
    spx_status st;
    {
        std::lock_guard<std::mutex> g(S->mu);
        st = submit_locked(S, req, ticket);
    }
    if (st == SPX_OK) S->cv_sched.notify_one();
    return st;
}

extern "C" spx_status spx_server_wait(spx_server S, uint64_t ticket, double* latency_us) {
    if (!S) return spx_fail(SPX_ERR_INVALID_ARG, "server is NULL");
    std::unique_lock<std::mutex> lk(S->mu);
    auto it = S->reqs.find(ticket);
    if (it == S->reqs.end()) return spx_fail(SPX_ERR_INVALID_ARG, "unknown ticket");
    Req* q = it->second;
    S->cv_done.wait(lk, [&] { return q->done; });
    S->reqs.erase(it);
    lk.unlock();
    const spx_status st = q->status;
    if (latency_us) *latency_us = q->t_done - q->t_submit;
    delete q;
    if (st != SPX_OK) return spx_fail(st, "request failed on the device");
    return SPX_OK;
}

extern "C" spx_status spx_server_replay(spx_server S, const spx_request* reqs,
                                        const double* arrival_us, int64_t count,
                                        double* latency_us, double* wall_us) {
    if (!S || count < 0 || (count > 0 && (!reqs || !arrival_us || !latency_us)))
        return spx_fail(SPX_ERR_INVALID_ARG, "NULL argument or negative count");
    std::vector<uint64_t> tickets;
    tickets.reserve((size_t)count);
    spx_status first_err = SPX_OK;
    const auto t0 = clock_type::now();
    double t_first = -1, t_last = 0;
    for (int64_t i = 0; i < count; ++i) {
        const auto due = t0 + std::chrono::duration_cast<clock_type::duration>(
                                  std::chrono::duration<double, std::micro>(arrival_us[i]));
        while (clock_type::now() < due) {
        }
        uint64_t t;
        const spx_status st = spx_server_submit(S, &reqs[i], &t);
        if (st != SPX_OK) {
            first_err = st;
            break;
        }
        tickets.push_back(t);
    }
    for (size_t i = 0; i < tickets.size(); ++i) {
        std::unique_lock<std::mutex> lk(S->mu);
        Req* q = S->reqs[tickets[i]];
        S->cv_done.wait(lk, [&] { return q->done; });
        if (t_first < 0 || q->t_submit < t_first) t_first = q->t_submit;
        t_last = std::max(t_last, q->t_done);
        latency_us[i] = q->t_done - q->t_submit;
        if (q->status != SPX_OK && first_err == SPX_OK) first_err = q->status;
        S->reqs.erase(tickets[i]);
        delete q;
    }
    for (int64_t i = (int64_t)tickets.size(); i < count; ++i) latency_us[i] = -1.0;
    if (wall_us) *wall_us = t_first < 0 ? 0.0 : t_last - t_first;
    if (first_err != SPX_OK) return spx_fail(first_err, "a request was rejected or failed");
    return SPX_OK;
}

extern "C" spx_status spx_server_get_stats(spx_server S, spx_server_stats* st) {
    if (!S || !st) return spx_fail(SPX_ERR_INVALID_ARG, "NULL argument");
    std::lock_guard<std::mutex> g(S->mu);
    st->requests = S->n_done;
    st->batches = S->n_batches;
    st->max_batch_seen = S->widest;
    st->bytes_resident = S->used;
    st->memory_budget = S->o.memory_budget;
    st->matrices = (int32_t)S->mats.size();
    st->in_flight = S->in_flight;
    st->bytes_staging = (int64_t)S->o.slots * S->stage_max;
    return SPX_OK;
}
