// spx_prof.cpp -- per-kernel launch timing with HIP events (measurement aid).
//
// With profiling enabled every kernel launch of the library is bracketed by two events recorded
// on the launch stream.  spx_profile_collect waits for the recorded events, folds them into
// per-kernel statistics and returns them.  Event pairs are kept pending until collected.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <cstring>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/spx.h"
#include "spx_prof.h"

namespace {
struct Pending {
    const char* name;
    hipEvent_t e0, e1;
};
struct Stat {
    int64_t launches = 0;
    double total = 0, mn = 1e300, mx = 0;
};
std::atomic<bool> g_on{false};
std::mutex g_mu;
std::vector<Pending> g_pending;
std::vector<hipEvent_t> g_pool;
std::map<std::string, Stat> g_stats;

hipEvent_t get_event() {
    {
        std::lock_guard<std::mutex> lk(g_mu);
        if (!g_pool.empty()) {
            hipEvent_t e = g_pool.back();
            g_pool.pop_back();
            return e;
        }
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) {
        (void)hipGetLastError();
        return nullptr;
    }
    return e;
}

void drain_locked() {
    for (const Pending& p : g_pending) {
        float ms = 0.f;
        if (hipEventSynchronize(p.e1) == hipSuccess && hipEventElapsedTime(&ms, p.e0, p.e1) == hipSuccess) {
            Stat& s = g_stats[p.name];
            s.launches += 1;
            s.total += ms;
            s.mn = std::min(s.mn, (double)ms);
            s.mx = std::max(s.mx, (double)ms);
        } else {
            (void)hipGetLastError();
        }
        g_pool.push_back(p.e0);
        g_pool.push_back(p.e1);
    }
    g_pending.clear();
}
}  // namespace

bool spx_prof_on() { return g_on.load(std::memory_order_relaxed); }

hipEvent_t spx_prof_begin(hipStream_t s) {
    hipEvent_t e = get_event();
    if (e && hipEventRecord(e, s) != hipSuccess) {
        (void)hipGetLastError();
        return nullptr;
    }
    return e;
}

void spx_prof_end(const char* name, hipStream_t s, hipEvent_t start) {
    hipEvent_t e = get_event();
    if (!e || hipEventRecord(e, s) != hipSuccess) {
        (void)hipGetLastError();
        return;
    }
    std::lock_guard<std::mutex> lk(g_mu);
    g_pending.push_back({name, start, e});
}

extern "C" spx_status spx_profile_enable(int32_t enable) {
    std::lock_guard<std::mutex> lk(g_mu);
    drain_locked();
    g_stats.clear();
    g_on.store(enable != 0);
    return SPX_OK;
}

extern "C" spx_status spx_profile_collect(spx_kernel_stat* out, int32_t max, int32_t* count) {
    if (!count || (max > 0 && !out)) return SPX_ERR_INVALID_ARG;
    std::lock_guard<std::mutex> lk(g_mu);
    drain_locked();
    int32_t i = 0;
    for (const auto& kv : g_stats) {
        if (i < max) {
            spx_kernel_stat& o = out[i];
            std::memset(&o, 0, sizeof o);
            std::strncpy(o.name, kv.first.c_str(), sizeof o.name - 1);
            o.launches = kv.second.launches;
            o.total_ms = kv.second.total;
            o.min_ms = kv.second.mn;
            o.max_ms = kv.second.mx;
        }
        ++i;
    }
    *count = i;
    return SPX_OK;
}
