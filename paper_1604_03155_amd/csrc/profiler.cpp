// Pass profiler: HIP events recorded between consecutive passes of apply /
// gradient calls, collected on demand and aggregated per pass name.
#include <algorithm>
#include <cstring>
#include <map>
#include <string>
#include <vector>

#include "plan.h"

namespace vg {

namespace {
struct Rec {
    const char* name;
    hipEvent_t a, b;
    double bytes;
};
std::mutex g_mu;
int g_mode = 0;  // 0 off, 1 every pass, 2 the pass with the most bytes
std::vector<Rec> g_recs;
std::vector<hipEvent_t> g_pool;

hipEvent_t take_event() {
    if (!g_pool.empty()) {
        hipEvent_t e = g_pool.back();
        g_pool.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}
}  // namespace

int profiler_mode() {
    std::lock_guard<std::mutex> lk(g_mu);
    return g_mode;
}

// Record one event on `s`; returns it (nullptr when disabled or on failure).
void* profiler_mark(hipStream_t s) {
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_mode) return nullptr;
    hipEvent_t e = take_event();
    if (e && hipEventRecord(e, s) != hipSuccess) return nullptr;
    return e;
}

void profiler_add(const char* name, void* a, void* b, double bytes) {
    if (!a || !b) return;
    std::lock_guard<std::mutex> lk(g_mu);
    g_recs.push_back({name, (hipEvent_t)a, (hipEvent_t)b, bytes});
}

}  // namespace vg

using namespace vg;

extern "C" vg_status vg_profiler_enable(int enable) {
    if (enable < 0 || enable > 2) return fail(VG_ERR_INVALID_ARG, "profiler mode must be 0, 1 or 2");
    std::lock_guard<std::mutex> lk(g_mu);
    g_mode = enable;
    return VG_OK;
}

extern "C" vg_status vg_profiler_collect(vg_pass_time* out, int max_entries, int* n_entries) {
    if (!n_entries || (max_entries > 0 && !out)) return fail(VG_ERR_INVALID_ARG, "NULL argument");
    std::lock_guard<std::mutex> lk(g_mu);
    struct Agg {
        int n = 0;
        double ms = 0.0, bytes = 0.0;
        size_t order = 0;
    };
    std::map<std::string, Agg> agg;
    std::vector<hipEvent_t> used;
    vg_status st = VG_OK;
    for (size_t i = 0; i < g_recs.size(); ++i) {
        const Rec& r = g_recs[i];
        float ms = 0.f;
        hipError_t e = hipEventSynchronize(r.b);
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, r.a, r.b);
        if (e != hipSuccess) {
            st = from_hip(e, "profiler event");
            continue;
        }
        Agg& a = agg[r.name];
        if (a.n == 0) a.order = i;
        a.n += 1;
        a.ms += ms;
        a.bytes = r.bytes;
        used.push_back(r.a);
        used.push_back(r.b);
    }
    std::vector<std::pair<size_t, std::string>> order;
    for (auto& kv : agg) order.push_back({kv.second.order, kv.first});
    std::sort(order.begin(), order.end());
    int n = 0;
    for (auto& o : order) {
        if (n >= max_entries) break;
        const Agg& a = agg[o.second];
        std::memset(&out[n], 0, sizeof(vg_pass_time));
        std::strncpy(out[n].name, o.second.c_str(), sizeof(out[n].name) - 1);
        out[n].launches = a.n;
        out[n].total_ms = a.ms;
        out[n].bytes_per_launch = a.bytes;
        ++n;
    }
    *n_entries = n;
    std::sort(used.begin(), used.end());
    used.erase(std::unique(used.begin(), used.end()), used.end());
    for (hipEvent_t e : used) g_pool.push_back(e);
    g_recs.clear();
    return st;
}
