// Plan-time autotuner: times the apply program under candidate layout
// configurations (intermediate pitch padding, XCD-aware tile order, four-step
// split of long 2D columns, specialised vs generic kernels) on the plan's own
// device and keeps the fastest.  Inputs are zero arrays: the kernels' cost
// does not depend on the data.
#include <algorithm>
#include <chrono>
#include <cstring>

#include "plan.h"

namespace vg {

namespace {

struct DevMem {
    void* p = nullptr;
    ~DevMem() {
        if (p) (void)hipFree(p);
    }
};

// Time `reps` applies (after one untimed run); returns ms per apply or a
// negative value if the candidate cannot run.
double time_apply(vg_plan* p, void* f, void* phi, hipStream_t s, int reps) {
    DevMem ws;
    if (p->apply_prog.ws_bytes && dev_malloc(&ws.p, p->apply_prog.ws_bytes) != hipSuccess) return -1.0;
    if (run_program(p, p->apply_prog, f, phi, nullptr, ws.p, s) != VG_OK) return -1.0;
    hipEvent_t a = nullptr, b = nullptr;
    if (hipEventCreate(&a) != hipSuccess) return -1.0;
    if (hipEventCreate(&b) != hipSuccess) {
        (void)hipEventDestroy(a);
        return -1.0;
    }
    double ms = -1.0;
    bool ok = hipEventRecord(a, s) == hipSuccess;
    for (int i = 0; ok && i < reps; ++i) ok = run_program(p, p->apply_prog, f, phi, nullptr, ws.p, s) == VG_OK;
    if (ok) ok = hipEventRecord(b, s) == hipSuccess && hipEventSynchronize(b) == hipSuccess;
    float t = 0.f;
    if (ok && hipEventElapsedTime(&t, a, b) == hipSuccess) ms = (double)t / reps;
    (void)hipEventDestroy(a);
    (void)hipEventDestroy(b);
    return ms;
}

std::vector<LayoutConfig> candidates(const vg_plan* p) {
    const bool full = p->tune == VG_TUNE_FULL;
    std::vector<int> pads = full ? std::vector<int>{0, 256, 512, 1024} : std::vector<int>{256, 0};
    std::vector<int> splits = {0};
    const int L = 2 * p->N;
    if (p->d == 2 && L > 1024) {
        const std::vector<int> all = four_step_splits(L, p->fp64);
        splits.assign(all.begin(), all.begin() + std::min<size_t>(all.size(), full ? 6 : 3));
        if (splits.empty()) splits = {0};
    }
    std::vector<LayoutConfig> out;
    for (int s : splits)
        for (int pad : pads)
            for (int x : {1, 0}) {
                LayoutConfig c;
                c.pad_bytes = pad;
                c.xcd_map = x;
                c.fs_L1 = s;
                out.push_back(c);
            }
    if (full) {
        LayoutConfig c;
        c.generic = 1;
        out.push_back(c);
    }
    return out;
}

}  // namespace

vg_status autotune(vg_plan* p, hipStream_t s) {
    if (p->tune == VG_TUNE_OFF) return VG_OK;
    const auto t0 = std::chrono::steady_clock::now();
    long long V = 1;
    for (int i = 0; i < p->d; ++i) V *= p->N;
    const size_t bytes = (size_t)V * (p->fp64 ? 16 : 8);
    DevMem f, phi;
    hipError_t he = dev_malloc(&f.p, bytes);
    if (he == hipSuccess) he = dev_malloc(&phi.p, bytes);
    if (he == hipSuccess) he = hipMemsetAsync(f.p, 0, bytes, s);
    if (he != hipSuccess) return from_hip(he, "autotune buffers");
    const int reps = p->tune == VG_TUNE_FULL ? 10 : 3;
    const LayoutConfig start = p->cfg;
    LayoutConfig best = start;
    double best_ms = -1.0;
    int n = 0;
    for (const LayoutConfig& c : candidates(p)) {
        p->cfg = c;
        if (build_programs(p, s) != VG_OK) continue;
        const double ms = time_apply(p, f.p, phi.p, s, reps);
        ++n;
        if (ms > 0.0 && (best_ms < 0.0 || ms < best_ms)) {
            best_ms = ms;
            best = c;
        }
    }
    he = hipStreamSynchronize(s);
    if (he != hipSuccess) return from_hip(he, "autotune");
    p->cfg = best_ms > 0.0 ? best : start;
    vg_status st = build_programs(p, s);
    if (st != VG_OK) return st;
    p->tune_candidates = n;
    p->tune_ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
    return VG_OK;
}

}  // namespace vg
