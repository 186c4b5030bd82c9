// Batched applies over plans of mixed size and kernel.
#include <algorithm>
#include <cstring>

#include "plan.h"

namespace vg {

namespace {
size_t align256(size_t x) { return (x + 255) & ~size_t(255); }
std::mutex g_batch_mutex;
void* g_batch_ws = nullptr;
size_t g_batch_ws_bytes = 0;
}  // namespace

int fft_max_lds_bytes_for_device() {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 65536;
    int v = 0;
    if (hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess || v <= 0) return 65536;
    return v;
}

size_t batched_workspace_size(int count, const vg_plan* const* plans) {
    size_t total = 0;
    for (int i = 0; i < count; ++i) total += align256(plans[i] ? plans[i]->apply_prog.ws_bytes : 0);
    return total;
}

void batched_release_plan(const vg_plan*) {}

vg_status batched_apply(int count, const vg_plan* const* plans, const void* const* f, void* const* phi,
                        void* workspace, hipStream_t stream) {
    const size_t need = batched_workspace_size(count, plans);
    void* ws = workspace;
    std::unique_lock<std::mutex> lk(g_batch_mutex, std::defer_lock);
    if (!ws) {
        lk.lock();
        if (g_batch_ws_bytes < need) {
            if (g_batch_ws) (void)hipFree(g_batch_ws);
            g_batch_ws = nullptr;
            g_batch_ws_bytes = 0;
            hipError_t e = dev_malloc(&g_batch_ws, need);
            if (e != hipSuccess) return from_hip(e, "batched workspace");
            g_batch_ws_bytes = need;
        }
        ws = g_batch_ws;
    }
    size_t off = 0;
    for (int i = 0; i < count; ++i) {
        void* w = static_cast<unsigned char*>(ws) + off;
        vg_status st = run_program(plans[i], plans[i]->apply_prog, f[i], phi[i], nullptr, w, stream);
        if (st != VG_OK) return st;
        off += align256(plans[i]->apply_prog.ws_bytes);
    }
    return VG_OK;
}

}  // namespace vg
