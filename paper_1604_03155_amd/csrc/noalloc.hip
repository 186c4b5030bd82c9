// Allocation-free apply (vg_apply_noalloc): the apply program of vg_apply,
// with its workspace in a file-scope device array instead of a caller buffer
// or the plan's internal allocation, for callers that cannot allocate.
#include <atomic>
#include <exception>
#include <mutex>
#include <new>

#include "plan.h"

namespace vg {
namespace {

// The workspace of vg_apply_noalloc.  Every GPU the library runs on holds
// its own copy until the process ends.  In host code `scratch` names a
// host-side stand-in, not device memory: host code uses only the per-device
// address that hipGetSymbolAddress returns.
static __device__ __align__(256) unsigned char scratch[VG_NOALLOC_WORKSPACE_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_lookup_mutex;
std::atomic<void*> g_scratch[kMaxDevices];

// Device address of the current device's array, looked up on the first call
// made with that device current.
vg_status scratch_address(int device, void** out) {
    if (device < 0 || device >= kMaxDevices) return fail(VG_ERR_DEVICE, "device index out of range");
    void* ptr = g_scratch[device].load(std::memory_order_acquire);
    if (!ptr) {
        std::lock_guard<std::mutex> lk(g_lookup_mutex);
        ptr = g_scratch[device].load(std::memory_order_relaxed);
        if (!ptr) {
            hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
            if (e != hipSuccess || !ptr) return from_hip(e == hipSuccess ? hipErrorInvalidSymbol : e, "scratch lookup");
            g_scratch[device].store(ptr, std::memory_order_release);
        }
    }
    *out = ptr;
    return VG_OK;
}

}  // namespace
}  // namespace vg

using namespace vg;

extern "C" vg_status vg_apply_noalloc(const vg_plan* p, const void* f, void* phi, void* stream) {
    try {
        if (!p) return fail(VG_ERR_INVALID_ARG, "plan is NULL");
        if (!f || !phi) return fail(VG_ERR_INVALID_ARG, "f and phi must be device pointers");
        if (p->apply_prog.ws_bytes > (size_t)VG_NOALLOC_WORKSPACE_BYTES)
            return fail(VG_ERR_UNSUPPORTED_SIZE,
                        "vg_apply_noalloc: the plan's workspace exceeds VG_NOALLOC_WORKSPACE_BYTES (128 MiB); "
                        "use vg_apply with a workspace");
        int dev = -1;
        hipError_t e = hipGetDevice(&dev);
        if (e != hipSuccess) return from_hip(e, "hipGetDevice");
        if (dev != p->device) return fail(VG_ERR_INVALID_ARG, "the plan belongs to another device");
        void* ws = nullptr;
        vg_status st = scratch_address(dev, &ws);
        if (st != VG_OK) return st;
        return run_program_noalloc(p, p->apply_prog, f, phi, nullptr, ws, reinterpret_cast<hipStream_t>(stream));
    } catch (const std::bad_alloc&) {
        return fail(VG_ERR_OUT_OF_MEMORY, "host allocation failed");
    } catch (...) {
        return fail(VG_ERR_INTERNAL, "unexpected exception");
    }
}
