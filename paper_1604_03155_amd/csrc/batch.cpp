// Batched applies over plans of mixed d, N, kernel and k.
//
// Every plan's apply program is a short chain of passes (3D: rows, axis 2,
// fused axis 1, axis 2 inverse, rows inverse); pass s of density j depends
// only on pass s - 1 of density j.  The batch therefore runs stage by stage:
// at stage s, all densities whose pass s has the same specialised kernel
// (length, direction, kind, table type) share ONE grouped launch whose
// workgroups take (density, tile) items; passes without a grouped kernel
// launch once per density.  The whole launch sequence is captured once in a
// HIP graph and replayed while (plans, arrays, workspace) repeat, so a batch
// of 64 densities costs a handful of graph nodes instead of 320 launches.
#include <algorithm>
#include <cstdint>
#include <cstring>
#include <list>
#include <map>
#include <memory>
#include <tuple>

#include "batch_cache.h"
#include "plan.h"

namespace vg {

namespace {
size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

struct BatchLaunch {
    bool grouped = false;
    PassDesc desc;        // single launch: the pass; grouped: the prototype
    int mode = 0, kind = 0;
    size_t desc_off = 0;  // grouped: byte offsets of descriptors / starts in the blob
    size_t start_off = 0;
    int nitems = 0;
    unsigned ntiles = 0;
    const char* name = nullptr;
};

// The library's internal batched workspace (calls with workspace == NULL).
// Entries that use it hold a reference, so a buffer replaced by a larger one
// stays allocated while a pinned entry (recorded into a caller's graph)
// still points into it.
struct DevBlock {
    void* p = nullptr;
    size_t bytes = 0;
    ~DevBlock() {
        if (p) (void)hipFree(p);
    }
};

struct BatchEntry {
    std::vector<const vg_plan*> plans;
    std::vector<const void*> f;
    std::vector<void*> phi;
    void* ws = nullptr;
    int device = 0;
    bool fp64 = false;
    double bytes = 0.0;
    std::vector<BatchLaunch> launches;
    void* blob = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    bool graph_failed = false;
    bool pinned = false;                  // recorded into a caller's capture: never evicted
    std::shared_ptr<DevBlock> ws_hold;    // the internal workspace block, when ws points into it

    ~BatchEntry() {
        if (exec) (void)hipGraphExecDestroy(exec);
        if (graph) (void)hipGraphDestroy(graph);
        if (blob) (void)hipFree(blob);
    }
};

constexpr size_t kMaxEntries = 8;

std::mutex g_batch_mutex;
std::shared_ptr<DevBlock> g_batch_ws;           // internal workspace
BatchCache<BatchEntry> g_entries;               // most recently used first
std::map<int, hipStream_t> g_capture_streams;   // per device

// a dropped entry's graph may still be running
void sync_device() { (void)hipDeviceSynchronize(); }

long long tiles_of(const PassDesc& d, int mode) {
    return mode == MODE_COL ? (long long)d.outer * ((d.inner + d.C - 1) / d.C) : ((long long)d.outer + d.C - 1) / d.C;
}

bool env_flag(const char* name) {
    const char* v = std::getenv(name);
    return v && *v && std::strcmp(v, "0") != 0;
}

// Group key of a specialised pass: everything that selects the kernel (the
// table's dimension and type only matter to the fused kinds).
using GroupKey = std::tuple<int, int, int, int, int, int, int, int, int>;
GroupKey key_of(const BoundStep& b) {
    const bool fused = b.kind == KIND_FUSED || b.kind == KIND_FUSED_GRAD || b.kind == KIND_FUSED_DERIV;
    return GroupKey(b.desc.L, b.mode, b.kind, b.desc.C, fused ? b.desc.d : 0, fused ? b.desc.table_complex | (b.desc.table_full << 1) : 0,
                    b.desc.post_tw, b.desc.fs_L1 != 0 ? 1 : 0, b.desc.specialised);
}

vg_status build_entry(BatchEntry& e) {
    const int count = (int)e.plans.size();
    std::vector<std::vector<BoundStep>> progs(count);
    size_t off = 0;
    size_t nstage = 0;
    e.bytes = 0.0;
    for (int i = 0; i < count; ++i) {
        const vg_plan* p = e.plans[i];
        void* w = static_cast<unsigned char*>(e.ws) + off;
        progs[i] = bind_program(p, p->apply_prog, e.f[i], e.phi[i], nullptr, w);
        off += align256(p->apply_prog.ws_bytes);
        nstage = std::max(nstage, progs[i].size());
        for (const BoundStep& b : progs[i]) e.bytes += b.bytes;
    }
    const bool group = !env_flag("VG_BATCH_NO_GROUP");
    // host images of the grouped launches' descriptor and offset arrays
    std::vector<unsigned char> host;
    auto reserve = [&](size_t bytes) {
        const size_t o = align256(host.size());
        host.resize(o + bytes);
        return o;
    };
    e.launches.clear();
    for (size_t s = 0; s < nstage; ++s) {
        std::map<GroupKey, std::vector<int>> groups;  // key -> densities, in batch order
        std::vector<int> singles;
        for (int i = 0; i < count; ++i) {
            if (s >= progs[i].size()) continue;
            const BoundStep& b = progs[i][s];
            if (group && b.desc.specialised && b.kind < 100 && fast_group_supported(b.desc.L))
                groups[key_of(b)].push_back(i);
            else
                singles.push_back(i);
        }
        for (auto& kv : groups) {
            const std::vector<int>& items = kv.second;
            if (items.size() == 1) {
                singles.push_back(items[0]);
                continue;
            }
            BatchLaunch bl;
            bl.grouped = true;
            const BoundStep& b0 = progs[items[0]][s];
            bl.desc = b0.desc;
            bl.mode = b0.mode;
            bl.kind = b0.kind;
            bl.name = b0.name;
            bl.nitems = (int)items.size();
            bl.desc_off = reserve(sizeof(PassDesc) * items.size());
            bl.start_off = reserve(sizeof(unsigned) * (items.size() + 1));
            long long total = 0;
            for (size_t j = 0; j < items.size(); ++j) {
                const BoundStep& b = progs[items[j]][s];
                std::memcpy(host.data() + bl.desc_off + j * sizeof(PassDesc), &b.desc, sizeof(PassDesc));
                const unsigned st = (unsigned)total;
                std::memcpy(host.data() + bl.start_off + j * sizeof(unsigned), &st, sizeof(unsigned));
                total += tiles_of(b.desc, b.mode);
                if (total > 0x7fffffffLL) return fail(VG_ERR_UNSUPPORTED_SIZE, "batched pass has too many tiles");
            }
            const unsigned tot = (unsigned)total;
            std::memcpy(host.data() + bl.start_off + items.size() * sizeof(unsigned), &tot, sizeof(unsigned));
            bl.ntiles = tot;
            e.launches.push_back(bl);
        }
        std::sort(singles.begin(), singles.end());
        for (int i : singles) {
            const BoundStep& b = progs[i][s];
            BatchLaunch bl;
            bl.desc = b.desc;
            bl.mode = b.mode;
            bl.kind = b.kind;
            bl.name = b.name;
            e.launches.push_back(bl);
        }
    }
    if (!host.empty()) {
        hipError_t he = dev_malloc(&e.blob, host.size());
        if (he != hipSuccess) return from_hip(he, "batched descriptors");
        he = hipMemcpy(e.blob, host.data(), host.size(), hipMemcpyHostToDevice);
        if (he != hipSuccess) return from_hip(he, "batched descriptor upload");
    }
    return VG_OK;
}

vg_status issue(const BatchEntry& e, hipStream_t stream) {
    for (const BatchLaunch& bl : e.launches) {
        hipError_t he;
        if (bl.grouped) {
            GroupArgs g;
            g.descs = reinterpret_cast<const PassDesc*>(static_cast<const unsigned char*>(e.blob) + bl.desc_off);
            g.starts = reinterpret_cast<const unsigned*>(static_cast<const unsigned char*>(e.blob) + bl.start_off);
            g.nitems = bl.nitems;
            g.ntiles = bl.ntiles;
            he = launch_fast_group(bl.desc, g, bl.mode, bl.kind, e.fp64, stream);
        } else {
            he = launch_fft_pass(bl.desc, bl.mode, bl.kind, e.fp64, stream);
        }
        if (he != hipSuccess) return from_hip(he, bl.name);
    }
    return VG_OK;
}

vg_status capture(BatchEntry& e) {
    hipStream_t& cs = g_capture_streams[e.device];
    if (!cs) {
        hipError_t he = hipStreamCreateWithFlags(&cs, hipStreamNonBlocking);
        if (he != hipSuccess) {
            cs = nullptr;
            return from_hip(he, "capture stream");
        }
    }
    hipError_t he = hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal);
    if (he != hipSuccess) return from_hip(he, "begin capture");
    const vg_status st = issue(e, cs);
    hipGraph_t g = nullptr;
    he = hipStreamEndCapture(cs, &g);
    if (st != VG_OK) {
        if (g) (void)hipGraphDestroy(g);
        return st;
    }
    if (he != hipSuccess) return from_hip(he, "end capture");
    e.graph = g;
    he = hipGraphInstantiate(&e.exec, g, nullptr, nullptr, 0);
    if (he != hipSuccess) {
        e.exec = nullptr;
        return from_hip(he, "graph instantiate");
    }
    return VG_OK;
}

bool same_key(const BatchEntry& e, int count, const vg_plan* const* plans, const void* const* f, void* const* phi,
              void* ws, int dev) {
    if ((int)e.plans.size() != count || e.ws != ws || e.device != dev) return false;
    for (int i = 0; i < count; ++i)
        if (e.plans[i] != plans[i] || e.f[i] != f[i] || e.phi[i] != phi[i]) return false;
    return true;
}

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

void batched_release_plan(const vg_plan* p) {
    std::lock_guard<std::mutex> lk(g_batch_mutex);
    // pinned entries too: a caller's graph that recorded a batch with this
    // plan is invalid once the plan (its tables) is gone
    g_entries.drop_if([&](const BatchEntry& e) { return std::find(e.plans.begin(), e.plans.end(), p) != e.plans.end(); },
                      sync_device);
}

vg_status batched_apply(int count, const vg_plan* const* plans, const void* const* f, void* const* phi,
                        void* workspace, hipStream_t stream) {
    std::lock_guard<std::mutex> lk(g_batch_mutex);
    int dev = 0;
    hipError_t he = hipGetDevice(&dev);
    if (he != hipSuccess) return from_hip(he, "hipGetDevice");
    for (int i = 0; i < count; ++i)
        if (plans[i]->device != dev)
            return fail(VG_ERR_INVALID_ARG, "every plan of a batch must live on the current device");
    hipStreamCaptureStatus cst = hipStreamCaptureStatusNone;
    he = hipStreamIsCapturing(stream, &cst);
    if (he != hipSuccess) return from_hip(he, "hipStreamIsCapturing");
    const bool capturing = cst != hipStreamCaptureStatusNone;

    const size_t need = batched_workspace_size(count, plans);
    void* ws = workspace;
    if (!ws) {
        if (!g_batch_ws || g_batch_ws->bytes < need) {
            if (capturing) return fail(VG_ERR_NOT_CAPTURABLE, "batched call under capture needs a workspace allocation");
            // unpinned entries on the old buffer go; pinned ones keep it alive
            if (g_batch_ws) {
                DevBlock* old = g_batch_ws.get();
                g_entries.evict_if([&](const BatchEntry& x) { return x.ws_hold.get() == old; }, sync_device);
                sync_device();
            }
            auto blk = std::make_shared<DevBlock>();
            he = dev_malloc(&blk->p, need);
            if (he != hipSuccess) return from_hip(he, "batched workspace");
            blk->bytes = need;
            g_batch_ws = blk;
        }
        ws = g_batch_ws->p;
    }

    BatchEntry* e = g_entries.find(
        [&](const BatchEntry& x) { return same_key(x, count, plans, f, phi, ws, dev); });
    if (!e) {
        if (capturing)
            return fail(VG_ERR_NOT_CAPTURABLE,
                        "first batched call with these plans and arrays must run outside stream capture");
        g_entries.trim(kMaxEntries - 1, sync_device);
        auto ne = std::make_unique<BatchEntry>();
        ne->plans.assign(plans, plans + count);
        ne->f.assign(f, f + count);
        ne->phi.assign(phi, phi + count);
        ne->ws = ws;
        if (!workspace) ne->ws_hold = g_batch_ws;
        ne->device = dev;
        ne->fp64 = plans[0]->fp64;
        vg_status st = build_entry(*ne);
        if (st != VG_OK) return st;
        if (env_flag("VG_BATCH_NO_GRAPH") || capture(*ne) != VG_OK) ne->graph_failed = true;
        e = g_entries.push_front(std::move(ne));
    }

    void* mark = capturing ? nullptr : profiler_mark(stream);
    if (capturing || !e->exec) {
        // the caller's own capture records the launches (which point into
        // this entry's descriptors and workspace: pin it); or no graph
        vg_status st = issue(*e, stream);
        if (st != VG_OK) return st;
        if (capturing) e->pinned = true;
    } else {
        he = hipGraphLaunch(e->exec, stream);
        if (he != hipSuccess) return from_hip(he, "graph launch");
    }
    if (mark) profiler_add("batched", mark, profiler_mark(stream), e->bytes);
    return VG_OK;
}

}  // namespace vg
