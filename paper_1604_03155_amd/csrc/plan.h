// Host-side plan object of the volume-potential library (internal).
#pragma once

#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "common.h"
#include "../../include/vg.h"

namespace vg {

// One launch of a pass: descriptor plus how to launch it.  Buffer fields of
// the descriptor are filled in at apply time from symbolic buffer ids.
enum BufId : int {
    BUF_F = 0,     // caller's density
    BUF_PHI = 1,   // caller's potential (may be null for gradient-only)
    BUF_GRAD0 = 2, // caller's gradient component 0 (then 1, 2)
    BUF_WS0 = 8,   // workspace sub-buffers 0..7
    BUF_NONE = 63
};

struct PassStep {
    PassDesc desc;   // in/out/out2 filled at apply time
    int mode;        // MODE_ROW / MODE_COL
    int kind;        // PassKind (or 100 + KIND_INV for derivative-only inverse)
    int in_buf, out_buf, out2_buf;
    const char* name;
    double bytes;    // algorithmic HBM bytes of one launch (reads + writes)
};

struct Program {
    std::vector<PassStep> steps;
    std::vector<size_t> ws_offsets;  // byte offsets of workspace sub-buffers
    size_t ws_bytes = 0;
};


}  // namespace vg

namespace vg {
// Layout and kernel choices of a plan's programs (the autotuner's search
// space).  pad_bytes: extra pitch of the 2N x 2N planes (3D) / 2N rows (2D)
// of the intermediates; xcd_map: XCD-aware tile order in the specialised
// kernels; fs_L1: first factor of the four-step split of long 2D columns (0:
// the default choice); generic: run every pass on the generic kernel.
struct LayoutConfig {
    int pad_bytes = 256;
    int xcd_map = 1;
    int fs_L1 = 0;
    int generic = 0;
};
}  // namespace vg

struct vg_plan {
    int d = 0, N = 0, kernel = 0, precision = 0, P = 4, tune = 0;
    vg::LayoutConfig cfg;
    double tune_ms = 0.0;     // wall time of the autotuner
    int tune_candidates = 0;  // configurations timed
    int tune_cached = 0;      // 1: the layout came from the persistent tune cache
    double k = 0.0, L = 0.0;
    double h[3] = {0.0, 0.0, 0.0};  // convection vector (VG_CONVECTION)
    int device = 0;
    bool fp64 = false;
    std::vector<int> radices;     // Stockham radix plan of length 2N
    std::map<int, void*> twiddles; // device twiddle tables e^{-2 pi i t / L} per length L
    void* table = nullptr;        // device, (N+1)^d Khat octant / (2N)^d
    size_t table_bytes = 0;       // allocated bytes (padding and boundary block included)
    size_t table_alg_bytes = 0;   // bytes of the octant itself, (N+1)^d entries (read once per fused pass)
    int tab_pitch = 0;            // see PassDesc::tab_pitch
    unsigned tab_bnd = 0;         // see PassDesc::tab_bnd
    int table_complex = 0;
    void* T_dev = nullptr;        // device, N^d complex128 (keep_operator)
    double precompute_ms = 0.0;
    vg::Program apply_prog, grad_prog;
    vg::Program real_prog;   // real densities with a real kernel (Laplace, biharmonic); empty if unsupported
    // internal workspace for calls with workspace == NULL
    mutable std::mutex ws_mutex;
    mutable void* internal_ws = nullptr;
    mutable size_t internal_ws_bytes = 0;
};

namespace vg {

// Set the calling thread's error message; returns `st`.
vg_status fail(vg_status st, const std::string& msg);
vg_status from_hip(hipError_t e, const char* what);

// Radix plan for length L with radices in {8, 4, 2, 3, 5, 7}; empty if L has
// another prime factor.
std::vector<int> radix_plan(int L);

// Build the apply / gradient programs for a plan with its layout config
// p->cfg (allocates the twiddle tables they need); VG_ERR_UNSUPPORTED_SIZE if
// some pass cannot run.
vg_status build_programs(vg_plan* p, hipStream_t s);

// Autotuner (tune.cpp): with p->tune != VG_TUNE_OFF, time the apply program
// under candidate layout configs and keep the fastest (programs rebuilt).
vg_status autotune(vg_plan* p, hipStream_t s);

// Four-step splits L = L1 * L2 of a long 2D column axis usable by the plan
// (L1 even, both factors with radix plans), nearest to sqrt(L) first, those
// with specialised kernels for both factors before the others.
std::vector<int> four_step_splits(int L, bool fp64);

// A program step with its buffers bound to device addresses.
struct BoundStep {
    PassDesc desc;
    int mode, kind;
    const char* name;
    double bytes;
};
BoundStep bind_step(const vg_plan* p, const Program& prog, const PassStep& st, const void* f, void* phi, void* grad,
                    void* ws);
std::vector<BoundStep> bind_program(const vg_plan* p, const Program& prog, const void* f, void* phi, void* grad,
                                    void* ws);

// Run a program: bind buffers and launch every step on `stream`.
vg_status run_program(const vg_plan* p, const Program& prog, const void* f, void* phi, void* grad,
                      void* ws, hipStream_t stream);
// The same launches without host containers or profiler events.
vg_status run_program_noalloc(const vg_plan* p, const Program& prog, const void* f, void* phi, void* grad,
                              void* ws, hipStream_t stream);


// Pass profiler hooks (profiler.cpp).
int profiler_mode();  // 0 off, 1 every pass, 2 the pass with the most bytes
void* profiler_mark(hipStream_t s);
void profiler_add(const char* name, void* a, void* b, double bytes);

// Device allocation with the test hook VG_TEST_FAIL_ALLOC=n (the n-th
// allocation made through this function fails).
hipError_t dev_malloc(void** ptr, size_t bytes);

}  // namespace vg
