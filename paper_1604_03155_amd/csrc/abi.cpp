// C ABI entry points (include/vg.h): argument validation, status codes and
// thread-local error messages.  No C++ exception crosses this boundary.
#include <cmath>
#include <cstring>
#include <memory>
#include <new>

#include "plan.h"

namespace vg {
const char* last_error_cstr();
vg_status precompute(vg_plan* p, hipStream_t s, bool keep_T);
void finalize_bytes(vg_plan* p);
vg_status batched_apply(int count, const vg_plan* const* plans, const void* const* f, void* const* phi,
                        void* workspace, hipStream_t stream);
size_t batched_workspace_size(int count, const vg_plan* const* plans);
void batched_release_plan(const vg_plan* p);
size_t ls_workspace_size(const vg_plan* p);
vg_status ls_solve(const vg_plan* p, const void* q, const void* phi_in, void* sigma, double tol, int max_iter,
                   void* workspace, hipStream_t st, vg_ls_result* res);
int fft_max_lds_bytes_for_device();
}  // namespace vg

using namespace vg;

namespace {

void free_plan(vg_plan* p) {
    if (!p) return;
    batched_release_plan(p);
    for (auto& kv : p->twiddles)
        if (kv.second) (void)hipFree(kv.second);
    if (p->table) (void)hipFree(p->table);
    if (p->T_dev) (void)hipFree(p->T_dev);
    if (p->internal_ws) (void)hipFree(p->internal_ws);
    delete p;
}

vg_status check_device() {
    int n = 0;
    hipError_t e = hipGetDeviceCount(&n);
    if (e != hipSuccess || n <= 0) return fail(VG_ERR_NO_DEVICE, "no HIP device is visible");
    return VG_OK;
}

vg_status get_ws(const vg_plan* p, size_t need, void* given, void** out) {
    if (given) {
        *out = given;
        return VG_OK;
    }
    std::lock_guard<std::mutex> lk(p->ws_mutex);
    if (p->internal_ws_bytes < need) {
        if (p->internal_ws) (void)hipFree(p->internal_ws);
        p->internal_ws = nullptr;
        p->internal_ws_bytes = 0;
        hipError_t e = dev_malloc(&p->internal_ws, need);
        if (e != hipSuccess) return from_hip(e, "internal workspace");
        p->internal_ws_bytes = need;
    }
    *out = p->internal_ws;
    return VG_OK;
}

template <typename F>
vg_status guarded(F&& fn) {
    try {
        return fn();
    } catch (const std::bad_alloc&) {
        return fail(VG_ERR_OUT_OF_MEMORY, "host allocation failed");
    } catch (...) {
        return fail(VG_ERR_INTERNAL, "unexpected exception");
    }
}

}  // namespace

extern "C" {

vg_status vg_plan_create(int d, int N, vg_kernel kernel, double k, vg_plan** out) {
    return vg_plan_create_ex(d, N, kernel, k, nullptr, out);
}

vg_status vg_plan_create_ex(int d, int N, vg_kernel kernel, double k, const vg_plan_opts* opts, vg_plan** out) {
    return guarded([&]() -> vg_status {
        if (!out) return fail(VG_ERR_INVALID_ARG, "out is NULL");
        *out = nullptr;
        if (d != 2 && d != 3) return fail(VG_ERR_INVALID_ARG, "d must be 2 or 3");
        if (N < 4 || (N % 2)) return fail(VG_ERR_INVALID_ARG, "N must be even and at least 4");
        if (kernel != VG_LAPLACE && kernel != VG_HELMHOLTZ && kernel != VG_BIHARMONIC &&
            kernel != VG_LAPLACE_HELMHOLTZ && kernel != VG_CONVECTION)
            return fail(VG_ERR_INVALID_ARG, "unknown kernel");
        const bool helm = kernel == VG_HELMHOLTZ || kernel == VG_LAPLACE_HELMHOLTZ;
        const bool conv = kernel == VG_CONVECTION;
        if (helm && !(std::isfinite(k) && k > 0.0))
            return fail(VG_ERR_INVALID_ARG, "Helmholtz needs a finite k > 0");
        vg_plan_opts o;
        std::memset(&o, 0, sizeof(o));
        if (opts) o = *opts;
        double hvec[3] = {0.0, 0.0, 0.0}, hnorm = 0.0;
        if (conv) {
            bool finite = true;
            for (int i = 0; i < d; ++i) {
                hvec[i] = o.h[i];
                finite = finite && std::isfinite(hvec[i]);
                hnorm += hvec[i] * hvec[i];
            }
            hnorm = std::sqrt(hnorm);
            if (!finite || !(hnorm > 0.0) || !std::isfinite(hnorm))
                return fail(VG_ERR_INVALID_ARG, "the convection kernel needs a finite vector h with |h| > 0");
            if (d == 3 && N > 256) return fail(VG_ERR_UNSUPPORTED_SIZE, "3D convection plans need N <= 256");
            double tb = (o.precision == VG_FP64) ? 16.0 : 8.0;
            for (int i = 0; i < d; ++i) tb *= 2.0 * N;
            if (tb > 4294967296.0) return fail(VG_ERR_UNSUPPORTED_SIZE, "convection table above 4 GiB");
        }
        if (o.precision != VG_FP32 && o.precision != VG_FP64) return fail(VG_ERR_INVALID_ARG, "unknown precision");
        const double L = (o.L == 0.0) ? (d == 3 ? 1.8 : 1.5) : o.L;
        if (!(std::isfinite(L) && L > std::sqrt((double)d)))
            return fail(VG_ERR_INVALID_ARG, "L must exceed sqrt(d): the truncated kernel must cover the box");
        const int P = (o.P == 0) ? 4 : o.P;
        if (P < 2 || !((double)P > 1.0 + L) || P > 16)
            return fail(VG_ERR_INVALID_ARG, "P must satisfy 1 + L < P <= 16");
        if (o.tune < VG_TUNE_OFF || o.tune > VG_TUNE_FULL) return fail(VG_ERR_INVALID_ARG, "unknown tune mode");
        const std::vector<int> rad = radix_plan(2 * N);
        if (rad.empty() || (int)rad.size() > kMaxStages)
            return fail(VG_ERR_UNSUPPORTED_SIZE, "2N must factor into 2, 3, 5 and 7");
        if (d == 3 && (long long)2 * N * 2 * N > 0x7fffffffLL)
            return fail(VG_ERR_UNSUPPORTED_SIZE, "N too large for 3D");
        if (d == 2 && N > 16384) return fail(VG_ERR_UNSUPPORTED_SIZE, "N too large for 2D");
        vg_status st = check_device();
        if (st != VG_OK) return st;

        std::unique_ptr<vg_plan, void (*)(vg_plan*)> p(new vg_plan(), free_plan);
        p->d = d;
        p->N = N;
        p->kernel = kernel;
        p->k = helm ? k : (conv ? hnorm : 0.0);
        for (int i = 0; i < 3; ++i) p->h[i] = hvec[i];
        p->L = L;
        p->P = P;
        p->precision = o.precision;
        p->fp64 = o.precision == VG_FP64;
        p->tune = o.tune;
        p->radices = rad;
        p->table_complex = (helm || conv) ? 1 : 0;
        // long 2D column axes (four-step): launch-order tiles measured faster
        // than the XCD-grouped order (2D N = 1024 to 4096), and 512-byte row
        // padding up to 2N = 4096 (2D N = 2048: 0.222 -> 0.192 ms)
        if (d == 2 && 2 * N > 1024) {
            p->cfg.xcd_map = 0;
            if (2 * N <= 4096) p->cfg.pad_bytes = 512;
        }
        hipError_t he = hipGetDevice(&p->device);
        if (he != hipSuccess) return from_hip(he, "hipGetDevice");
        hipStream_t s = reinterpret_cast<hipStream_t>(o.stream);
        st = build_programs(p.get(), s);  // rejects sizes no pass kernel can run
        if (st != VG_OK) return st;
        st = precompute(p.get(), s, o.keep_operator != 0);
        if (st != VG_OK) return st;
        finalize_bytes(p.get());  // the fused passes' byte counts include the table, now sized
        st = autotune(p.get(), s);
        if (st != VG_OK) return st;
        *out = p.release();
        return VG_OK;
    });
}

void vg_plan_destroy(vg_plan* plan) { free_plan(plan); }

vg_status vg_plan_get_info(const vg_plan* p, vg_plan_info* info) {
    if (!p || !info) return fail(VG_ERR_INVALID_ARG, "NULL argument");
    info->d = p->d;
    info->N = p->N;
    info->kernel = p->kernel;
    info->precision = p->precision;
    info->k = p->k;
    info->L = p->L;
    info->P = p->P;
    info->precompute_ms = p->precompute_ms;
    info->table_bytes = p->table_bytes;
    info->workspace_bytes = p->apply_prog.ws_bytes;
    info->gradient_workspace_bytes = p->grad_prog.ws_bytes;
    info->tune = p->tune;
    info->tune_ms = p->tune_ms;
    info->tune_candidates = p->tune_candidates;
    info->pad_bytes = p->cfg.pad_bytes;
    info->xcd_map = p->cfg.xcd_map;
    info->four_step_L1 = p->cfg.fs_L1;
    info->generic_passes = p->cfg.generic;
    info->tune_cached = p->tune_cached;
    return VG_OK;
}

size_t vg_workspace_size(const vg_plan* p) { return p ? p->apply_prog.ws_bytes : 0; }
size_t vg_gradient_workspace_size(const vg_plan* p) { return p ? p->grad_prog.ws_bytes : 0; }

vg_status vg_apply(const vg_plan* p, const void* f, void* phi, void* workspace, void* stream) {
    return guarded([&]() -> vg_status {
        if (!p) return fail(VG_ERR_INVALID_ARG, "plan is NULL");
        if (!f || !phi) return fail(VG_ERR_INVALID_ARG, "f and phi must be device pointers");
        void* ws = nullptr;
        vg_status st = get_ws(p, p->apply_prog.ws_bytes, workspace, &ws);
        if (st != VG_OK) return st;
        return run_program(p, p->apply_prog, f, phi, nullptr, ws, reinterpret_cast<hipStream_t>(stream));
    });
}

vg_status vg_gradient(const vg_plan* p, const void* f, void* phi, void* grad, void* workspace, void* stream) {
    return guarded([&]() -> vg_status {
        if (!p) return fail(VG_ERR_INVALID_ARG, "plan is NULL");
        if (!f || !grad) return fail(VG_ERR_INVALID_ARG, "f and grad must be device pointers");
        if (p->grad_prog.steps.empty())
            return fail(VG_ERR_UNSUPPORTED_SIZE, "no gradient kernels for this size (a gradient pass exceeds the LDS)");
        void* ws = nullptr;
        vg_status st = get_ws(p, p->grad_prog.ws_bytes, workspace, &ws);
        if (st != VG_OK) return st;
        return run_program(p, p->grad_prog, f, phi, grad, ws, reinterpret_cast<hipStream_t>(stream));
    });
}

size_t vg_real_workspace_size(const vg_plan* p) { return p ? p->real_prog.ws_bytes : 0; }

vg_status vg_apply_real(const vg_plan* p, const void* f, void* phi, void* workspace, void* stream) {
    return guarded([&]() -> vg_status {
        if (!p) return fail(VG_ERR_INVALID_ARG, "plan is NULL");
        if (!f || !phi) return fail(VG_ERR_INVALID_ARG, "f and phi must be device pointers");
        if (p->table_complex)
            return fail(VG_ERR_INVALID_ARG, "real applies need a real kernel (VG_LAPLACE or VG_BIHARMONIC)");
        if (p->real_prog.steps.empty())
            return fail(VG_ERR_UNSUPPORTED_SIZE, "no real-data kernels for this N (needs specialised lengths N and 2N)");
        void* ws = nullptr;
        vg_status st = get_ws(p, p->real_prog.ws_bytes, workspace, &ws);
        if (st != VG_OK) return st;
        return run_program(p, p->real_prog, f, phi, nullptr, ws, reinterpret_cast<hipStream_t>(stream));
    });
}

size_t vg_batched_workspace_size(int count, const vg_plan* const* plans) {
    if (count <= 0 || !plans) return 0;
    return batched_workspace_size(count, plans);
}

vg_status vg_apply_batched(int count, const vg_plan* const* plans, const void* const* f, void* const* phi,
                           void* workspace, void* stream) {
    return guarded([&]() -> vg_status {
        if (count <= 0) return fail(VG_ERR_INVALID_ARG, "count must be positive");
        if (!plans || !f || !phi) return fail(VG_ERR_INVALID_ARG, "NULL array argument");
        for (int i = 0; i < count; ++i) {
            if (!plans[i] || !f[i] || !phi[i]) return fail(VG_ERR_INVALID_ARG, "NULL entry in a batch array");
            if (plans[i]->precision != plans[0]->precision)
                return fail(VG_ERR_INVALID_ARG, "all plans of a batch must share one precision");
        }
        return batched_apply(count, plans, f, phi, workspace, reinterpret_cast<hipStream_t>(stream));
    });
}

size_t vg_ls_workspace_size(const vg_plan* p) { return p ? ls_workspace_size(p) : 0; }

vg_status vg_ls_solve(const vg_plan* p, const void* q, const void* phi_in, void* sigma, double tol, int max_iter,
                      void* workspace, void* stream, vg_ls_result* result) {
    return guarded([&]() -> vg_status {
        if (!p || !q || !phi_in || !sigma) return fail(VG_ERR_INVALID_ARG, "NULL argument");
        if (p->kernel != VG_HELMHOLTZ) return fail(VG_ERR_INVALID_ARG, "the Lippmann-Schwinger solve needs a Helmholtz plan");
        if (!(tol > 0.0) || max_iter < 1) return fail(VG_ERR_INVALID_ARG, "tol must be positive and max_iter >= 1");
        vg_ls_result local;
        vg_status st = ls_solve(p, q, phi_in, sigma, tol, max_iter, workspace, reinterpret_cast<hipStream_t>(stream),
                                result ? result : &local);
        return st;
    });
}

vg_status vg_plan_kernel_hat(const vg_plan* p, double* host_out) {
    return guarded([&]() -> vg_status {
        if (!p || !host_out) return fail(VG_ERR_INVALID_ARG, "NULL argument");
        long long n = 1;
        for (int i = 0; i < p->d; ++i) n *= (p->kernel == VG_CONVECTION ? 2 * p->N : p->N + 1);
        std::vector<unsigned char> h(p->table_bytes);
        hipError_t e = hipMemcpy(h.data(), p->table, p->table_bytes, hipMemcpyDeviceToHost);
        if (e != hipSuccess) return from_hip(e, "table download");
        double sc = 1.0;
        for (int i = 0; i < p->d; ++i) sc *= 2.0 * p->N;
        // 3D octant rows are padded to tab_pitch entries
        const long long row = p->kernel == VG_CONVECTION ? 2LL * p->N : p->N + 1;
        const long long pitch = p->kernel == VG_CONVECTION ? row : p->tab_pitch;
        for (long long i = 0; i < n; ++i) {
            const long long src = (i / row) * pitch + i % row;
            double re = 0, im = 0;
            if (p->fp64) {
                const double* q = reinterpret_cast<const double*>(h.data());
                re = p->table_complex ? q[2 * src] : q[src];
                im = p->table_complex ? q[2 * src + 1] : 0.0;
            } else {
                const float* q = reinterpret_cast<const float*>(h.data());
                re = p->table_complex ? q[2 * src] : q[src];
                im = p->table_complex ? q[2 * src + 1] : 0.0;
            }
            host_out[2 * i] = re * sc;
            host_out[2 * i + 1] = im * sc;
        }
        return VG_OK;
    });
}

vg_status vg_plan_operator_entries(const vg_plan* p, double* host_out) {
    if (!p || !host_out) return fail(VG_ERR_INVALID_ARG, "NULL argument");
    if (!p->T_dev) return fail(VG_ERR_INVALID_ARG, "plan was created without keep_operator");
    long long n = 1;
    for (int i = 0; i < p->d; ++i) n *= (p->kernel == VG_CONVECTION ? 2 * p->N - 1 : p->N);
    return from_hip(hipMemcpy(host_out, p->T_dev, (size_t)n * 16, hipMemcpyDeviceToHost), "operator download");
}

const char* vg_status_string(vg_status s) {
    switch (s) {
        case VG_OK: return "VG_OK";
        case VG_ERR_INVALID_ARG: return "VG_ERR_INVALID_ARG";
        case VG_ERR_UNSUPPORTED_SIZE: return "VG_ERR_UNSUPPORTED_SIZE";
        case VG_ERR_OUT_OF_MEMORY: return "VG_ERR_OUT_OF_MEMORY";
        case VG_ERR_NO_DEVICE: return "VG_ERR_NO_DEVICE";
        case VG_ERR_DEVICE: return "VG_ERR_DEVICE";
        case VG_ERR_NOT_CAPTURABLE: return "VG_ERR_NOT_CAPTURABLE";
        case VG_ERR_INTERNAL: return "VG_ERR_INTERNAL";
    }
    return "VG_ERR_UNKNOWN";
}

const char* vg_last_error(void) { return last_error_cstr(); }

}  // extern "C"
