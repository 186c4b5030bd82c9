// Lippmann-Schwinger solve (Section 5.3) by Bi-CGStab with the plan's
// convolution as the matrix-vector product.
//
// The dual Lippmann-Schwinger equation for the density sigma of the scattered
// field phi_s = g_k * sigma is
//     -sigma + k^2 q (g_k * sigma) = -k^2 q phi_in,
// q the contrast (compactly supported in the box), phi_in the incident field.
// Each Bi-CGStab iteration applies the operator twice; every step runs on the
// device (the apply passes plus the fused vector kernels of blas1.hip); the
// host only combines the five dot products of an iteration into the scalars
// alpha, beta, omega and checks convergence.
#include <cmath>
#include <complex>

#include "blas1.h"
#include "plan.h"

namespace vg {

namespace {
size_t align256(size_t x) { return (x + 255) & ~size_t(255); }

using cd = std::complex<double>;

struct LsLayout {
    size_t apply_ws, vec, part, out, total;
};

LsLayout ls_layout(const vg_plan* p) {
    long long V = 1;
    for (int i = 0; i < p->d; ++i) V *= p->N;
    LsLayout l;
    l.apply_ws = align256(p->apply_prog.ws_bytes);
    l.vec = align256((size_t)V * (p->fp64 ? 16 : 8));
    l.part = align256((size_t)kDotBlocks * 6 * sizeof(double));
    l.out = align256(6 * sizeof(double));
    l.total = l.apply_ws + 6 * l.vec + l.part + l.out;
    return l;
}

template <typename R>
vg_status solve(const vg_plan* p, const void* q, const void* phi_in, void* x, double tol, int max_iter,
                unsigned char* ws, hipStream_t st, vg_ls_result* res) {
    const LsLayout lay = ls_layout(p);
    long long n = 1;
    for (int i = 0; i < p->d; ++i) n *= p->N;
    void* aws = ws;
    unsigned char* vb = ws + lay.apply_ws;
    void* r = vb;
    void* rh = vb + lay.vec;
    void* pv = vb + 2 * lay.vec;
    void* v = vb + 3 * lay.vec;
    void* s = vb + 4 * lay.vec;
    void* t = vb + 5 * lay.vec;
    double* part = reinterpret_cast<double*>(vb + 6 * lay.vec);
    double* dout = reinterpret_cast<double*>(vb + 6 * lay.vec + lay.part);
    const double k2 = p->k * p->k;
    const size_t vbytes = (size_t)n * sizeof(cplx<R>);
    hipError_t e;
    auto chk = [&](hipError_t he, const char* what) -> vg_status { return he == hipSuccess ? VG_OK : from_hip(he, what); };
    auto matvec = [&](const void* in, void* out) -> vg_status {
        vg_status sv = run_program(p, p->apply_prog, in, out, nullptr, aws, st);
        if (sv != VG_OK) return sv;
        return chk(ls_post<R>(in, q, out, k2, n, st), "operator epilogue");
    };
    // host values of up to three dot products
    cd hv[3];
    auto dot = [&](int count, const void* a0, const void* b0, const void* a1, const void* b1, const void* a2,
                   const void* b2) -> vg_status {
        DotArgs<R> da;
        da.a[0] = (const cplx<R>*)a0;
        da.b[0] = (const cplx<R>*)b0;
        da.a[1] = (const cplx<R>*)a1;
        da.b[1] = (const cplx<R>*)b1;
        da.a[2] = (const cplx<R>*)a2;
        da.b[2] = (const cplx<R>*)b2;
        da.count = count;
        vg_status sv = chk(dots<R>(da, part, dout, n, st), "dot products");
        if (sv != VG_OK) return sv;
        double h[6];
        sv = chk(hipMemcpyAsync(h, dout, sizeof(h), hipMemcpyDeviceToHost, st), "dot copy");
        if (sv != VG_OK) return sv;
        sv = chk(hipStreamSynchronize(st), "dot sync");
        if (sv != VG_OK) return sv;
        for (int j = 0; j < 3; ++j) hv[j] = cd(h[2 * j], h[2 * j + 1]);
        return VG_OK;
    };
    res->iterations = 0;
    res->matvecs = 0;
    res->converged = 0;
    res->residual = 0.0;
    // x = 0, r = b = -k^2 q phi_in, rhat = r
    if ((e = hipMemsetAsync(x, 0, vbytes, st)) != hipSuccess) return from_hip(e, "solution init");
    vg_status sv = chk(ls_rhs<R>(q, phi_in, r, k2, n, st), "right-hand side");
    if (sv != VG_OK) return sv;
    if ((e = hipMemcpyAsync(rh, r, vbytes, hipMemcpyDeviceToDevice, st)) != hipSuccess) return from_hip(e, "copy");
    if ((sv = dot(1, r, r, nullptr, nullptr, nullptr, nullptr)) != VG_OK) return sv;
    const double bnorm = std::sqrt(hv[0].real());
    if (bnorm == 0.0) {
        res->converged = 1;
        return VG_OK;
    }
    cd rho = hv[0], rho_old(1.0, 0.0), alpha(1.0, 0.0), omega(1.0, 0.0);
    double rnorm = bnorm;
    for (int it = 1; it <= max_iter; ++it) {
        if (std::abs(rho) == 0.0) break;  // breakdown: (rhat, r) = 0
        if (it == 1) {
            if ((e = hipMemcpyAsync(pv, r, vbytes, hipMemcpyDeviceToDevice, st)) != hipSuccess) return from_hip(e, "copy");
        } else {
            const cd beta = (rho / rho_old) * (alpha / omega);
            if ((sv = chk(p_update<R>(r, v, pv, Cd{beta.real(), beta.imag()}, Cd{omega.real(), omega.imag()}, n, st),
                          "p update")) != VG_OK)
                return sv;
        }
        if ((sv = matvec(pv, v)) != VG_OK) return sv;
        ++res->matvecs;
        if ((sv = dot(1, rh, v, nullptr, nullptr, nullptr, nullptr)) != VG_OK) return sv;
        if (std::abs(hv[0]) == 0.0) break;
        alpha = rho / hv[0];
        // s = r - alpha v
        const cd ma = -alpha;
        if ((sv = chk(axpy<R>(r, Cd{ma.real(), ma.imag()}, v, s, n, st), "s update")) != VG_OK) return sv;
        if ((sv = dot(1, s, s, nullptr, nullptr, nullptr, nullptr)) != VG_OK) return sv;
        const double snorm = std::sqrt(hv[0].real());
        res->iterations = it;
        if (snorm <= tol * bnorm) {
            // converged at the half step: x += alpha p, r = s
            if ((sv = chk(axpy<R>(x, Cd{alpha.real(), alpha.imag()}, pv, x, n, st), "x update")) != VG_OK) return sv;
            rnorm = snorm;
            res->converged = 1;
            break;
        }
        if ((sv = matvec(s, t)) != VG_OK) return sv;
        ++res->matvecs;
        if ((sv = dot(2, t, s, t, t, nullptr, nullptr)) != VG_OK) return sv;
        if (hv[1].real() == 0.0) break;
        omega = hv[0] / hv[1].real();
        if ((sv = chk(xr_update<R>(x, r, pv, s, t, Cd{alpha.real(), alpha.imag()}, Cd{omega.real(), omega.imag()}, n, st),
                      "x, r update")) != VG_OK)
            return sv;
        if ((sv = dot(2, rh, r, r, r, nullptr, nullptr)) != VG_OK) return sv;
        rho_old = rho;
        rho = hv[0];
        rnorm = std::sqrt(hv[1].real());
        if (rnorm <= tol * bnorm) {
            res->converged = 1;
            break;
        }
        if (std::abs(omega) == 0.0) break;
    }
    res->residual = rnorm / bnorm;
    return VG_OK;
}
}  // namespace

size_t ls_workspace_size(const vg_plan* p) { return ls_layout(p).total; }

vg_status ls_solve(const vg_plan* p, const void* q, const void* phi_in, void* sigma, double tol, int max_iter,
                   void* workspace, hipStream_t st, vg_ls_result* res) {
    const LsLayout lay = ls_layout(p);
    void* ws = workspace;
    void* owned = nullptr;
    if (!ws) {
        hipError_t e = dev_malloc(&owned, lay.total);
        if (e != hipSuccess) return from_hip(e, "solver workspace");
        ws = owned;
    }
    vg_status sv = p->fp64 ? solve<double>(p, q, phi_in, sigma, tol, max_iter, static_cast<unsigned char*>(ws), st, res)
                           : solve<float>(p, q, phi_in, sigma, tol, max_iter, static_cast<unsigned char*>(ws), st, res);
    if (owned) {
        (void)hipStreamSynchronize(st);
        (void)hipFree(owned);
    }
    return sv;
}

}  // namespace vg
