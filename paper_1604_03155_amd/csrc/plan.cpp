// Plan creation: validation, FP64 device precompute of the kernel table
// (Sections 2 and 4), twiddles, and the pass programs of apply and gradient.
#include "plan.h"

#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <complex>

namespace vg {

namespace {
thread_local std::string g_last_error;
std::atomic<long> g_alloc_count{0};

size_t align256(size_t x) { return (x + 255) & ~size_t(255); }
}  // namespace

vg_status fail(vg_status st, const std::string& msg) {
    g_last_error = msg;
    return st;
}

const char* last_error_cstr() { return g_last_error.c_str(); }

vg_status from_hip(hipError_t e, const char* what) {
    if (e == hipSuccess) return VG_OK;
    if (e == hipErrorOutOfMemory) return fail(VG_ERR_OUT_OF_MEMORY, std::string(what) + ": out of device memory");
    if (e == hipErrorStreamCaptureUnsupported || e == hipErrorStreamCaptureInvalidated)
        return fail(VG_ERR_NOT_CAPTURABLE, std::string(what) + ": " + hipGetErrorString(e));
    return fail(VG_ERR_DEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

hipError_t dev_malloc(void** ptr, size_t bytes) {
    *ptr = nullptr;
    const char* hook = std::getenv("VG_TEST_FAIL_ALLOC");
    const long n = ++g_alloc_count;
    if (hook && *hook) {
        const long target = std::atol(hook);
        if (target > 0 && n == target) return hipErrorOutOfMemory;
    }
    if (bytes == 0) bytes = 256;
    return hipMalloc(ptr, bytes);
}

std::vector<int> radix_plan(int L) {
    std::vector<int> r;
    if (L < 2) return r;
    int x = L, a = 0;
    while (x % 2 == 0) {
        x /= 2;
        ++a;
    }
    std::vector<int> odd;
    for (int p : {3, 5, 7}) {
        while (x % p == 0) {
            x /= p;
            odd.push_back(p);
        }
    }
    if (x != 1) return {};
    while (a >= 3) {
        r.push_back(8);
        a -= 3;
    }
    if (a == 2) r.push_back(4);
    if (a == 1) r.push_back(2);
    for (int p : odd) r.push_back(p);
    return r;
}

namespace {

// ----------------------------------------------------------- host tables --
// cos / sin of 2 pi t / n, evaluated in long double from the exact integer
// ratio and rounded once to the target precision.
long double twopi_frac_cos(long long t, long long n) {
    const long double pi = 3.141592653589793238462643383279502884L;
    return cosl(2.0L * pi * (long double)(t % n) / (long double)n);
}
long double twopi_frac_sin(long long t, long long n) {
    const long double pi = 3.141592653589793238462643383279502884L;
    return sinl(2.0L * pi * (long double)(t % n) / (long double)n);
}

// C[n][m] = w_m cos(2 pi n m / period) * scale, n in [0, nout), m in [0, kin)
std::vector<double> cos_matrix(int nout, int kin, long long period, const std::vector<double>& w, double scale) {
    std::vector<long double> ct((size_t)period);
    for (long long t = 0; t < period; ++t) ct[(size_t)t] = twopi_frac_cos(t, period);
    std::vector<double> c((size_t)nout * kin);
    for (int n = 0; n < nout; ++n)
        for (int m = 0; m < kin; ++m)
            c[(size_t)n * kin + m] = (double)(ct[(size_t)(((long long)n * m) % period)] * (long double)w[m] * scale);
    return c;
}

double factorial(int n) {
    double f = 1.0;
    for (int i = 2; i <= n; ++i) f *= i;
    return f;
}

double besselj_int(int nu, double x) {
    if (nu < 0) return ((-nu) % 2 ? -1.0 : 1.0) * std::cyl_bessel_j((double)(-nu), x);
    return std::cyl_bessel_j((double)nu, x);
}

// m-th derivative of J_nu: 2^-m sum_j (-1)^j C(m, j) J_{nu-m+2j}
double besselj_deriv(int nu, int m, double x) {
    double acc = 0.0, binom = 1.0;
    for (int j = 0; j <= m; ++j) {
        acc += ((j % 2) ? -1.0 : 1.0) * binom * besselj_int(nu - m + 2 * j, x);
        binom = binom * (m - j) / (j + 1);
    }
    return std::ldexp(acc, -m);
}

void fill_greens_params(const vg_plan* p, GreensParams& g) {
    std::memset(&g, 0, sizeof(g));
    g.d = p->d;
    g.kernel = p->kernel;
    g.k = p->k;
    g.L = p->L;
    g.ds = 2.0 * M_PI / p->P;
    const double L = p->L, k = p->k;
    const bool conv = p->kernel == VG_CONVECTION;
    const bool helm = p->kernel == VG_HELMHOLTZ || p->kernel == VG_LAPLACE_HELMHOLTZ || conv;
    if (conv) {
        // evaluated as the Helmholtz transform with k = |h| at |s - h|
        g.kernel = VG_HELMHOLTZ;
        g.full = 1;
        g.M = p->P * p->N;
        for (int i = 0; i < 3; ++i) g.h[i] = p->h[i];
    }
    if (helm && p->d == 3) {
        // power series of (1/s) int_0^L sin(sr) e^{ikr} dr in x^2 = (sL)^2:
        // a_j = L^2 (-1)^j/(2j+1)! sum_p (ikL)^p / (p! (2j+2+p))
        g.ntaylor = 10;
        for (int j = 0; j < 10; ++j) {
            std::complex<double> inner = 0.0, ikl_p = 1.0;
            for (int q = 0; q < 40; ++q) {
                inner += ikl_p / (factorial(q) * (2 * j + 2 + q));
                ikl_p *= std::complex<double>(0.0, k * L);
            }
            const std::complex<double> a = L * L * ((j % 2) ? -1.0 : 1.0) / factorial(2 * j + 1) * inner;
            g.taylor_r[j] = a.real();
            g.taylor_i[j] = a.imag();
        }
    }
    if (helm && p->d == 2) {
        const double x = k * L;
        const std::complex<double> H0(std::cyl_bessel_j(0.0, x), std::cyl_neumann(0.0, x));
        const std::complex<double> H1(std::cyl_bessel_j(1.0, x), std::cyl_neumann(1.0, x));
        g.H0r = H0.real();
        g.H0i = H0.imag();
        g.H1r = H1.real();
        g.H1i = H1.imag();
        // Taylor coefficients of N(s)/(s - k) about s = k, N the numerator of
        // Table 2's transform: c_{n-1} = N^(n)(k)/n!, with
        // u = s J1(Ls): u^(n) = k L^n J1^(n) + n L^(n-1) J1^(n-1); v = J0(Ls): v^(n) = L^n J0^(n).
        // 24 terms over |s - k| < 1: the printed quotient loses about
        // eps k / |s - k| to cancellation, which the wide window keeps near
        // 1e-14 relative up to k ~ 1000 (measured against 40-digit values)
        g.ntaylor = 24;
        for (int n = 1; n <= 24; ++n) {
            const double un = k * std::pow(L, n) * besselj_deriv(1, n, x) + n * std::pow(L, n - 1) * besselj_deriv(1, n - 1, x);
            const double vn = std::pow(L, n) * besselj_deriv(0, n, x);
            const std::complex<double> Nn = std::complex<double>(0.0, 0.5 * M_PI * L) * (H0 * un - k * H1 * vn);
            const std::complex<double> c = Nn / factorial(n);
            g.taylor_r[n - 1] = c.real();
            g.taylor_i[n - 1] = c.imag();
        }
        g.window = 1.0;
    }
}

// The precompute's timing events, released on every return path.
struct EventPair {
    hipEvent_t a = nullptr, b = nullptr;
    ~EventPair() {
        if (a) (void)hipEventDestroy(a);
        if (b) (void)hipEventDestroy(b);
    }
};

struct DevBuf {
    void* p = nullptr;
    ~DevBuf() {
        if (p) (void)hipFree(p);
    }
    hipError_t alloc(size_t bytes) { return dev_malloc(&p, bytes); }
    template <typename T>
    T* as() const { return reinterpret_cast<T*>(p); }
};

vg_status upload(DevBuf& b, const std::vector<double>& h, hipStream_t s) {
    hipError_t e = b.alloc(h.size() * sizeof(double));
    if (e != hipSuccess) return from_hip(e, "precompute table allocation");
    e = hipMemcpyAsync(b.p, h.data(), h.size() * sizeof(double), hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    return from_hip(e, "precompute table upload");
}

}  // namespace

// Convection kernel (Tables 1-2, last row): G_h(s) = G_{|h|}(|s - h|) has no
// per-axis symmetry, so T lives on all offsets |n_j| <= N-1 (2N-1 per axis)
// and Khat on the full (2N)^d box.  Each axis is a complex DFT contraction,
// done as a cosine and a sine contraction combined as a + sign i b.
vg_status precompute_full(vg_plan* p, hipStream_t s, bool keep_T) {
    const int d = p->d, N = p->N;
    const long long M = (long long)p->P * N, NT = 2LL * N - 1, L = 2LL * N;
    auto dft = [&](long long rows_out, long long cols_in, bool lattice, bool sine) {
        // lattice: [nn][m], angle 2 pi m_s n / M, scale 1/M (T);
        // otherwise [k][nn], angle 2 pi k n / (2N), scale 1/(2N) (Khat)
        std::vector<double> c((size_t)(rows_out * cols_in));
        for (long long r = 0; r < rows_out; ++r)
            for (long long q = 0; q < cols_in; ++q) {
                long long t, period;
                double scale;
                if (lattice) {
                    const long long ms = q < M / 2 ? q : q - M;
                    t = ms * (r - (N - 1));
                    period = M;
                    scale = 1.0 / (double)M;
                } else {
                    t = r * (q - (N - 1));
                    period = L;
                    scale = 1.0 / (double)L;
                }
                t %= period;
                if (t < 0) t += period;
                const long double v = sine ? twopi_frac_sin(t, period) : twopi_frac_cos(t, period);
                c[(size_t)(r * cols_in + q)] = (double)(v * (long double)scale);
            }
        return c;
    };
    DevBuf dCl, dSl, dCk, dSk;
    vg_status st = upload(dCl, dft(NT, M, true, false), s);
    if (st == VG_OK) st = upload(dSl, dft(NT, M, true, true), s);
    if (st == VG_OK) st = upload(dCk, dft(L, NT, false, false), s);
    if (st == VG_OK) st = upload(dSk, dft(L, NT, false, true), s);
    if (st != VG_OK) return st;
    GreensParams g;
    fill_greens_params(p, g);
    EventPair ev;
    hipError_t he = hipEventCreate(&ev.a);
    if (he == hipSuccess) he = hipEventCreate(&ev.b);
    if (he != hipSuccess) return from_hip(he, "hipEventCreate");
    hipEvent_t e0 = ev.a, e1 = ev.b;
    (void)hipEventRecord(e0, s);
    auto chk = [&](hipError_t e, const char* what) -> vg_status { return from_hip(e, what); };
    // one complex contraction of the middle index of X[O][Min][I]: Y = X C + sign i X S
    DevBuf tmp;
    auto contract = [&](const DevBuf& in, DevBuf& out, const DevBuf& C, const DevBuf& S, long long O, int Min, int Nout,
                        long long I, int sign) -> vg_status {
        const size_t n = (size_t)(O * Nout * I);
        hipError_t e = out.alloc(n * 16);
        if (e == hipSuccess && !tmp.p) e = tmp.alloc(n * 16);
        if (e != hipSuccess) return chk(e, "precompute buffer");
        if ((e = launch_cos_contract(in.as<c64>(), out.as<c64>(), C.as<double>(), O, Min, Nout, I, s)) != hipSuccess)
            return chk(e, "contraction");
        if ((e = launch_cos_contract(in.as<c64>(), tmp.as<c64>(), S.as<double>(), O, Min, Nout, I, s)) != hipSuccess)
            return chk(e, "contraction");
        if ((e = launch_combine(out.as<c64>(), tmp.as<c64>(), out.as<c64>(), (long long)n, sign, s)) != hipSuccess)
            return chk(e, "combine");
        if ((e = hipStreamSynchronize(s)) != hipSuccess) return chk(e, "precompute");
        (void)hipFree(tmp.p);
        tmp.p = nullptr;
        return VG_OK;
    };
    DevBuf X1, X2, T, K1, K2, K;
    {
        long long rows = 1;
        for (int i = 0; i < d - 1; ++i) rows *= M;
        const size_t n = (size_t)(rows * NT);
        if ((he = X1.alloc(n * 16)) != hipSuccess || (he = tmp.alloc(n * 16)) != hipSuccess) return chk(he, "precompute buffer");
        if ((he = launch_greens_contract_full(g, (int)NT, dCl.as<double>(), X1.as<c64>(), s)) != hipSuccess) return chk(he, "kernel spectrum");
        if ((he = launch_greens_contract_full(g, (int)NT, dSl.as<double>(), tmp.as<c64>(), s)) != hipSuccess) return chk(he, "kernel spectrum");
        if ((he = launch_combine(X1.as<c64>(), tmp.as<c64>(), X1.as<c64>(), (long long)n, +1, s)) != hipSuccess) return chk(he, "combine");
        if ((he = hipStreamSynchronize(s)) != hipSuccess) return chk(he, "precompute");
        (void)hipFree(tmp.p);
        tmp.p = nullptr;
    }
    DevBuf* Tb;
    if (d == 3) {
        if ((st = contract(X1, X2, dCl, dSl, M, (int)M, (int)NT, NT, +1)) != VG_OK) return st;
        (void)hipFree(X1.p);
        X1.p = nullptr;
        if ((st = contract(X2, T, dCl, dSl, 1, (int)M, (int)NT, NT * NT, +1)) != VG_OK) return st;
        (void)hipFree(X2.p);
        X2.p = nullptr;
        if ((st = contract(T, K1, dCk, dSk, 1, (int)NT, (int)L, NT * NT, -1)) != VG_OK) return st;
        if ((st = contract(K1, K2, dCk, dSk, L, (int)NT, (int)L, NT, -1)) != VG_OK) return st;
        (void)hipFree(K1.p);
        K1.p = nullptr;
        if ((st = contract(K2, K, dCk, dSk, L * L, (int)NT, (int)L, 1, -1)) != VG_OK) return st;
        Tb = &T;
    } else {
        if ((st = contract(X1, T, dCl, dSl, 1, (int)M, (int)NT, NT, +1)) != VG_OK) return st;
        (void)hipFree(X1.p);
        X1.p = nullptr;
        if ((st = contract(T, K1, dCk, dSk, 1, (int)NT, (int)L, NT, -1)) != VG_OK) return st;
        if ((st = contract(K1, K, dCk, dSk, L, (int)NT, (int)L, 1, -1)) != VG_OK) return st;
        Tb = &T;
    }
    long long nK = 1;
    for (int i = 0; i < d; ++i) nK *= L;
    p->table_complex = 1;
    const size_t esz = p->fp64 ? 16 : 8;
    p->table_bytes = (size_t)nK * esz;
    p->table_alg_bytes = p->table_bytes;
    p->tab_pitch = (int)L;
    p->tab_bnd = 0;
    if ((he = dev_malloc(&p->table, p->table_bytes)) != hipSuccess) return chk(he, "kernel table");
    if ((he = launch_round_table(K.as<c64>(), p->table, nK / L, (int)L, (int)L, p->fp64 ? 0 : 1, 1, 0, 0, 0, s)) !=
        hipSuccess)
        return chk(he, "table rounding");
    (void)hipEventRecord(e1, s);
    if ((he = hipStreamSynchronize(s)) != hipSuccess) return chk(he, "precompute");
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, e0, e1);
    p->precompute_ms = ms;
    if (keep_T) {
        p->T_dev = Tb->p;
        Tb->p = nullptr;
    }
    return VG_OK;
}

// FP64 precompute: kernel spectrum -> T (octant) -> Khat (octant) -> table.
vg_status precompute(vg_plan* p, hipStream_t s, bool keep_T) {
    if (p->kernel == VG_CONVECTION) return precompute_full(p, s, keep_T);
    const int d = p->d, N = p->N;
    const long long M = (long long)p->P * N;
    const int M2 = (int)(M / 2 + 1);
    std::vector<double> w(M2, 2.0);
    w[0] = 1.0;
    w[M2 - 1] = 1.0;
    const std::vector<double> Cm = cos_matrix(N, M2, M, w, 1.0 / (double)M);
    std::vector<double> v(N, 2.0);
    v[0] = 1.0;
    const std::vector<double> Dm = cos_matrix(N + 1, N, 2LL * N, v, 1.0 / (2.0 * N));

    DevBuf dC, dD;
    vg_status st = upload(dC, Cm, s);
    if (st != VG_OK) return st;
    st = upload(dD, Dm, s);
    if (st != VG_OK) return st;

    GreensParams g;
    fill_greens_params(p, g);

    EventPair ev;
    hipError_t he = hipEventCreate(&ev.a);
    if (he == hipSuccess) he = hipEventCreate(&ev.b);
    if (he != hipSuccess) return from_hip(he, "hipEventCreate");
    hipEvent_t e0 = ev.a, e1 = ev.b;
    (void)hipEventRecord(e0, s);

    const long long Nl = N, M2l = M2, N1 = N + 1;
    DevBuf X1, X2, T, Y1, Y2, K;
    auto chk = [&](hipError_t e, const char* what) -> vg_status { return from_hip(e, what); };
    if (d == 3) {
        if ((he = X1.alloc((size_t)M2l * M2l * Nl * 16)) != hipSuccess) return chk(he, "precompute buffer");
        if ((he = launch_greens_contract(g, M2, N, dC.as<double>(), X1.as<c64>(), s)) != hipSuccess) return chk(he, "kernel spectrum");
        if ((he = X2.alloc((size_t)M2l * Nl * Nl * 16)) != hipSuccess) return chk(he, "precompute buffer");
        if ((he = launch_cos_contract(X1.as<c64>(), X2.as<c64>(), dC.as<double>(), M2l, M2, N, Nl, s)) != hipSuccess) return chk(he, "T axis 2");
        (void)hipStreamSynchronize(s);
        (void)hipFree(X1.p);
        X1.p = nullptr;
        if ((he = T.alloc((size_t)Nl * Nl * Nl * 16)) != hipSuccess) return chk(he, "precompute buffer");
        if ((he = launch_cos_contract(X2.as<c64>(), T.as<c64>(), dC.as<double>(), 1, M2, N, Nl * Nl, s)) != hipSuccess) return chk(he, "T axis 1");
        (void)hipStreamSynchronize(s);
        (void)hipFree(X2.p);
        X2.p = nullptr;
        if ((he = Y1.alloc((size_t)N1 * Nl * Nl * 16)) != hipSuccess) return chk(he, "precompute buffer");
        if ((he = launch_cos_contract(T.as<c64>(), Y1.as<c64>(), dD.as<double>(), 1, N, N + 1, Nl * Nl, s)) != hipSuccess) return chk(he, "Khat axis 1");
        if ((he = Y2.alloc((size_t)N1 * N1 * Nl * 16)) != hipSuccess) return chk(he, "precompute buffer");
        if ((he = launch_cos_contract(Y1.as<c64>(), Y2.as<c64>(), dD.as<double>(), N1, N, N + 1, Nl, s)) != hipSuccess) return chk(he, "Khat axis 2");
        (void)hipStreamSynchronize(s);
        (void)hipFree(Y1.p);
        Y1.p = nullptr;
        if ((he = K.alloc((size_t)N1 * N1 * N1 * 16)) != hipSuccess) return chk(he, "precompute buffer");
        if ((he = launch_cos_contract(Y2.as<c64>(), K.as<c64>(), dD.as<double>(), N1 * N1, N, N + 1, 1, s)) != hipSuccess) return chk(he, "Khat axis 3");
    } else {
        if ((he = X1.alloc((size_t)M2l * Nl * 16)) != hipSuccess) return chk(he, "precompute buffer");
        if ((he = launch_greens_contract(g, M2, N, dC.as<double>(), X1.as<c64>(), s)) != hipSuccess) return chk(he, "kernel spectrum");
        if ((he = T.alloc((size_t)Nl * Nl * 16)) != hipSuccess) return chk(he, "precompute buffer");
        if ((he = launch_cos_contract(X1.as<c64>(), T.as<c64>(), dC.as<double>(), 1, M2, N, Nl, s)) != hipSuccess) return chk(he, "T axis 1");
        if ((he = Y1.alloc((size_t)N1 * Nl * 16)) != hipSuccess) return chk(he, "precompute buffer");
        if ((he = launch_cos_contract(T.as<c64>(), Y1.as<c64>(), dD.as<double>(), 1, N, N + 1, Nl, s)) != hipSuccess) return chk(he, "Khat axis 1");
        if ((he = K.alloc((size_t)N1 * N1 * 16)) != hipSuccess) return chk(he, "precompute buffer");
        if ((he = launch_cos_contract(Y1.as<c64>(), K.as<c64>(), dD.as<double>(), N1, N, N + 1, 1, s)) != hipSuccess) return chk(he, "Khat axis 2");
    }
    long long nK = 1;
    for (int i = 0; i < d; ++i) nK *= N1;
    p->table_complex = (p->kernel == VG_HELMHOLTZ || p->kernel == VG_LAPLACE_HELMHOLTZ) ? 1 : 0;
    const size_t esz = (p->fp64 ? 8 : 4) * (p->table_complex ? 2 : 1);
    // 3D rows padded to 16 entries from N = 96 on (below, the table is
    // L2-resident, and its reads from HBM grow with the padding); the FP32
    // tables of the staged lengths also carry the boundary block
    const long long rows = nK / N1;
    p->tab_pitch = (d == 3 && N >= 96) ? (int)((N1 + 15) / 16 * 16) : (int)N1;
    const long long nPad = rows * p->tab_pitch;
    const int bsc = (d == 3 && !p->fp64) ? staged_fetch_C(2 * N) : 0;
    const int bs = (bsc == 16 || p->table_complex) ? bsc : 0;  // 8-wide: complex tables only
    const int nb = (bs > 0 && N % bs == 0) ? N / bs : 0;
    p->tab_bnd = nb ? (unsigned)nPad : 0u;
    p->table_alg_bytes = (size_t)nK * esz;
    p->table_bytes = (size_t)(nPad + (long long)nb * N1 * N1) * esz;
    if ((he = dev_malloc(&p->table, p->table_bytes)) != hipSuccess) return chk(he, "kernel table");
    if ((he = launch_round_table(K.as<c64>(), p->table, rows, (int)N1, p->tab_pitch, p->fp64 ? 0 : 1,
                                 p->table_complex, nPad, nb, bs, s)) != hipSuccess)
        return chk(he, "table rounding");
    (void)hipEventRecord(e1, s);
    if ((he = hipStreamSynchronize(s)) != hipSuccess) return chk(he, "precompute");
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, e0, e1);
    p->precompute_ms = ms;
    if (keep_T) {
        p->T_dev = T.p;  // ownership moves to the plan
        T.p = nullptr;
    }
    return VG_OK;
}

// Twiddle table e^{-2 pi i t / L}, t in [0, L), computed in long double from
// the exact integer angle and rounded once (cached per length on the plan).
vg_status twiddle_table(vg_plan* p, int L, hipStream_t s) {
    if (p->twiddles.count(L)) return VG_OK;
    const size_t esz = p->fp64 ? 16 : 8;
    std::vector<unsigned char> h((size_t)L * esz);
    for (int t = 0; t < L; ++t) {
        const long double c = twopi_frac_cos(t, L), sn = -twopi_frac_sin(t, L);
        if (p->fp64) {
            double* q = reinterpret_cast<double*>(h.data()) + 2 * t;
            q[0] = (double)c;
            q[1] = (double)sn;
        } else {
            float* q = reinterpret_cast<float*>(h.data()) + 2 * t;
            q[0] = (float)c;
            q[1] = (float)sn;
        }
    }
    void* d = nullptr;
    hipError_t e = dev_malloc(&d, h.size());
    if (e != hipSuccess) return from_hip(e, "twiddle allocation");
    p->twiddles[L] = d;
    e = hipMemcpyAsync(d, h.data(), h.size(), hipMemcpyHostToDevice, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    return from_hip(e, "twiddle upload");
}

int fast_pass_C(int L, int mode, bool fp64);
bool fast_pass_fits(int L, int mode, bool fp64, long long ise, long long ose, long long iiq, long long oiq);
int fft_max_lds_bytes_for_device();

// ------------------------------------------------------------- programs --
namespace {

int lds_buffers_generic(int kind) {
    return (kind == KIND_FUSED || kind == KIND_FUSED_GRAD || kind == KIND_FUSED_DERIV || kind == KIND_INV_GRAD) ? 3 : 2;
}

// Tile width of one step: the specialised kernel's when one exists for its
// length (and the step needs no four-step twiddles), else the generic
// kernel's, sized so its ping-pong LDS stays within 64 KiB where possible.
// Returns 0 when not even one pencil fits in LDS.
int choose_C(const vg_plan* p, const PassStep& st, bool* specialised) {
    *specialised = false;
    const PassDesc& d = st.desc;
    if (d.real_mode) {
        // real-data variants exist for the specialised kernels only, and not
        // for rows whose complex pencil exceeds 64 KiB
        if (st.mode == MODE_ROW && (size_t)d.L * (p->fp64 ? 16 : 8) > 65536) return 0;
        const int fc = fast_pass_C(d.L, st.mode, p->fp64);
        const bool rowm = st.mode == MODE_ROW;
        if (fc > 0 && fast_pass_fits(d.L, st.mode, p->fp64, d.in_se, d.out_se, rowm ? d.in_so : 1, rowm ? d.out_so : 1)) {
            *specialised = true;
            return fc;
        }
        return 0;
    }
    // the specialised kernels cover the four-step steps of column passes:
    // step A (forward + twiddle), step B (fused, full length) and A' (inverse)
    const bool four = d.post_tw != 0 || d.fs_L1 != 0;
    const bool four_ok = !four || (st.mode == MODE_COL && ((st.kind == KIND_FWD && d.post_tw == 1 && !d.fs_L1) ||
                                                          ((st.kind == KIND_FUSED || st.kind == KIND_FUSED_GRAD ||
                                                            st.kind == KIND_FUSED_DERIV) &&
                                                           d.fs_L1 && d.post_tw == 2 && p->d == 2)));
    if (four_ok && !p->cfg.generic && !std::getenv("VG_GENERIC_PASSES")) {
        const int wc = four ? 0 : wide_col_C(d.L, st.mode, st.kind, p->fp64);
        const int fc = wc ? wc : fast_pass_C(d.L, st.mode, p->fp64);
        const bool rowm = st.mode == MODE_ROW;
        if (fc > 0 && fast_pass_fits(d.L, st.mode, p->fp64, d.in_se, d.out_se, rowm ? d.in_so : 1, rowm ? d.out_so : 1)) {
            *specialised = true;
            return fc;
        }
    }
    const size_t es = p->fp64 ? 16 : 8;
    const int nbuf = lds_buffers_generic(st.kind >= 100 ? KIND_INV : st.kind);
    int c = st.mode == MODE_COL ? 16 : 4;
    while (c > 1 && (size_t)nbuf * c * d.L * es > 65536) c /= 2;
    if ((size_t)nbuf * c * d.L * es > (size_t)fft_max_lds_bytes_for_device()) return 0;
    return c;
}

PassDesc base_desc(const vg_plan* p, int L) {
    PassDesc d;
    std::memset(&d, 0, sizeof(d));
    d.L = L;
    const std::vector<int> rad = radix_plan(L);
    d.nst = (int)rad.size();
    for (int i = 0; i < d.nst; ++i) d.radix[i] = rad[i];
    d.table = p->table;
    d.d = p->d;
    d.tabN = p->N;
    d.table_complex = p->table_complex;
    d.kscale = M_PI;  // the 2N box has period 2 in x: kappa = pi * m
    return d;
}

PassStep row_step(const vg_plan* p, int kind, int in_buf, long long in_pitch, int n_in, int out_buf,
                  long long out_pitch, int n_out, long long rows, const char* name, int out2_buf = BUF_NONE,
                  int L = 0) {
    PassStep s;
    s.desc = base_desc(p, L ? L : 2 * p->N);
    s.desc.in_so = in_pitch;
    s.desc.in_se = 1;
    s.desc.out_so = out_pitch;
    s.desc.out_se = 1;
    s.desc.n_in = n_in;
    s.desc.n_out = n_out;
    s.desc.inner = 1;
    s.desc.outer = (int)rows;
    s.mode = MODE_ROW;
    s.kind = kind;
    s.in_buf = in_buf;
    s.out_buf = out_buf;
    s.out2_buf = out2_buf;
    s.name = name;
    s.bytes = 0;
    return s;
}

PassStep col_step(const vg_plan* p, int kind, int in_buf, long long in_so, long long in_se, int n_in, int out_buf,
                  long long out_so, long long out_se, int n_out, long long inner, long long outer, const char* name,
                  int out2_buf = BUF_NONE, int L = 0) {
    PassStep s;
    s.desc = base_desc(p, L ? L : 2 * p->N);
    s.desc.in_so = in_so;
    s.desc.in_se = in_se;
    s.desc.out_so = out_so;
    s.desc.out_se = out_se;
    s.desc.n_in = n_in;
    s.desc.n_out = n_out;
    s.desc.inner = (int)inner;
    s.desc.outer = (int)outer;
    s.mode = MODE_COL;
    s.kind = kind;
    s.in_buf = in_buf;
    s.out_buf = out_buf;
    s.out2_buf = out2_buf;
    s.name = name;
    s.bytes = 0;
    return s;
}

void set_ws(Program& prog, const std::vector<size_t>& sizes_bytes) {
    prog.ws_offsets.clear();
    size_t off = 0;
    for (size_t b : sizes_bytes) {
        prog.ws_offsets.push_back(off);
        off += align256(b);
    }
    prog.ws_bytes = off;
}

}  // namespace

// Splits L = L1 L2 of a long 2D column axis, best first: both lengths with
// specialised kernels, then the fused step-B length L2 closest to 32, then
// the larger L1 (the autotuner measured L2 = 32 fastest: 2D N = 2048
// 0.222 -> 0.192 ms, N = 4096 0.818 -> 0.745 ms against L1 ~ L2).
std::vector<int> four_step_splits(int L, bool fp64) {
    std::vector<std::pair<double, int>> c;
    for (int a = 2; a < L; a += 2) {
        if (L % a) continue;
        const int b = L / a;
        if (radix_plan(a).empty() || radix_plan(b).empty()) continue;
        const bool fast = fast_pass_C(a, MODE_COL, fp64) > 0 && fast_pass_C(b, MODE_COL, fp64) > 0;
        c.push_back({std::fabs(std::log2((double)b) - 5.0) - 1e-6 * std::log2((double)a) + (fast ? 0.0 : 100.0), a});
    }
    std::stable_sort(c.begin(), c.end(), [](const auto& x, const auto& y) { return x.first < y.first - 1e-12; });
    std::vector<int> out;
    for (auto& e : c) out.push_back(e.second);
    return out;
}


void finalize_bytes(vg_plan* p);

// Intermediate layouts.  A column tile whose rows are a large power of two
// apart (a whole 2N x 2N plane in 3D, a 2N row in 2D) keeps hitting the same
// HBM channels, so those pitches are lengthened by cfg.pad_bytes (256 unless
// the autotuner picks another value).
//
// A 2D column axis too long for one LDS-resident pencil runs as four steps
// (L = L1 L2, n = L2 n1 + n2, k = k1 + L1 k2):
//   A : for each n2, length-L1 forward DFT over n1 (upper half zero), times
//       W_L^{n2 k1}, stored back at row L2 k1 + n2;
//   B : for each k1, length-L2 forward DFT over n2 -> spectral index
//       k1 + L1 k2, times Khat (and i kappa), length-L2 inverse, times
//       W_L^{-n2 k1}, stored back in place;
//   A': for each n2, length-L1 inverse over k1, rows with n1 < L1/2 kept.
vg_status build_programs(vg_plan* p, hipStream_t stream) {
    const long long N = p->N, L = 2 * N;
    const size_t es = p->fp64 ? 16 : 8;
    const long long PAD = (long long)p->cfg.pad_bytes / (long long)es;
    const int W0 = BUF_WS0, W1 = BUF_WS0 + 1, W2 = BUF_WS0 + 2, W3 = BUF_WS0 + 3, W4 = BUF_WS0 + 4;
    Program& A = p->apply_prog;
    Program& G = p->grad_prog;
    // Long specialised columns (2N >= 512) run the fused gradient pass as two
    // passes (derivative spectrum, then phi's) that each keep the register
    // budget of a plain fused pass: the single two-output pass holds two
    // spectra per thread and drops to 1 wave per SIMD (measured at N = 256:
    // 0.93 -> 0.36 + 0.33 ms; at N = 128 the single pass is faster, 0.065 vs
    // 0.096 ms).  Shorter or generic columns keep the single pass.
    auto split_fused_grad = [&](long long len) {
        return !p->cfg.generic && len >= 512 && fast_pass_C((int)len, MODE_COL, p->fp64) > 0;
    };
    const bool split_grad = split_fused_grad(L);
    A.steps.clear();
    G.steps.clear();
    if (p->d == 3) {
        const long long PL = L * L + PAD;   // plane pitch of the [N][L][L] intermediates
        const long long PS = N * L;         // [N][N][L] intermediates stay dense (pencil stride L)
        const size_t b2 = (size_t)(N * PS) * es, b4 = (size_t)(N * PL) * es;
        // apply: f -(rows, axis 3)-> W0[N][N][L] -(axis 2)-> W1[N][L][L]
        //        -(axis 1: fwd, Khat, inv, crop; in place)-> W1
        //        -(axis 2 inverse, crop)-> W0[N][N][L] -(rows inverse, crop)-> phi
        set_ws(A, {b2, b4});
        A.steps.push_back(row_step(p, KIND_FWD, BUF_F, N, (int)N, W0, L, (int)L, N * N, "p1_row_fwd"));
        A.steps.push_back(col_step(p, KIND_FWD, W0, PS, L, (int)N, W1, PL, L, (int)L, L, N, "p2_col_fwd"));
        A.steps.push_back(col_step(p, KIND_FUSED, W1, 0, PL, (int)N, W1, 0, PL, (int)N, L * L, 1, "p3_fused"));
        A.steps.push_back(col_step(p, KIND_INV, W1, PL, L, (int)L, W0, PS, L, (int)N, L, N, "p4_col_inv"));
        A.steps.push_back(row_step(p, KIND_INV, W0, L, (int)L, BUF_PHI, N, (int)N, N * N, "p5_row_inv"));
        // gradient: W0 (2V), W1 (4V), W2 (4V), W3 (2V), W4 (2V)
        set_ws(G, {b2, b4, b4, b2, b2});
        G.steps.push_back(row_step(p, KIND_FWD, BUF_F, N, (int)N, W0, L, (int)L, N * N, "g1_row_fwd"));
        G.steps.push_back(col_step(p, KIND_FWD, W0, PS, L, (int)N, W1, PL, L, (int)L, L, N, "g2_col_fwd"));
        if (split_grad) {
            // derivative spectrum first (W1 -> W2), then phi's in place
            G.steps.push_back(col_step(p, KIND_FUSED_DERIV, W1, 0, PL, (int)N, W2, 0, PL, (int)N, L * L, 1,
                                       "g3_fused_deriv"));
            G.steps.push_back(col_step(p, KIND_FUSED, W1, 0, PL, (int)N, W1, 0, PL, (int)N, L * L, 1, "g3_fused"));
        } else {
            G.steps.push_back(col_step(p, KIND_FUSED_GRAD, W1, 0, PL, (int)N, W1, 0, PL, (int)N, L * L, 1,
                                       "g3_fused_grad", W2));
        }
        G.steps.push_back(col_step(p, KIND_INV_GRAD, W1, PL, L, (int)L, W0, PS, L, (int)N, L, N,
                                   "g4_col_inv_grad", W3));
        G.steps.push_back(col_step(p, KIND_INV, W2, PL, L, (int)L, W4, PS, L, (int)N, L, N, "g4_col_inv"));
        G.steps.push_back(row_step(p, KIND_INV_GRAD, W0, L, (int)L, BUF_PHI, N, (int)N, N * N, "g5_row_inv_grad",
                                   BUF_GRAD0 + 2));
        G.steps.push_back(row_step(p, KIND_INV, W3, L, (int)L, BUF_GRAD0 + 1, N, (int)N, N * N, "g5_row_inv_d2"));
        G.steps.push_back(row_step(p, KIND_INV, W4, L, (int)L, BUF_GRAD0 + 0, N, (int)N, N * N, "g5_row_inv_d1"));
    } else {
        const long long RP = L + PAD;  // row pitch of the [rows][L] intermediates
        PassStep fused = col_step(p, KIND_FUSED, W0, 0, RP, (int)N, W0, 0, RP, (int)N, L, 1, "p2_fused");
        bool spec = false;
        const bool single = choose_C(p, fused, &spec) > 0 && (spec || L <= 1024);
        if (single) {
            const size_t b2 = (size_t)(N * RP) * es;
            set_ws(A, {b2});
            A.steps.push_back(row_step(p, KIND_FWD, BUF_F, N, (int)N, W0, RP, (int)L, N, "p1_row_fwd"));
            A.steps.push_back(fused);
            A.steps.push_back(row_step(p, KIND_INV, W0, RP, (int)L, BUF_PHI, N, (int)N, N, "p3_row_inv"));
            set_ws(G, {b2, b2});
            G.steps.push_back(row_step(p, KIND_FWD, BUF_F, N, (int)N, W0, RP, (int)L, N, "g1_row_fwd"));
            if (split_grad) {
                G.steps.push_back(col_step(p, KIND_FUSED_DERIV, W0, 0, RP, (int)N, W1, 0, RP, (int)N, L, 1,
                                           "g2_fused_deriv"));
                G.steps.push_back(col_step(p, KIND_FUSED, W0, 0, RP, (int)N, W0, 0, RP, (int)N, L, 1, "g2_fused"));
            } else {
                G.steps.push_back(col_step(p, KIND_FUSED_GRAD, W0, 0, RP, (int)N, W0, 0, RP, (int)N, L, 1,
                                           "g2_fused_grad", W1));
            }
            G.steps.push_back(row_step(p, KIND_INV_GRAD, W0, RP, (int)L, BUF_PHI, N, (int)N, N, "g3_row_inv_grad",
                                       BUF_GRAD0 + 1));
            G.steps.push_back(row_step(p, KIND_INV, W1, RP, (int)L, BUF_GRAD0 + 0, N, (int)N, N, "g3_row_inv_d1"));
        } else {
            const std::vector<int> splits = four_step_splits((int)L, p->fp64);
            if (splits.empty()) return fail(VG_ERR_UNSUPPORTED_SIZE, "no four-step split of 2N");
            int L1 = splits[0];
            if (p->cfg.fs_L1 && std::find(splits.begin(), splits.end(), p->cfg.fs_L1) != splits.end()) L1 = p->cfg.fs_L1;
            const int L2 = (int)(L / L1);
            const size_t bL = (size_t)(L * RP) * es;  // all L rows carry data between the steps
            auto stepA = [&](int kind, int buf, const char* name) {
                // outer n2 (row offset RP), columns (inner L), elements n1 (stride L2 rows)
                PassStep s = col_step(p, kind, buf, RP, (long long)L2 * RP, kind == KIND_FWD ? L1 / 2 : L1, buf, RP,
                                      (long long)L2 * RP, kind == KIND_FWD ? L1 : L1 / 2, L, L2, name, BUF_NONE, L1);
                s.desc.L_big = (int)L;
                s.desc.post_tw = kind == KIND_FWD ? 1 : 0;
                return s;
            };
            auto stepB = [&](int kind, int buf, int buf2, const char* name, int obuf = -1) {
                // outer k1 (offset L2 rows), columns, elements n2 (stride one row)
                PassStep s = col_step(p, kind, buf, (long long)L2 * RP, RP, L2, obuf < 0 ? buf : obuf, (long long)L2 * RP,
                                      RP, L2, L, L1, name, buf2, L2);
                s.desc.L_big = (int)L;
                s.desc.post_tw = 2;
                s.desc.fs_L1 = L1;
                return s;
            };
            set_ws(A, {bL});
            A.steps.push_back(row_step(p, KIND_FWD, BUF_F, N, (int)N, W0, RP, (int)L, N, "p1_row_fwd"));
            A.steps.push_back(stepA(KIND_FWD, W0, "p2a_col_fwd"));
            A.steps.push_back(stepB(KIND_FUSED, W0, BUF_NONE, "p2b_fused"));
            A.steps.push_back(stepA(KIND_INV, W0, "p2c_col_inv"));
            A.steps.push_back(row_step(p, KIND_INV, W0, RP, (int)L, BUF_PHI, N, (int)N, N, "p3_row_inv"));
            set_ws(G, {bL, bL});
            G.steps.push_back(row_step(p, KIND_FWD, BUF_F, N, (int)N, W0, RP, (int)L, N, "g1_row_fwd"));
            G.steps.push_back(stepA(KIND_FWD, W0, "g2a_col_fwd"));
            if (split_fused_grad(L2)) {
                G.steps.push_back(stepB(KIND_FUSED_DERIV, W0, BUF_NONE, "g2b_fused_deriv", W1));
                G.steps.push_back(stepB(KIND_FUSED, W0, BUF_NONE, "g2b_fused"));
            } else {
                G.steps.push_back(stepB(KIND_FUSED_GRAD, W0, W1, "g2b_fused_grad"));
            }
            G.steps.push_back(stepA(KIND_INV, W0, "g2c_col_inv"));
            G.steps.push_back(stepA(KIND_INV, W1, "g2c_col_inv_d1"));
            G.steps.push_back(row_step(p, KIND_INV_GRAD, W0, RP, (int)L, BUF_PHI, N, (int)N, N, "g3_row_inv_grad",
                                       BUF_GRAD0 + 1));
            G.steps.push_back(row_step(p, KIND_INV, W1, RP, (int)L, BUF_GRAD0 + 0, N, (int)N, N, "g3_row_inv_d1"));
        }
    }
    // Real densities with a real table (Laplace, biharmonic): the half
    // spectrum k3 in [0, N] (H = N + 1 values) of the last axis.  A real row
    // of N values is read as N/2 complex pairs, so the row passes are
    // length-N transforms with R2C / C2R processing (real_mode 1, 2); the
    // column passes and the fused pass run on H columns (real_mode 4).
    Program& Rr = p->real_prog;
    Rr.steps.clear();
    if (!p->table_complex) {
        const long long H = N + 1;
        auto rrow = [&](int kind, int in_buf, long long ip, int nin, int out_buf, long long op, int nout, long long rows,
                        const char* name, int mode) {
            PassStep s = row_step(p, kind, in_buf, ip, nin, out_buf, op, nout, rows, name, BUF_NONE, (int)N);
            s.desc.real_mode = mode;
            s.desc.L_big = (int)L;
            return s;
        };
        if (p->d == 3) {
            const long long PLr = L * H + PAD;
            set_ws(Rr, {(size_t)(N * N * H) * es, (size_t)(N * PLr) * es});
            Rr.steps.push_back(rrow(KIND_FWD, BUF_F, N / 2, (int)(N / 2), W0, H, (int)H, N * N, "r1_row_r2c", 1));
            Rr.steps.push_back(col_step(p, KIND_FWD, W0, N * H, H, (int)N, W1, PLr, H, (int)L, H, N, "r2_col_fwd"));
            PassStep f = col_step(p, KIND_FUSED, W1, 0, PLr, (int)N, W1, 0, PLr, (int)N, L * H, 1, "r3_fused");
            f.desc.real_mode = 4;
            Rr.steps.push_back(f);
            Rr.steps.push_back(col_step(p, KIND_INV, W1, PLr, H, (int)L, W0, N * H, H, (int)N, H, N, "r4_col_inv"));
            Rr.steps.push_back(rrow(KIND_INV, W0, H, (int)H, BUF_PHI, N / 2, (int)(N / 2), N * N, "r5_row_c2r", 2));
        } else {
            const long long RPr = H + PAD;
            PassStep f = col_step(p, KIND_FUSED, W0, 0, RPr, (int)N, W0, 0, RPr, (int)N, H, 1, "r2_fused");
            f.desc.real_mode = 4;
            bool spec = false;
            if (choose_C(p, f, &spec) > 0) {
                set_ws(Rr, {(size_t)(N * RPr) * es});
                Rr.steps.push_back(rrow(KIND_FWD, BUF_F, N / 2, (int)(N / 2), W0, RPr, (int)H, N, "r1_row_r2c", 1));
                Rr.steps.push_back(f);
                Rr.steps.push_back(rrow(KIND_INV, W0, RPr, (int)H, BUF_PHI, N / 2, (int)(N / 2), N, "r3_row_c2r", 2));
            } else {
                // long columns: four steps as in the complex program, on H columns
                const std::vector<int> splits = four_step_splits((int)L, p->fp64);
                if (!splits.empty()) {
                    int L1 = splits[0];
                    if (p->cfg.fs_L1 && std::find(splits.begin(), splits.end(), p->cfg.fs_L1) != splits.end())
                        L1 = p->cfg.fs_L1;
                    const int L2 = (int)(L / L1);
                    set_ws(Rr, {(size_t)(L * RPr) * es});
                    auto sA = [&](int kind, const char* name) {
                        PassStep s = col_step(p, kind, W0, RPr, (long long)L2 * RPr, kind == KIND_FWD ? L1 / 2 : L1, W0, RPr,
                                              (long long)L2 * RPr, kind == KIND_FWD ? L1 : L1 / 2, H, L2, name, BUF_NONE, L1);
                        s.desc.L_big = (int)L;
                        s.desc.post_tw = kind == KIND_FWD ? 1 : 0;
                        return s;
                    };
                    PassStep sB = col_step(p, KIND_FUSED, W0, (long long)L2 * RPr, RPr, L2, W0, (long long)L2 * RPr, RPr, L2,
                                           H, L1, "r2b_fused", BUF_NONE, L2);
                    sB.desc.L_big = (int)L;
                    sB.desc.post_tw = 2;
                    sB.desc.fs_L1 = L1;
                    sB.desc.real_mode = 4;
                    Rr.steps.push_back(rrow(KIND_FWD, BUF_F, N / 2, (int)(N / 2), W0, RPr, (int)H, N, "r1_row_r2c", 1));
                    Rr.steps.push_back(sA(KIND_FWD, "r2a_col_fwd"));
                    Rr.steps.push_back(sB);
                    Rr.steps.push_back(sA(KIND_INV, "r2c_col_inv"));
                    Rr.steps.push_back(rrow(KIND_INV, W0, RPr, (int)H, BUF_PHI, N / 2, (int)(N / 2), N, "r3_row_c2r", 2));
                }
            }
        }
    }
    // twiddles, tile widths and support check for every step
    for (Program* pr : {&A, &G, &Rr}) {
        for (PassStep& st : pr->steps) {
            vg_status s2 = twiddle_table(p, st.desc.L, stream);
            if (s2 != VG_OK) return s2;
            st.desc.tw = p->twiddles[st.desc.L];
            if (st.desc.L_big) {
                s2 = twiddle_table(p, st.desc.L_big, stream);
                if (s2 != VG_OK) return s2;
                st.desc.tw_big = p->twiddles[st.desc.L_big];
            }
            st.desc.xcd_map = p->cfg.xcd_map;
            {
                // streaming access only where column tile rows stay on whole
                // 128-byte lines (measured: the half-spectrum columns of the
                // real path, pitch N + 1, lose 25% with it)
                const long long es = p->fp64 ? 16 : 8;
                auto al = [&](long long x) { return (x * es) % 128 == 0; };
                st.desc.stream = (st.mode == MODE_ROW || (al(st.desc.in_se) && al(st.desc.out_se) &&
                                                          al(st.desc.in_so) && al(st.desc.out_so)))
                                     ? 3
                                     : 0;
            }
            st.desc.table_full = p->kernel == VG_CONVECTION ? 1 : 0;
            bool spec = false;
            st.desc.C = choose_C(p, st, &spec);
            st.desc.specialised = spec ? 1 : 0;
            if (st.desc.C == 0 && (pr == &Rr || pr == &G)) {
                // no real-data variant for this length, or a gradient pass
                // (two-output kinds hold more LDS) that fits no kernel: real
                // applies or gradients are unsupported, applies are not
                pr->steps.clear();
                pr->ws_offsets.clear();
                pr->ws_bytes = 0;
                break;
            }
            if (st.desc.C == 0) return fail(VG_ERR_UNSUPPORTED_SIZE, std::string("pass ") + st.name + ": pencil does not fit in LDS");
        }
    }
    finalize_bytes(p);
    return VG_OK;
}

namespace {
// Algorithmic bytes of a pass: each pencil reads its n_in nonzero inputs and
// writes its n_out kept outputs (twice for two-output kinds); fused passes
// also read the Khat octant once.
double pass_bytes(const vg_plan* p, const PassStep& s) {
    const double es = p->fp64 ? 16.0 : 8.0;
    const double pencils = (s.mode == MODE_COL) ? (double)s.desc.outer * s.desc.inner : (double)s.desc.outer;
    double outs = (s.out2_buf != BUF_NONE) ? 2.0 : 1.0;
    double b = pencils * es * (s.desc.n_in + outs * s.desc.n_out);
    if (s.kind == KIND_FUSED || s.kind == KIND_FUSED_GRAD || s.kind == KIND_FUSED_DERIV) b += (double)p->table_alg_bytes;
    return b;
}
}  // namespace

void finalize_bytes(vg_plan* p) {
    for (Program* pr : {&p->apply_prog, &p->grad_prog, &p->real_prog})
        for (PassStep& s : pr->steps) s.bytes = pass_bytes(p, s);
}

BoundStep bind_step(const vg_plan* p, const Program& prog, const PassStep& st, const void* f, void* phi, void* grad,
                    void* ws) {
    long long V = 1;
    for (int i = 0; i < p->d; ++i) V *= p->N;
    const size_t es = p->fp64 ? 16 : 8;
    auto resolve = [&](int id) -> void* {
        if (id == BUF_F) return const_cast<void*>(f);
        if (id == BUF_PHI) return phi;
        if (id >= BUF_GRAD0 && id < BUF_GRAD0 + 3)
            return grad ? static_cast<unsigned char*>(grad) + (size_t)(id - BUF_GRAD0) * V * es : nullptr;
        if (id >= BUF_WS0 && id < BUF_WS0 + 8) return static_cast<unsigned char*>(ws) + prog.ws_offsets[id - BUF_WS0];
        return nullptr;
    };
    BoundStep b;
    b.desc = st.desc;
    b.desc.table = p->table;  // programs are built before the precompute fills the table
    b.desc.tab_pitch = p->tab_pitch;
    b.desc.tab_bnd = p->tab_bnd;
    b.desc.in = resolve(st.in_buf);
    b.desc.out = resolve(st.out_buf);
    b.desc.out2 = resolve(st.out2_buf);
    b.kind = st.kind;
    if (b.kind == KIND_INV_GRAD && b.desc.out == nullptr) {
        // gradient without phi: derivative-only inverse into out2
        b.desc.out = b.desc.out2;
        b.desc.out2 = nullptr;
        b.kind = 100 + KIND_INV;
    }
    b.mode = st.mode;
    b.name = st.name;
    b.bytes = st.bytes;
    return b;
}

std::vector<BoundStep> bind_program(const vg_plan* p, const Program& prog, const void* f, void* phi, void* grad,
                                    void* ws) {
    std::vector<BoundStep> out;
    out.reserve(prog.steps.size());
    for (const PassStep& st : prog.steps) out.push_back(bind_step(p, prog, st, f, phi, grad, ws));
    return out;
}

vg_status run_program(const vg_plan* p, const Program& prog, const void* f, void* phi, void* grad, void* ws,
                      hipStream_t stream) {
    const std::vector<BoundStep> steps = bind_program(p, prog, f, phi, grad, ws);
    const int pm = profiler_mode();
    if (pm == 2) {
        // events around the pass with the most bytes only
        size_t dom = 0;
        for (size_t i = 1; i < steps.size(); ++i)
            if (steps[i].bytes > steps[dom].bytes) dom = i;
        for (size_t i = 0; i < steps.size(); ++i) {
            const BoundStep& st = steps[i];
            void* a = i == dom ? profiler_mark(stream) : nullptr;
            hipError_t e = launch_fft_pass(st.desc, st.mode, st.kind, p->fp64, stream);
            if (e != hipSuccess) return from_hip(e, st.name);
            if (a) profiler_add(st.name, a, profiler_mark(stream), st.bytes);
        }
        return VG_OK;
    }
    void* mark = pm ? profiler_mark(stream) : nullptr;
    for (const BoundStep& st : steps) {
        hipError_t e = launch_fft_pass(st.desc, st.mode, st.kind, p->fp64, stream);
        if (e != hipSuccess) return from_hip(e, st.name);
        if (mark) {
            void* next = profiler_mark(stream);
            profiler_add(st.name, mark, next, st.bytes);
            mark = next;
        }
    }
    return VG_OK;
}


// The same launches as run_program with no host containers and no profiler
// events: the path of the allocation-free entry point.
vg_status run_program_noalloc(const vg_plan* p, const Program& prog, const void* f, void* phi, void* grad, void* ws,
                              hipStream_t stream) {
    for (const PassStep& ps : prog.steps) {
        const BoundStep st = bind_step(p, prog, ps, f, phi, grad, ws);
        hipError_t e = launch_fft_pass(st.desc, st.mode, st.kind, p->fp64, stream);
        if (e != hipSuccess) return from_hip(e, st.name);
    }
    return VG_OK;
}

}  // namespace vg
