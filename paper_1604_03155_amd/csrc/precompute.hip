// FP64 plan precompute (Sections 2 and 4).
//
// 1. Kernel spectrum: G^L(|s_m|) on the P N-per-axis lattice s_m = (2 pi/P) m
//    (Section 2), from the closed forms of Table 1 (3D) and Table 2 (2D):
//    Laplace, Helmholtz, biharmonic and Delta (Delta + k^2).
//    Where a printed form is 0/0 (s = 0, s = k) an algebraically equal form or
//    a series of the same radial integral is used.
// 2. T(n) = M^-d sum_m G(|s_m|) e^{2 pi i m.n/M}, n in [0, N)^d.  G depends on
//    |m_j| only, so per axis the sum folds onto m in [0, M/2] with weights
//    1, 2, ..., 2, 1 and cosines: T is a chain of d dense contractions with the
//    matrix C[n][m] = w_m cos(2 pi m n / M) / M (built on the host).  The first
//    contraction evaluates G on the fly, so the (M/2+1)^d lattice is never
//    stored.
// 3. Khat(k) = sum_{|n_j|<=N-1} T(n) e^{-2 pi i k.n/(2N)} on k in [0, N]^d: the
//    same chain with D[k][n] = v_n cos(pi k n / N) / (2N), v_0 = 1, v_n = 2,
//    which also folds in the 1/(2N)^d of the inverse FFT.
#include "common.h"

namespace vg {

namespace {

__device__ __forceinline__ double sinc_d(double x) {
    const double ax = fabs(x);
    if (ax < 1e-4) {
        const double x2 = x * x;
        return 1.0 - x2 / 6.0 + x2 * x2 / 120.0;
    }
    return sin(x) / x;
}

__device__ __forceinline__ c64 cexp_i(double a) {
    double s, c;
    sincos(a, &s, &c);
    return mk(c, s);
}

// Table 1, Delta: G = 2 (sin(Ls/2)/s)^2 = (L^2/2) sinc^2(L s / 2)
__device__ c64 g_laplace3d(double s, const GreensParams& g) {
    const double v = sinc_d(0.5 * g.L * s);
    return mk(0.5 * g.L * g.L * v * v, 0.0);
}

// Table 1, Delta + k^2:
//   G = [-1 + e^{ikL}(cos Ls - i k L sinc(Ls))] / ((k - s)(k + s))   (far from s = k)
//   G = -[A(k+s) - A(k-s)] / (2 s),  A(w) = i L e^{iwL/2} sinc(wL/2)  (|s - k| < k/2)
//   power series in (sL)^2 with host coefficients when max(s, k) L < 1
__device__ c64 g_helmholtz3d(double s, const GreensParams& g) {
    const double k = g.k, L = g.L;
    if (fmax(s, k) * L < 1.0) {
        const double x2 = (s * L) * (s * L);
        c64 acc = mk(0.0, 0.0);
        for (int j = g.ntaylor - 1; j >= 0; --j) acc = mk(acc.x * x2 + g.taylor_r[j], acc.y * x2 + g.taylor_i[j]);
        return acc;
    }
    if (fabs(s - k) < 0.5 * k) {
        const double wp = k + s, wm = k - s;
        const c64 ep = cexp_i(0.5 * wp * L), em = cexp_i(0.5 * wm * L);
        const double sp = sinc_d(0.5 * wp * L), sm = sinc_d(0.5 * wm * L);
        // A(w) = i L e sinc -> (-L e.y sinc, L e.x sinc)
        const c64 Ap = mk(-L * ep.y * sp, L * ep.x * sp);
        const c64 Am = mk(-L * em.y * sm, L * em.x * sm);
        const double f = -1.0 / (2.0 * s);
        return mk((Ap.x - Am.x) * f, (Ap.y - Am.y) * f);
    }
    const c64 e = cexp_i(k * L);
    double sn, cs;
    sincos(L * s, &sn, &cs);
    const double sc = (s * L == 0.0) ? 1.0 : sn / (L * s);
    // e * (cs - i kL sc)
    const double br = cs, bi = -k * L * sc;
    const double nr = -1.0 + (e.x * br - e.y * bi);
    const double ni = e.x * bi + e.y * br;
    const double den = (k - s) * (k + s);
    return mk(nr / den, ni / den);
}

// Table 2, Delta: G = L^2 [(1 - J0(x))/x^2 - log(L) J1(x)/x], x = L s, with
// the Bessel power series for x < 1.
__device__ c64 g_laplace2d(double s, const GreensParams& g) {
    const double L = g.L;
    const double x = L * s;
    double a, b;
    if (x < 1.0) {
        const double x2 = x * x;
        // (1 - J0)/x^2 = sum_{m>=1} (-1)^(m+1) x^(2m-2) / (4^m (m!)^2)
        // J1/x        = sum_{m>=0} (-1)^m x^(2m) / (2^(2m+1) m! (m+1)!)
        double ta = 0.25, tb = 0.5;
        a = 0.0;
        b = 0.0;
        for (int m = 1; m < 20; ++m) {
            a += ta;
            ta *= -x2 / (4.0 * (m + 1) * (m + 1));
        }
        for (int m = 0; m < 20; ++m) {
            b += tb;
            tb *= -x2 / (4.0 * (m + 1) * (m + 2));
        }
    } else {
        a = (1.0 - j0(x)) / (x * x);
        b = j1(x) / x;
    }
    return mk(L * L * (a - log(L) * b), 0.0);
}

// Table 2, Delta + k^2:
//   G = [1 + (i pi/2) L (s J1(Ls) H0 - k J0(Ls) H1)] / ((s - k)(s + k)),
//   H0 = H_0^(1)(kL), H1 = H_1^(1)(kL); Taylor expansion about s = k inside
//   the window (host coefficients of N(s)/(s - k)).
__device__ c64 g_helmholtz2d(double s, const GreensParams& g) {
    const double k = g.k, L = g.L;
    if (fabs(s - k) < g.window) {
        const double ds = s - k;
        c64 acc = mk(0.0, 0.0);
        for (int n = g.ntaylor - 1; n >= 0; --n) acc = mk(acc.x * ds + g.taylor_r[n], acc.y * ds + g.taylor_i[n]);
        const double inv = 1.0 / (s + k);
        return mk(acc.x * inv, acc.y * inv);
    }
    const double x = L * s;
    const double u = s * j1(x), v = k * j0(x);
    // (i pi/2) L (u H0 - v H1)
    const double tr = u * g.H0r - v * g.H1r, ti = u * g.H0i - v * g.H1i;
    const double h = 0.5 * M_PI * L;
    const double nr = 1.0 - h * ti, ni = h * tr;
    const double den = (s - k) * (s + k);
    return mk(nr / den, ni / den);
}

// Table 1, Delta^2 (kernel r/(8 pi)):
//   G = [(2 - x^2) cos x + 2 x sin x - 2] / (2 s^4),  x = L s;
// for x < 1 (where the numerator cancels to O(x^4)) the power series of the
// radial integral (1/(2s)) int_0^L r^2 sin(sr) dr:
//   G = (L^4/2) sum_n (-1)^n x^(2n) / ((2n + 4)(2n + 1)!).
__device__ c64 g_biharmonic3d(double s, const GreensParams& g) {
    const double L = g.L, x = L * s;
    if (x < 1.0) {
        const double x2 = x * x;
        double term = 1.0, acc = 0.0;  // term = (-1)^n x^(2n) / (2n+1)!
        for (int n = 0; n < 12; ++n) {
            acc += term / (2 * n + 4);
            term *= -x2 / ((2.0 * n + 2.0) * (2.0 * n + 3.0));
        }
        return mk(0.5 * L * L * L * L * acc, 0.0);
    }
    double sn, cs;
    sincos(x, &sn, &cs);
    const double s2 = s * s;
    return mk(((2.0 - x * x) * cs + 2.0 * x * sn - 2.0) / (2.0 * s2 * s2), 0.0);
}

// Table 2, Delta^2 (kernel -(r^2/(8 pi))(log r - 1)):
//   G = (J0(x) - 1)/s^4 - L^3 (log L - 1) J1(x)/(4s) + L log L J1(x)/s^3
//       - L^2 (2 log L - 1) J0(x)/(4 s^2),  x = L s;
// for x < 1 the series of -(1/4) int_0^L r^3 (log r - 1) J0(sr) dr:
//   G = -(L^4/4) sum_n (-1)^n (x/2)^(2n)/(n!)^2 [(log L - 1)/(2n+4) - 1/(2n+4)^2].
__device__ c64 g_biharmonic2d(double s, const GreensParams& g) {
    const double L = g.L, x = L * s, lg = log(L);
    if (x < 1.0) {
        const double q = 0.25 * x * x;
        double term = 1.0, acc = 0.0;  // term = (-1)^n (x/2)^(2n) / (n!)^2
        for (int n = 0; n < 14; ++n) {
            const double m1 = 2.0 * n + 4.0;
            acc += term * ((lg - 1.0) / m1 - 1.0 / (m1 * m1));
            term *= -q / ((n + 1.0) * (n + 1.0));
        }
        return mk(-0.25 * L * L * L * L * acc, 0.0);
    }
    const double J0 = j0(x), J1 = j1(x), s2 = s * s;
    return mk((J0 - 1.0) / (s2 * s2) - L * L * L * (lg - 1.0) * J1 / (4.0 * s) + L * lg * J1 / (s2 * s) -
                  L * L * (2.0 * lg - 1.0) * J0 / (4.0 * s2),
              0.0);
}

// kernel: 0 Delta, 1 Delta + k^2, 2 Delta^2, 3 Delta (Delta + k^2) (G_k - G_0)
__device__ __forceinline__ c64 g_eval(double s, const GreensParams& g) {
    if (g.d == 3) {
        if (g.kernel == 0) return g_laplace3d(s, g);
        if (g.kernel == 1) return g_helmholtz3d(s, g);
        if (g.kernel == 2) return g_biharmonic3d(s, g);
        const c64 a = g_helmholtz3d(s, g), b = g_laplace3d(s, g);
        return mk(a.x - b.x, a.y - b.y);
    }
    if (g.kernel == 0) return g_laplace2d(s, g);
    if (g.kernel == 1) return g_helmholtz2d(s, g);
    if (g.kernel == 2) return g_biharmonic2d(s, g);
    const c64 a = g_helmholtz2d(s, g), b = g_laplace2d(s, g);
    return mk(a.x - b.x, a.y - b.y);
}

// Y[row, n] = sum_m Cm[n][m] X[row, m], X complex, Cm real (Nout x K).
// X[row, m] lives at (row / I) * K * I + m * I + (row % I); Y likewise with
// Nout.  GEN: X is G(|s|) on the octant lattice, row = flattened leading
// indices (I == 1), m = last index.
constexpr int TR = 64, TN = 64, TK = 16;

// s + c += v with the rounding error of the addition carried in c (Knuth's
// TwoSum).
__device__ __forceinline__ void two_sum_acc(double& s, double& c, double v) {
    const double t = s + v;
    const double bp = t - s;
    const double err = (s - (t - bp)) + (v - bp);
    s = t;
    c += err;
}

template <bool GEN>
__global__ void __launch_bounds__(256) contract_kernel(const c64* __restrict__ X, c64* __restrict__ Y,
                                                       const double* __restrict__ Cm, long long rows, int K,
                                                       int Nout, long long I, GreensParams g) {
    __shared__ c64 xs[TK][TR];
    __shared__ double cs[TK][TN + 1];
    const int tid = threadIdx.x;
    const int tx = tid % 16, ty = tid / 16;
    const long long r0 = (long long)blockIdx.x * TR;
    const int n0 = blockIdx.y * TN;
    c64 acc[4][4], comp[4][4];
#pragma unroll
    for (int a = 0; a < 4; ++a)
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            acc[a][b] = mk(0.0, 0.0);
            comp[a][b] = mk(0.0, 0.0);
        }

    for (int m0 = 0; m0 < K; m0 += TK) {
        // stage X tile (TR rows x TK m)
        for (int idx = tid; idx < TR * TK; idx += 256) {
            int rr, mm;
            if (I == 1) {
                rr = idx / TK;
                mm = idx % TK;
            } else {
                rr = idx % TR;
                mm = idx / TR;
            }
            const long long row = r0 + rr;
            const int m = m0 + mm;
            c64 v = mk(0.0, 0.0);
            if (row < rows && m < K) {
                if (GEN && g.full) {
                    // row -> leading lattice indices (FFT order), shifted by h:
                    // |s_m - h| with s_m = ds * signed(m); the last axis is m
                    const int hm = g.M / 2;
                    double ds2 = g.ds * (double)(m < hm ? m : m - g.M) - g.h[g.d - 1];
                    double sq = ds2 * ds2;
                    long long rem = row;
                    for (int ax = g.d - 2; ax >= 0; --ax) {
                        const long long mi = rem % K;
                        rem /= K;
                        const double sv = g.ds * (double)(mi < hm ? mi : mi - g.M) - g.h[ax];
                        sq += sv * sv;
                    }
                    v = g_eval(sqrt(sq), g);
                } else if (GEN) {
                    // row -> leading octant indices
                    double sq = (double)m * m;
                    long long rem = row;
                    for (int ax = 0; ax < g.d - 1; ++ax) {
                        const long long mi = rem % K;
                        rem /= K;
                        sq += (double)mi * mi;
                    }
                    v = g_eval(g.ds * sqrt(sq), g);
                } else {
                    const long long o = row / I, i = row - (row / I) * I;
                    v = X[(o * K + m) * I + i];
                }
            }
            xs[mm][rr] = v;
        }
        for (int idx = tid; idx < TN * TK; idx += 256) {
            const int mm = idx % TK, nn = idx / TK;
            const int m = m0 + mm, n = n0 + nn;
            cs[mm][nn] = (m < K && n < Nout) ? Cm[(long long)n * K + m] : 0.0;
        }
        __syncthreads();
        // the chunk's TK terms are summed on their own, then added to the
        // running sums with compensation (TwoSum), so rounding grows with
        // TK + K/TK terms instead of K
        c64 part[4][4];
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int b = 0; b < 4; ++b) part[a][b] = mk(0.0, 0.0);
#pragma unroll 4
        for (int mm = 0; mm < TK; ++mm) {
            c64 xv[4];
            double cv[4];
#pragma unroll
            for (int a = 0; a < 4; ++a) xv[a] = xs[mm][ty * 4 + a];
#pragma unroll
            for (int b = 0; b < 4; ++b) cv[b] = cs[mm][tx * 4 + b];
#pragma unroll
            for (int a = 0; a < 4; ++a)
#pragma unroll
                for (int b = 0; b < 4; ++b) {
                    part[a][b].x = fma(xv[a].x, cv[b], part[a][b].x);
                    part[a][b].y = fma(xv[a].y, cv[b], part[a][b].y);
                }
        }
#pragma unroll
        for (int a = 0; a < 4; ++a)
#pragma unroll
            for (int b = 0; b < 4; ++b) {
                two_sum_acc(acc[a][b].x, comp[a][b].x, part[a][b].x);
                two_sum_acc(acc[a][b].y, comp[a][b].y, part[a][b].y);
            }
        __syncthreads();
    }
#pragma unroll
    for (int a = 0; a < 4; ++a) {
        const long long row = r0 + ty * 4 + a;
        if (row >= rows) continue;
        const long long o = row / I, i = row - (row / I) * I;
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            const int n = n0 + tx * 4 + b;
            if (n < Nout) Y[(o * Nout + n) * I + i] = mk(acc[a][b].x + comp[a][b].x, acc[a][b].y + comp[a][b].y);
        }
    }
}

__global__ void combine_kernel(const c64* __restrict__ a, const c64* __restrict__ b, c64* __restrict__ out, long long n,
                               double sign) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const c64 x = a[i], y = b[i];
    out[i] = mk(x.x - sign * y.y, x.y + sign * y.x);
}

__device__ __forceinline__ void put_entry(void* out, long long i, c64 v, int to_fp32, int complex_out) {
    if (to_fp32) {
        if (complex_out) {
            reinterpret_cast<c32*>(out)[i] = mk((float)v.x, (float)v.y);
        } else {
            reinterpret_cast<float*>(out)[i] = (float)v.x;
        }
    } else {
        if (complex_out) {
            reinterpret_cast<c64*>(out)[i] = v;
        } else {
            reinterpret_cast<double*>(out)[i] = v.x;
        }
    }
}

// One thread per padded table slot: row r, entry e < pitch (pads are zero).
__global__ void round_table_kernel(const c64* __restrict__ in, void* __restrict__ out, long long rows, int N1,
                                   int pitch, int to_fp32, int complex_out, long long bnd, int nb, int bs) {
    const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= rows * pitch) return;
    const long long r = i / pitch;
    const int e = (int)(i - r * pitch);
    const c64 v = e < N1 ? in[r * N1 + e] : mk(0.0, 0.0);
    put_entry(out, i, v, to_fp32, complex_out);
    if (nb > 0 && e >= bs && e % bs == 0 && e / bs <= nb) {
        // r = k1 N1 + k2 (3D octant rows)
        const long long k1 = r / N1, k2 = r - (r / N1) * N1;
        put_entry(out, bnd + (k2 * nb + (e / bs - 1)) * N1 + k1, v, to_fp32, complex_out);
    }
}

}  // namespace

// First contraction with on-the-fly kernel spectrum: the octant has M2 = M/2+1
// points per axis; the output is (M2)^(d-1) x n_out.
hipError_t launch_greens_contract(const GreensParams& g, int M2, int n_out, const double* cmat, c64* out,
                                  hipStream_t s) {
    long long rows = 1;
    for (int ax = 0; ax < g.d - 1; ++ax) rows *= M2;
    const dim3 grid((unsigned)((rows + TR - 1) / TR), (unsigned)((n_out + TN - 1) / TN));
    hipLaunchKernelGGL(contract_kernel<true>, grid, dim3(256), 0, s, nullptr, out, cmat, rows, M2, n_out, 1LL, g);
    return hipGetLastError();
}

hipError_t launch_greens_contract_full(const GreensParams& g, int n_out, const double* cmat, c64* out, hipStream_t s) {
    long long rows = 1;
    for (int ax = 0; ax < g.d - 1; ++ax) rows *= g.M;
    const dim3 grid((unsigned)((rows + TR - 1) / TR), (unsigned)((n_out + TN - 1) / TN));
    hipLaunchKernelGGL(contract_kernel<true>, grid, dim3(256), 0, s, nullptr, out, cmat, rows, g.M, n_out, 1LL, g);
    return hipGetLastError();
}

hipError_t launch_combine(const c64* a, const c64* b, c64* out, long long n, int sign, hipStream_t s) {
    const unsigned blocks = (unsigned)((n + 255) / 256);
    hipLaunchKernelGGL(combine_kernel, dim3(blocks), dim3(256), 0, s, a, b, out, n, (double)sign);
    return hipGetLastError();
}

// Contraction of the middle index of X[O][Min][I] with Cm (Nout x Min).
hipError_t launch_cos_contract(const c64* in, c64* out, const double* cmat, long long O, int Min, int Nout,
                               long long I, hipStream_t s) {
    const long long rows = O * I;
    const dim3 grid((unsigned)((rows + TR - 1) / TR), (unsigned)((Nout + TN - 1) / TN));
    GreensParams g{};
    hipLaunchKernelGGL(contract_kernel<false>, grid, dim3(256), 0, s, in, out, cmat, rows, Min, Nout, I, g);
    return hipGetLastError();
}

hipError_t launch_round_table(const c64* in, void* out, long long rows, int N1, int pitch, int to_fp32,
                              int complex_out, long long bnd, int nb, int bs, hipStream_t s) {
    if (pitch < N1 || (nb > 0 && (bs <= 0 || (long long)(N1 - 1) < (long long)bs * nb))) return hipErrorInvalidValue;
    const long long n = rows * pitch;
    if (n <= 0) return hipSuccess;
    const unsigned blocks = (unsigned)((n + 255) / 256);
    hipLaunchKernelGGL(round_table_kernel, dim3(blocks), dim3(256), 0, s, in, out, rows, N1, pitch, to_fp32,
                       complex_out, bnd, nb, bs);
    return hipGetLastError();
}

}  // namespace vg
