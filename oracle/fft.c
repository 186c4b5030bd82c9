/*
 * FP64 discrete Fourier transforms for the oracle.  TEST INFRASTRUCTURE ONLY:
 * nothing in the product library links or calls this file.
 *
 * Definition (the DFT every transform of the method is made of, Sections 2
 * and 4):
 *     X[k] = sum_{j=0}^{n-1} x[j] W_n^{j k},   W_n = exp(sign * 2 pi i / n),
 * sign = -1 forward, +1 inverse (unnormalised; the caller divides by n).
 *
 * Algorithm: recursive Cooley-Tukey decimation in time.  With p the smallest
 * prime factor of n and m = n / p, the p interleaved subsequences
 * x_r[j] = x[r + p j] (r < p, j < m) are transformed (length m), and
 *     X[k + q m] = sum_{r<p} W_n^{r (k + q m)} X_r[k]
 *                = sum_{r<p} W_p^{r q} (W_n^{r k} X_r[k]),    k < m, q < p.
 * A prime length is summed by the definition.  Powers W_n^t use a table of
 * W_n0^t, t in [0, n0) for the top-level length n0 (W_n^t = W_n0^{t n0 / n}),
 * with the exponent reduced modulo n0 in integers and cos / sin evaluated in
 * long double, rounded once to double.
 *
 * A multi-dimensional transform applies the 1D transform along every axis in
 * turn (the d-dimensional DFT is separable).  Arrays are C-ordered, complex
 * values interleaved (re, im), transformed in place.  OpenMP threads take
 * pencils (1D lines along the axis).
 */
#include <math.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

typedef struct {
    double re, im;
} cpx;

static long long smallest_prime_factor(long long n) {
    for (long long p = 2; p * p <= n; ++p)
        if (n % p == 0) return p;
    return n;
}

/* W_n0^t for t in [0, n0): exp(sign 2 pi i t / n0). */
static cpx* twiddle_table(long long n0, int sign) {
    cpx* w = (cpx*)malloc((size_t)n0 * sizeof(cpx));
    if (!w) return NULL;
    const long double two_pi = 6.283185307179586476925286766559005768L;
    for (long long t = 0; t < n0; ++t) {
        const long double a = two_pi * (long double)t / (long double)n0;
        w[t].re = (double)cosl(a);
        w[t].im = (double)(sign * sinl(a));
    }
    return w;
}

static inline cpx cmul(cpx a, cpx b) {
    cpx c;
    c.re = a.re * b.re - a.im * b.im;
    c.im = a.re * b.im + a.im * b.re;
    return c;
}

/*
 * y[0..n) = DFT_n of x[0], x[xs], ..., x[(n-1) xs].  W_n^t = w[t * wstep]
 * for 0 <= t < n (wstep = n0 / n).  tmp holds at least the largest prime
 * factor of n values.
 */
static void fft_rec(const cpx* x, long long xs, cpx* y, long long n, const cpx* w, long long wstep, cpx* tmp) {
    if (n == 1) {
        y[0] = x[0];
        return;
    }
    const long long p = smallest_prime_factor(n);
    if (p == n) {
        for (long long k = 0; k < n; ++k) {
            double re = 0.0, im = 0.0;
            for (long long j = 0; j < n; ++j) {
                const cpx t = cmul(x[j * xs], w[((j * k) % n) * wstep]);
                re += t.re;
                im += t.im;
            }
            y[k].re = re;
            y[k].im = im;
        }
        return;
    }
    const long long m = n / p;
    for (long long r = 0; r < p; ++r) fft_rec(x + r * xs, xs * p, y + r * m, m, w, wstep * p, tmp);
    for (long long k = 0; k < m; ++k) {
        /* r k < p m = n: no reduction needed */
        for (long long r = 0; r < p; ++r) tmp[r] = cmul(y[r * m + k], w[(r * k) * wstep]);
        for (long long q = 0; q < p; ++q) {
            double re = 0.0, im = 0.0;
            for (long long r = 0; r < p; ++r) {
                /* W_p^{r q} = W_n^{(r q mod p) m} */
                const cpx t = cmul(tmp[r], w[((r * q) % p) * m * wstep]);
                re += t.re;
                im += t.im;
            }
            y[q * m + k].re = re;
            y[q * m + k].im = im;
        }
    }
}

/*
 * In-place DFT along `axis` of a C-ordered complex128 array of the given
 * shape.  sign = -1 forward, +1 inverse (unnormalised).  nthreads <= 0: the
 * OpenMP default.  Returns 0, or -1 on a bad argument / allocation failure.
 */
int oracle_fft_axis(double* data, int ndim, const long long* shape, int axis, int sign, int nthreads) {
    if (!data || ndim < 1 || axis < 0 || axis >= ndim || (sign != 1 && sign != -1)) return -1;
    long long n = shape[axis], stride = 1, outer = 1;
    for (int a = axis + 1; a < ndim; ++a) stride *= shape[a];
    for (int a = 0; a < axis; ++a) outer *= shape[a];
    if (n <= 0 || stride <= 0 || outer <= 0) return 0;
    if (n == 1) return 0;
    cpx* w = twiddle_table(n, sign);
    if (!w) return -1;
    cpx* arr = (cpx*)data;
    const long long pencils = outer * stride;
    int failed = 0;
#ifdef _OPENMP
    if (nthreads <= 0) nthreads = omp_get_max_threads();
#pragma omp parallel num_threads(nthreads) reduction(| : failed)
#endif
    {
        cpx* in = (cpx*)malloc((size_t)n * sizeof(cpx));
        cpx* out = (cpx*)malloc((size_t)n * sizeof(cpx));
        cpx* tmp = (cpx*)malloc((size_t)n * sizeof(cpx));
        if (!in || !out || !tmp) {
            failed = 1;
        } else {
#ifdef _OPENMP
#pragma omp for schedule(static)
#endif
            for (long long pc = 0; pc < pencils; ++pc) {
                const long long o = pc / stride, c = pc % stride;
                cpx* base = arr + o * n * stride + c;
                for (long long e = 0; e < n; ++e) in[e] = base[e * stride];
                fft_rec(in, 1, out, n, w, 1, tmp);
                for (long long e = 0; e < n; ++e) base[e * stride] = out[e];
            }
        }
        free(in);
        free(out);
        free(tmp);
    }
    free(w);
    return failed ? -1 : 0;
}

/* In-place d-dimensional DFT (every axis in turn). */
int oracle_fft_nd(double* data, int ndim, const long long* shape, int sign, int nthreads) {
    for (int a = 0; a < ndim; ++a) {
        const int st = oracle_fft_axis(data, ndim, shape, a, sign, nthreads);
        if (st != 0) return st;
    }
    return 0;
}
