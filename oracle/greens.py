"""Fourier transforms of the truncated free-space Green's functions (FP64).

Test infrastructure (see the package docstring).

Convention (Introduction, the Fourier transform eq. `ft`): F(s) = int e^{-i s.x} f(x) dx.
For a radial function the transform is radial and given by the one-dimensional
integrals of Section 2:
    3D:  F(s) = 4 pi int_0^inf sin(s r)/(s r) f(r) r^2 dr
    2D:  F(s) = 2 pi int_0^inf J_0(s r) f(r) r dr.
The truncated kernel is g^L = g * rect(r / 2L) (Introduction), so the integrals
stop at r = L; the paper's radii are L = 1.8 in 3D and L = 1.5 in 2D (Section 2).

Closed forms are Table 1 (3D) and Table 2 (2D).  Where a printed form divides two
quantities that both vanish (s -> 0, s -> k) it is replaced here by an
algebraically equal form or a convergent series, derived from the same radial
integral; each replacement is stated in its docstring.  The 2D Helmholtz kernel
is (i/4) H_0^(1)(k r) as in Table 2.
"""
from __future__ import annotations

import math

import numpy as np
from scipy import special as sp

L_DEFAULT = {3: 1.8, 2: 1.5}


def _sinc(x):
    """sin(x)/x with the value 1 at x = 0."""
    return np.sinc(np.asarray(x, dtype=np.float64) / math.pi)


def g_laplace3d(s, L=1.8):
    """Table 1, operator Delta: G(s) = 2 (sin(L s / 2) / s)^2, written as
    (L^2/2) sinc^2(L s / 2), which is finite and exact at s = 0 (value L^2/2)."""
    s = np.asarray(s, dtype=np.float64)
    return 0.5 * L * L * _sinc(0.5 * L * s) ** 2


def _helm3d_series(s, k, L, terms=30):
    """Double power series of (1/s) int_0^L sin(s r) e^{i k r} dr, used when both
    s L and k L are below 1.  Expanding sin(s r)/s and e^{i k r} and integrating
    r^(2j+1+p) term by term gives
        L^2 sum_j sum_p (-1)^j (sL)^(2j) (i k L)^p / ((2j+1)! p! (2j+2+p))."""
    sL = np.asarray(s, dtype=np.float64) * L
    ikL = 1j * k * L
    out = np.zeros(sL.shape, dtype=np.complex128)
    for j in range(terms):
        aj = ((-1.0) ** j) * sL ** (2 * j) / math.factorial(2 * j + 1)
        inner = 0.0 + 0.0j
        for p in range(terms):
            inner += ikL ** p / (math.factorial(p) * (2 * j + 2 + p))
        out += aj * inner
    return L * L * out


def g_helmholtz3d(s, k, L=1.8):
    """Table 1, operator Delta + k^2, kernel e^{ikr}/(4 pi r):
        G(s) = [-1 + e^{iLk} (cos(L s) - i (k/s) sin(L s))] / ((k - s)(k + s)).

    The radial integral is G(s) = (1/s) int_0^L sin(s r) e^{i k r} dr.  Three
    regions, all equal to that integral:
      * max(s, k) L < 1: its double power series (no cancellation);
      * |s - k| < k/2: writing sin as exponentials,
            G = -[A(k + s) - A(k - s)] / (2 s),  A(w) = i L e^{i w L/2} sinc(w L/2),
        which is smooth through s = k where the printed quotient is 0/0;
      * otherwise the printed form with (k/s) sin(Ls) = k L sinc(L s).
    """
    s = np.asarray(s, dtype=np.float64)
    out = np.empty(s.shape, dtype=np.complex128)
    k = float(k)
    series = np.maximum(s, k) * L < 1.0
    near = (~series) & (np.abs(s - k) < 0.5 * k)
    far = ~(series | near)
    if np.any(series):
        out[series] = _helm3d_series(s[series], k, L)
    if np.any(near):
        sn = s[near]

        def A(w):
            return 1j * L * np.exp(0.5j * w * L) * _sinc(0.5 * w * L)

        out[near] = -(A(k + sn) - A(k - sn)) / (2.0 * sn)
    if np.any(far):
        sf = s[far]
        num = -1.0 + np.exp(1j * L * k) * (np.cos(L * sf) - 1j * k * L * _sinc(L * sf))
        out[far] = num / ((k - sf) * (k + sf))
    return out


def g_laplace2d(s, L=1.5):
    """Table 2, operator Delta, kernel -(1/2 pi) log r:
        G(s) = (1 - J_0(L s)) / s^2 - L log(L) J_1(L s) / s
             = L^2 [ (1 - J_0(x)) / x^2 - log(L) J_1(x) / x ],  x = L s.
    For x < 1 both brackets are summed from the Bessel power series
        (1 - J_0(x))/x^2 = sum_{m>=1} (-1)^(m+1) x^(2m-2) / (4^m (m!)^2),
        J_1(x)/x        = sum_{m>=0} (-1)^m x^(2m) / (2^(2m+1) m! (m+1)!),
    which avoids the cancellation in 1 - J_0(x) near x = 0."""
    s = np.asarray(s, dtype=np.float64)
    x = L * s
    small = x < 1.0
    a = np.empty(x.shape)
    b = np.empty(x.shape)
    if np.any(small):
        xs = x[small]
        x2 = xs * xs
        sa = np.zeros_like(xs)
        sb = np.zeros_like(xs)
        for m in range(1, 20):
            sa += ((-1.0) ** (m + 1)) * x2 ** (m - 1) / (4.0 ** m * math.factorial(m) ** 2)
        for m in range(0, 20):
            sb += ((-1.0) ** m) * x2 ** m / (2.0 ** (2 * m + 1) * math.factorial(m) * math.factorial(m + 1))
        a[small] = sa
        b[small] = sb
    big = ~small
    if np.any(big):
        xb = x[big]
        a[big] = (1.0 - sp.j0(xb)) / (xb * xb)
        b[big] = sp.j1(xb) / xb
    return L * L * (a - math.log(L) * b)


def _bessel_j_derivative(nu, m, x):
    """m-th derivative of J_nu at x: 2^-m sum_j (-1)^j C(m,j) J_{nu-m+2j}(x)."""
    acc = 0.0
    for j in range(m + 1):
        acc += ((-1.0) ** j) * math.comb(m, j) * sp.jv(nu - m + 2 * j, x)
    return acc / (2.0 ** m)


def helm2d_taylor_coeffs(k, L=1.5, nmax=24):
    """Coefficients c_n = N^(n)(k)/n!, n = 1..nmax, of the numerator of Table 2's
    2D Helmholtz transform, N(s) = 1 + (i pi/2) L [H0 s J_1(L s) - k H1 J_0(L s)]
    with H0 = H_0^(1)(L k), H1 = H_1^(1)(L k).  N(k) = 0 by the Wronskian, so
    G(s) = sum_n c_n (s - k)^(n-1) / (s + k) near s = k.

    Derivatives: v(s) = J_0(L s) has v^(n) = L^n J_0^(n)(L s); u(s) = s J_1(L s)
    has u^(n) = s L^n J_1^(n)(L s) + n L^(n-1) J_1^(n-1)(L s)."""
    x = L * k
    H0 = sp.hankel1(0, x)
    H1 = sp.hankel1(1, x)
    coeffs = []
    for n in range(1, nmax + 1):
        un = k * L ** n * _bessel_j_derivative(1, n, x) + n * L ** (n - 1) * _bessel_j_derivative(1, n - 1, x)
        vn = L ** n * _bessel_j_derivative(0, n, x)
        Nn = 0.5j * math.pi * L * (H0 * un - k * H1 * vn)
        coeffs.append(Nn / math.factorial(n))
    return np.asarray(coeffs, dtype=np.complex128)


# The printed quotient loses about eps k / |s - k| to cancellation (measured
# 2.8e-12 at k = 200, |s - k| = 1.2e-2), so the series covers |s - k| < 1,
# where the printed form is back to ~3e-14; 24 terms leave a remainder
# below (1.5)^25 / 25! relative.
HELM2D_WINDOW = 1.0


def g_helmholtz2d(s, k, L=1.5):
    """Table 2, operator Delta + k^2, kernel (i/4) H_0^(1)(k r):
        G(s) = [1 + (i pi/2) L s J_1(L s) H_0^(1)(L k)
                  - (i pi/2) L k J_0(L s) H_1^(1)(L k)] / (s^2 - k^2).
    Within |s - k| < 1 the quotient is replaced by its Taylor expansion
    about s = k (helm2d_taylor_coeffs), since numerator and denominator both
    vanish there.  Accuracy degrades like eps/(kL)^2 for kL << 1, where 1 and
    (i pi/2) L k H_1(L k) nearly cancel; the library documents k L >= 0.5."""
    s = np.asarray(s, dtype=np.float64)
    k = float(k)
    x = L * k
    H0 = sp.hankel1(0, x)
    H1 = sp.hankel1(1, x)
    out = np.empty(s.shape, dtype=np.complex128)
    near = np.abs(s - k) < HELM2D_WINDOW
    far = ~near
    if np.any(far):
        sf = s[far]
        num = 1.0 + 0.5j * math.pi * L * (sf * sp.j1(L * sf) * H0 - k * sp.j0(L * sf) * H1)
        out[far] = num / ((sf - k) * (sf + k))
    if np.any(near):
        sn = s[near]
        c = helm2d_taylor_coeffs(k, L)
        q = np.zeros(sn.shape, dtype=np.complex128)
        ds = sn - k
        for n in range(len(c) - 1, -1, -1):
            q = q * ds + c[n]
        out[near] = q / (sn + k)
    return out


def g_biharmonic3d(s, L=1.8):
    """Table 1, operator Delta^2, kernel r/(8 pi):
        G(s) = [(2 - x^2) cos x + 2 x sin x - 2] / (2 s^4),  x = L s.
    The radial integral is G = (1/(2s)) int_0^L r^2 sin(s r) dr; expanding
    sin(s r) and integrating term by term gives, for x < 1 (where the printed
    numerator cancels to O(x^4)),
        G = (L^4/2) sum_n (-1)^n x^(2n) / ((2n + 4) (2n + 1)!)   (G(0) = L^4/8)."""
    s = np.asarray(s, dtype=np.float64)
    x = L * s
    out = np.empty(s.shape)
    small = x < 1.0
    if np.any(small):
        xs = x[small]
        acc = np.zeros_like(xs)
        for n in range(14):
            acc += ((-1.0) ** n) * xs ** (2 * n) / ((2 * n + 4) * math.factorial(2 * n + 1))
        out[small] = 0.5 * L ** 4 * acc
    big = ~small
    if np.any(big):
        sb, xb = s[big], x[big]
        out[big] = ((2.0 - xb * xb) * np.cos(xb) + 2.0 * xb * np.sin(xb) - 2.0) / (2.0 * sb ** 4)
    return out


def g_biharmonic2d(s, L=1.5):
    """Table 2, operator Delta^2, kernel -(r^2/(8 pi))(log r - 1):
        G(s) = (J_0(x) - 1)/s^4 - L^3 (log L - 1) J_1(x)/(4 s)
               + L log L J_1(x)/s^3 - L^2 (2 log L - 1) J_0(x)/(4 s^2),  x = L s.
    The radial integral is G = -(1/4) int_0^L r^3 (log r - 1) J_0(s r) dr; with
    the power series of J_0 and int_0^L r^m (log r - 1) dr =
    L^(m+1) [(log L - 1)/(m+1) - 1/(m+1)^2], for x < 1 (where the printed terms
    cancel from O(s^-4) to O(1))
        G = -(L^4/4) sum_n (-1)^n (x/2)^(2n)/(n!)^2 [(log L - 1)/(2n+4) - 1/(2n+4)^2]."""
    s = np.asarray(s, dtype=np.float64)
    x = L * s
    lg = math.log(L)
    out = np.empty(s.shape)
    small = x < 1.0
    if np.any(small):
        xs = x[small]
        acc = np.zeros_like(xs)
        for n in range(16):
            m1 = 2 * n + 4
            acc += ((-1.0) ** n) * (0.5 * xs) ** (2 * n) / math.factorial(n) ** 2 * ((lg - 1.0) / m1 - 1.0 / m1 ** 2)
        out[small] = -0.25 * L ** 4 * acc
    big = ~small
    if np.any(big):
        sb, xb = s[big], x[big]
        J0, J1 = sp.j0(xb), sp.j1(xb)
        out[big] = ((J0 - 1.0) / sb ** 4 - L ** 3 * (lg - 1.0) * J1 / (4.0 * sb) + L * lg * J1 / sb ** 3
                    - L * L * (2.0 * lg - 1.0) * J0 / (4.0 * sb * sb))
    return out


KERNELS = ("laplace", "helmholtz", "biharmonic", "laplace_helmholtz")


def kernel_transform(d, kernel, s, k=0.0, L=None):
    """Dispatch G^L(s) for d in {2, 3} and the kernels of Tables 1-2:
    'laplace' (Delta), 'helmholtz' (Delta + k^2), 'biharmonic' (Delta^2) and
    'laplace_helmholtz' (Delta (Delta + k^2), G = G_k - G_0 as in both tables)."""
    if L is None:
        L = L_DEFAULT[d]
    if d == 3 and kernel == "laplace":
        return g_laplace3d(s, L).astype(np.complex128)
    if d == 3 and kernel == "helmholtz":
        return g_helmholtz3d(s, k, L)
    if d == 3 and kernel == "biharmonic":
        return g_biharmonic3d(s, L).astype(np.complex128)
    if d == 2 and kernel == "laplace":
        return g_laplace2d(s, L).astype(np.complex128)
    if d == 2 and kernel == "helmholtz":
        return g_helmholtz2d(s, k, L)
    if d == 2 and kernel == "biharmonic":
        return g_biharmonic2d(s, L).astype(np.complex128)
    if kernel == "laplace_helmholtz":
        return kernel_transform(d, "helmholtz", s, k, L) - kernel_transform(d, "laplace", s, k, L)
    raise ValueError(f"unsupported d={d} kernel={kernel}")


# ---------------------------------------------------------------------------
# Independent definitions used only to pin the closed forms above.

def radial_quadrature(d, kernel, s, k=0.0, L=None, points=None):
    """G^L(s) straight from the Section 2 radial integrals of the truncated
    kernel, by adaptive quadrature (scipy.integrate.quad):
        3D: (1/s) int_0^L sin(s r) g(r) 4 pi r dr, g = e^{ikr}/(4 pi r)
            -> (1/s) int_0^L sin(s r) e^{ikr} dr  (s -> 0 limit: int r e^{ikr} dr)
        2D: 2 pi int_0^L J_0(s r) g(r) r dr, g = -(1/2pi) log r or (i/4) H_0^(1)(k r).
    Real and imaginary parts are integrated separately."""
    from scipy import integrate

    if L is None:
        L = L_DEFAULT[d]
    s = float(s)
    if kernel == "laplace_helmholtz":
        return (radial_quadrature(d, "helmholtz", s, k, L, points)
                - radial_quadrature(d, "laplace", s, k, L, points))
    if kernel == "biharmonic":
        # 3D: g = r/(8 pi): (1/s) int_0^L sin(s r) (r/(8 pi)) 4 pi r dr; 2D: 2 pi int_0^L J_0(s r) g(r) r dr
        if d == 3:
            f = (lambda r: 0.5 * r ** 3) if s == 0.0 else (lambda r: 0.5 * r * r * math.sin(s * r) / s)
        else:
            f = lambda r: -0.25 * r ** 3 * (math.log(r) - 1.0) * sp.j0(s * r) if r > 0 else 0.0
        return complex(integrate.quad(f, 0.0, L, limit=400, epsabs=1e-15, epsrel=1e-14, points=points)[0], 0.0)
    if d == 3:
        if s == 0.0:
            fr = lambda r: r * math.cos(k * r)
            fi = lambda r: r * math.sin(k * r)
        else:
            fr = lambda r: math.sin(s * r) * math.cos(k * r) / s
            fi = lambda r: math.sin(s * r) * math.sin(k * r) / s
    else:
        if kernel == "laplace":
            fr = lambda r: -r * math.log(r) * sp.j0(s * r) if r > 0 else 0.0
            fi = lambda r: 0.0
        else:
            fr = lambda r: 2 * math.pi * r * sp.j0(s * r) * (-0.25 * sp.y0(k * r)) if r > 0 else 0.0
            fi = lambda r: 2 * math.pi * r * sp.j0(s * r) * (0.25 * sp.j0(k * r))
    lim = 400
    re = integrate.quad(fr, 0.0, L, limit=lim, epsabs=1e-15, epsrel=1e-14, points=points)[0]
    im = integrate.quad(fi, 0.0, L, limit=lim, epsabs=1e-15, epsrel=1e-14, points=points)[0]
    if d == 3 and kernel == "laplace":
        im = 0.0
        if s == 0.0:
            re = integrate.quad(lambda r: r, 0.0, L)[0]
        else:
            re = integrate.quad(lambda r: math.sin(s * r) / s, 0.0, L, limit=lim,
                                epsabs=1e-15, epsrel=1e-14)[0]
    return complex(re, im)
