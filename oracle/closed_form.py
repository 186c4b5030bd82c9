"""Potentials of a normalised Gaussian source, in FP64 (Section 5.1).

Test infrastructure (see the package docstring).

Source: rho(r) = (2 pi sigma^2)^(-d/2) exp(-r^2 / (2 sigma^2)), the Gaussians of
Section 5.1 (3D and 2D).  Potential u = g * rho with the free-space kernels
    3D: g = e^{ikr}/(4 pi r)        (k = 0: Laplace)
    2D: g = (i/4) H_0^(1)(k r)       (Table 2),   g = -(1/2pi) log r (Laplace).

Every formula here was derived for this oracle and checked against the radial
shell quadratures at the bottom of the file (which follow only from the kernel
and the source, not from the closed forms):
* 3D Laplace: u = erf(a)/(4 pi r), a = r/(sqrt(2) sigma) -- as printed.
* 3D Helmholtz: u = [e^{-b^2} e^{ikr} - e^{-a^2} Re w(b + i a)] / (4 pi r),
  b = k sigma / sqrt(2), w the Faddeeva function.  The printed Section 5.1
  formula is the negative of this (it fails the shell quadrature and the k -> 0
  limit to the Laplace case); this is the reading used.
* 2D Laplace: u = -[E_1(r^2/(2 sigma^2)) + log r^2] / (4 pi).  The printed "Ei"
  is read as the exponential integral E_1 (Ei itself diverges here).
* 2D Helmholtz: u = (i/(4 sigma^2)) [H_0(kr) int_0^r J_0(ky) e^{-y^2/2s^2} y dy
                                    + J_0(kr) int_r^inf H_0(ky) e^{-y^2/2s^2} y dy],
  H_0 = H_0^(1).  The printed prefactor lacks the factor i and writes H_0(kr)
  inside the second integral; both are read as above (Graf's addition theorem
  averaged over circles gives exactly this).
* 3D biharmonic (g = r/(8 pi)): u = [sigma sqrt(2/pi) e^{-a^2}
  + erf(a)(sigma^2/r + r)] / (8 pi).  The printed formula lacks the factor
  e^{-a^2} on the first term (it then exceeds the shell average by
  sigma sqrt(2/pi)(1 - e^{-a^2})/(8 pi)); this is the reading used.
* 2D biharmonic (g = -(r^2/(8 pi))(log r - 1)): u = -(sigma^2/(8 pi))
  [(x + 1) Ein(x) - e^{-x}] + c_2 r^2 + c_1, x = r^2/(2 sigma^2),
  Ein(x) = E_1(x) + log x + gamma, c_1, c_2 as printed.  The printed "Ei" is
  read as E_1 (as for the 2D Laplace case) and the printed "c_1 r" as the
  constant c_1 (its units are those of r^2; with these readings the formula
  equals the circle-average integral below).
* Delta (Delta + k^2) (g = g_k - g_0, the difference whose transform is the
  tables' G_k - G_0): u = u_k - u_0.
"""
from __future__ import annotations

import math

import numpy as np
from scipy import special as sp
from scipy import integrate

SQRT2 = math.sqrt(2.0)
SQRTPI = math.sqrt(math.pi)


# ----------------------------------------------------------------- 3D ------

def u_laplace3d(r, sigma):
    r = np.asarray(r, dtype=np.float64)
    a = r / (SQRT2 * sigma)
    safe = np.where(r > 0, r, 1.0)
    val = sp.erf(a) / (4 * math.pi * safe)
    u0 = math.sqrt(2.0 / math.pi) / (4 * math.pi * sigma)
    small = a < 1e-5
    # erf(a)/r = (2/sqrt(pi)) (1 - a^2/3) / (sqrt2 sigma) + O(a^4)
    ser = u0 * (1.0 - a * a / 3.0)
    return np.where(small, ser, val)


def du_laplace3d(r, sigma):
    """du/dr = [sqrt(2/pi)(r/sigma) e^{-a^2} - erf(a)] / (4 pi r^2)."""
    r = np.asarray(r, dtype=np.float64)
    a = r / (SQRT2 * sigma)
    safe = np.where(r > 0, r, 1.0)
    val = (math.sqrt(2.0 / math.pi) * (r / sigma) * np.exp(-a * a) - sp.erf(a)) / (4 * math.pi * safe ** 2)
    # small r: u ~ u0 (1 - a^2/3) -> du/dr ~ -u0 * 2 a /(3 sqrt2 sigma)
    u0 = math.sqrt(2.0 / math.pi) / (4 * math.pi * sigma)
    ser = -u0 * 2.0 * a / (3.0 * SQRT2 * sigma)
    return np.where(a < 1e-4, ser, val)


def u_helmholtz3d(r, sigma, k):
    r = np.asarray(r, dtype=np.float64)
    a = r / (SQRT2 * sigma)
    b = k * sigma / SQRT2
    safe = np.where(r > 0, r, 1.0)
    Nf = np.exp(-b * b) * np.exp(1j * k * r) - np.exp(-a * a) * np.real(sp.wofz(b + 1j * a))
    val = Nf / (4 * math.pi * safe)
    # r -> 0: u(0) = [i k e^{-b^2} + sqrt(2/pi)(1 - 2 b F(b))/sigma] / (4 pi),
    # F = Dawson's integral.
    u0 = (1j * k * math.exp(-b * b) + math.sqrt(2.0 / math.pi) * (1.0 - 2.0 * b * sp.dawsn(b)) / sigma) / (4 * math.pi)
    return np.where(a < 1e-7, u0, val)


def du_helmholtz3d(r, sigma, k):
    """du/dr = (N' r - N)/(4 pi r^2), N = 4 pi r u,
    N' = i k e^{-b^2} e^{ikr} - e^{-a^2} (2 b Im w(z) - 2/sqrt(pi)) / (sqrt2 sigma)."""
    r = np.asarray(r, dtype=np.float64)
    a = r / (SQRT2 * sigma)
    b = k * sigma / SQRT2
    safe = np.where(r > 0, r, 1.0)
    w = sp.wofz(b + 1j * a)
    Nf = np.exp(-b * b) * np.exp(1j * k * r) - np.exp(-a * a) * np.real(w)
    Np = 1j * k * np.exp(-b * b) * np.exp(1j * k * r) - np.exp(-a * a) * (2 * b * np.imag(w) - 2 / SQRTPI) / (SQRT2 * sigma)
    val = (Np * safe - Nf) / (4 * math.pi * safe ** 2)
    return np.where(a < 1e-6, 0.0 * val, val)


# ----------------------------------------------------------------- 2D ------

def u_laplace2d(r, sigma):
    r = np.asarray(r, dtype=np.float64)
    x = r * r / (2 * sigma * sigma)
    # -[E1(x) + log r^2]/(4pi) = -[-gamma + log(2 sigma^2) + Ein(x)]/(4pi),
    # Ein(x) = E1(x) + gamma + log x; the second form is used for small x.
    safe = np.where(x > 0, x, 1.0)
    big = -(sp.exp1(safe) + np.log(np.where(r > 0, r * r, 1.0))) / (4 * math.pi)
    ein = np.zeros_like(x)
    for n in range(1, 40):
        ein = ein + ((-1.0) ** (n + 1)) * x ** n / (n * math.factorial(n))
    small_val = -(-np.euler_gamma + math.log(2 * sigma * sigma) + ein) / (4 * math.pi)
    return np.where(x < 0.5, small_val, big)


def du_laplace2d(r, sigma):
    """du/dr = -(1 - e^{-r^2/2 sigma^2}) / (2 pi r)."""
    r = np.asarray(r, dtype=np.float64)
    x = r * r / (2 * sigma * sigma)
    safe = np.where(r > 0, r, 1.0)
    return np.where(r > 0, -(-np.expm1(-x)) / (2 * math.pi * safe), 0.0)


def _quad_c(fr, fi, a, b):
    kw = dict(limit=400, epsabs=1e-16, epsrel=1e-13)
    return complex(integrate.quad(fr, a, b, **kw)[0], integrate.quad(fi, a, b, **kw)[0])


def _helm2d_parts(r, sigma, k):
    e = lambda y: math.exp(-y * y / (2 * sigma * sigma)) * y
    ymax = sigma * 40.0
    I1 = _quad_c(lambda y: sp.j0(k * y) * e(y), lambda y: 0.0, 0.0, r) if r > 0 else 0.0
    if r < ymax:
        I2 = _quad_c(lambda y: sp.j0(k * y) * e(y), lambda y: sp.y0(k * y) * e(y), r, ymax)
    else:
        I2 = 0.0
    return I1, I2


def u_helmholtz2d(r, sigma, k):
    """Evaluated by adaptive quadrature of the two radial integrals."""
    out = []
    for rv in np.atleast_1d(np.asarray(r, dtype=np.float64)):
        I1, I2 = _helm2d_parts(float(rv), sigma, k)
        H0 = sp.hankel1(0, k * rv) if rv > 0 else 0.0
        out.append((1j / (4 * sigma * sigma)) * (H0 * I1 + sp.j0(k * rv) * I2))
    return np.asarray(out)


def du_helmholtz2d(r, sigma, k):
    """du/dr = (i/(4 sigma^2)) [-k H_1(kr) I_1(r) - k J_1(kr) I_2(r)]."""
    out = []
    for rv in np.atleast_1d(np.asarray(r, dtype=np.float64)):
        I1, I2 = _helm2d_parts(float(rv), sigma, k)
        H1 = sp.hankel1(1, k * rv) if rv > 0 else 0.0
        out.append((1j / (4 * sigma * sigma)) * (-k * H1 * I1 - k * sp.j1(k * rv) * I2))
    return np.asarray(out)


# ---------------------------------------------------------- biharmonic ----

def u_biharmonic3d(r, sigma):
    r = np.asarray(r, dtype=np.float64)
    a = r / (SQRT2 * sigma)
    safe = np.where(r > 0, r, 1.0)
    val = (sigma * math.sqrt(2.0 / math.pi) * np.exp(-a * a) + sp.erf(a) * (sigma * sigma / safe + r)) / (8 * math.pi)
    # r -> 0: erf(a) sigma^2 / r -> sigma sqrt(2/pi) (1 - a^2/3), so
    # u ~ [2 sigma sqrt(2/pi) + O(r^2)] / (8 pi)
    u0 = 2.0 * sigma * math.sqrt(2.0 / math.pi) / (8 * math.pi)
    return np.where(a < 1e-6, u0, val)


def du_biharmonic3d(r, sigma):
    """du/dr = [sqrt(2/pi) (sigma/r) e^{-a^2} + erf(a)(1 - sigma^2/r^2)] / (8 pi)."""
    r = np.asarray(r, dtype=np.float64)
    a = r / (SQRT2 * sigma)
    safe = np.where(r > 0, r, 1.0)
    val = (math.sqrt(2.0 / math.pi) * (sigma / safe) * np.exp(-a * a) + sp.erf(a) * (1.0 - sigma * sigma / safe ** 2)) / (8 * math.pi)
    return np.where(a < 1e-4, 0.0, val)


def _ein(x):
    """Ein(x) = E_1(x) + log x + gamma = sum_{n>=1} (-1)^(n+1) x^n / (n n!)."""
    x = np.asarray(x, dtype=np.float64)
    safe = np.where(x > 0, x, 1.0)
    big = sp.exp1(safe) + np.log(safe) + np.euler_gamma
    ser = np.zeros_like(x)
    for n in range(1, 40):
        ser = ser + ((-1.0) ** (n + 1)) * x ** n / (n * math.factorial(n))
    return np.where(x < 0.5, ser, big)


def _bih2d_consts(sigma):
    lg = math.log(1.0 / (2 * sigma * sigma))
    c1 = sigma * sigma / (8 * math.pi) * (np.euler_gamma + lg)
    c2 = (0.5 * np.euler_gamma + 0.5 * lg + 1.0) / (8 * math.pi)
    return c1, c2


def u_biharmonic2d(r, sigma):
    r = np.asarray(r, dtype=np.float64)
    x = r * r / (2 * sigma * sigma)
    c1, c2 = _bih2d_consts(sigma)
    return -(sigma * sigma / (8 * math.pi)) * ((x + 1.0) * _ein(x) - np.exp(-x)) + c2 * r * r + c1


def du_biharmonic2d(r, sigma):
    """du/dr = -(r/(8 pi)) [Ein(x) + 1 + (1 - e^{-x})/x] + 2 c_2 r, using
    Ein'(x) = (1 - e^{-x})/x."""
    r = np.asarray(r, dtype=np.float64)
    x = r * r / (2 * sigma * sigma)
    c1, c2 = _bih2d_consts(sigma)
    safe = np.where(x > 0, x, 1.0)
    q = np.where(x > 1e-8, -np.expm1(-safe) / safe, 1.0 - 0.5 * x)
    return -(r / (8 * math.pi)) * (_ein(x) + 1.0 + q) + 2.0 * c2 * r


# ------------------------------------------------------- sources on grids --

def potential(d, kernel, k, r, sigma):
    if kernel == "laplace_helmholtz":
        return potential(d, "helmholtz", k, r, sigma) - potential(d, "laplace", k, r, sigma)
    if d == 3:
        if kernel == "biharmonic":
            return u_biharmonic3d(r, sigma).astype(np.complex128)
        return u_laplace3d(r, sigma).astype(np.complex128) if kernel == "laplace" else u_helmholtz3d(r, sigma, k)
    if kernel == "biharmonic":
        return u_biharmonic2d(r, sigma).astype(np.complex128)
    return u_laplace2d(r, sigma).astype(np.complex128) if kernel == "laplace" else u_helmholtz2d(r, sigma, k)


def dpotential(d, kernel, k, r, sigma):
    if kernel == "laplace_helmholtz":
        return dpotential(d, "helmholtz", k, r, sigma) - dpotential(d, "laplace", k, r, sigma)
    if d == 3:
        if kernel == "biharmonic":
            return du_biharmonic3d(r, sigma).astype(np.complex128)
        return du_laplace3d(r, sigma).astype(np.complex128) if kernel == "laplace" else du_helmholtz3d(r, sigma, k)
    if kernel == "biharmonic":
        return du_biharmonic2d(r, sigma).astype(np.complex128)
    return du_laplace2d(r, sigma).astype(np.complex128) if kernel == "laplace" else du_helmholtz2d(r, sigma, k)


def gaussian_sum_potential(d, kernel, k, centers, sigmas, amps, points):
    """u(x) = sum_j amp_j u_{sigma_j}(|x - c_j|) at points (P, d)."""
    points = np.asarray(points, dtype=np.float64)
    out = np.zeros(len(points), dtype=np.complex128)
    for j in range(len(sigmas)):
        r = np.linalg.norm(points - centers[j][None, :], axis=1)
        out += amps[j] * potential(d, kernel, k, r, float(sigmas[j]))
    return out


def gaussian_sum_gradient(d, kernel, k, centers, sigmas, amps, points):
    """grad u at points, shape (d, P)."""
    points = np.asarray(points, dtype=np.float64)
    out = np.zeros((d, len(points)), dtype=np.complex128)
    for j in range(len(sigmas)):
        diff = points - centers[j][None, :]
        r = np.linalg.norm(diff, axis=1)
        du = dpotential(d, kernel, k, r, float(sigmas[j]))
        safe = np.where(r > 0, r, 1.0)
        for ax in range(d):
            out[ax] += amps[j] * du * np.where(r > 0, diff[:, ax] / safe, 0.0)
    return out


# ------------------------------------------- independent shell quadratures --

def shell_quadrature_3d(r, sigma, k):
    """u(r) from the shell theorem: the average of e^{ik|x-y|}/(4 pi |x-y|) over
    a sphere |y| = t seen from |x| = r is (e^{ik(r+t)} - e^{ik|r-t|})/(8 pi i k r t)
    (the Laplace limit k -> 0 gives 1/(4 pi max(r, t))), so
        u(r) = int_0^inf rho(t) 4 pi t^2 <g>_t dt."""
    rho = lambda t: (2 * math.pi * sigma ** 2) ** -1.5 * math.exp(-t * t / (2 * sigma * sigma))
    tmax = 40 * sigma
    if k == 0.0:
        f = lambda t: rho(t) * 4 * math.pi * t * t / (4 * math.pi * max(r, t))
        pts = [r] if 0 < r < tmax else None
        return complex(integrate.quad(f, 0, tmax, points=pts, limit=400, epsabs=1e-16, epsrel=1e-13)[0], 0.0)

    def avg(t):
        if r == 0.0:
            return np.exp(1j * k * t) / (4 * math.pi * t) if t > 0 else 0.0
        return (np.exp(1j * k * (r + t)) - np.exp(1j * k * abs(r - t))) / (8j * math.pi * k * r * t)

    fr = lambda t: float(np.real(rho(t) * 4 * math.pi * t * t * avg(t))) if t > 0 else 0.0
    fi = lambda t: float(np.imag(rho(t) * 4 * math.pi * t * t * avg(t))) if t > 0 else 0.0
    pts = [r] if 0 < r < tmax else None
    kw = dict(points=pts, limit=400, epsabs=1e-16, epsrel=1e-13)
    return complex(integrate.quad(fr, 0, tmax, **kw)[0], integrate.quad(fi, 0, tmax, **kw)[0])


def shell_quadrature_2d_laplace(r, sigma):
    """u(r) = -int_0^inf rho(t) 2 pi t log(max(r, t)) dt / (2 pi): the circle
    average of log|x - y| over |y| = t is log max(|x|, t)."""
    rho = lambda t: math.exp(-t * t / (2 * sigma * sigma)) / (2 * math.pi * sigma * sigma)
    tmax = 40 * sigma
    f = lambda t: -rho(t) * t * math.log(max(r, t)) if max(r, t) > 0 else 0.0
    pts = [r] if 0 < r < tmax else None
    return integrate.quad(f, 0, tmax, points=pts, limit=400, epsabs=1e-16, epsrel=1e-13)[0]


def shell_quadrature_3d_biharmonic(r, sigma, derivative=False):
    """u(r) (or du/dr) for g = r/(8 pi): the average of |x - y| over the sphere
    |y| = t seen from |x| = r is r + t^2/(3r) for t < r and t + r^2/(3t) for
    t > r (d/dr: 1 - t^2/(3r^2) and 2r/(3t))."""
    rho = lambda t: (2 * math.pi * sigma ** 2) ** -1.5 * math.exp(-t * t / (2 * sigma * sigma))
    if derivative:
        avg = lambda t: (1.0 - t * t / (3 * r * r)) if t < r else 2.0 * r / (3.0 * t)
    else:
        avg = lambda t: (r + t * t / (3 * r)) if t < r else (t + r * r / (3 * t))
    f = lambda t: rho(t) * 4 * math.pi * t * t * avg(t) / (8 * math.pi)
    tmax = 40 * sigma
    pts = [r] if 0 < r < tmax else None
    return integrate.quad(f, 0, tmax, points=pts, limit=400, epsabs=1e-17, epsrel=1e-13)[0]


def circle_quadrature_2d_biharmonic(r, sigma, derivative=False):
    """u(r) (or du/dr) for g = -(R^2/(8 pi))(log R - 1), R = |x - y|: the circle
    average of R^2 log R over |y| = t is r^2 log r + t^2 (log r + 1) for t < r
    and t^2 log t + r^2 (log t + 1) for t > r (it solves the radial Poisson
    equation with source 4 log max(r, t) + 4, the average of the Laplacian);
    the average of R^2 is r^2 + t^2."""
    rho = lambda t: math.exp(-t * t / (2 * sigma * sigma)) / (2 * math.pi * sigma * sigma)

    def avg(t):
        if derivative:
            return (-(2 * r * math.log(r) - r + t * t / r) if t < r else -(2 * r * math.log(t))) / (8 * math.pi)
        if t < r:
            M = r * r * math.log(r) + t * t * (math.log(r) + 1.0)
        else:
            M = t * t * math.log(t) + r * r * (math.log(t) + 1.0)
        return -(M - (r * r + t * t)) / (8 * math.pi)

    f = lambda t: rho(t) * 2 * math.pi * t * avg(t) if t > 0 else 0.0
    tmax = 40 * sigma
    pts = [r] if 0 < r < tmax else None
    return integrate.quad(f, 0, tmax, points=pts, limit=400, epsabs=1e-17, epsrel=1e-13)[0]
