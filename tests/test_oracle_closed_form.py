"""Pins for the Gaussian-source closed forms (Section 5.1) used as end-to-end
references: each is compared with a radial quadrature that follows only from
the kernel and the source (shell averages in 3D, circle averages in 2D), at
radii inside, near and far from the source width."""
import numpy as np
import pytest

from oracle import closed_form as cf

SIGMA = 0.05
RADII = [1e-3, 0.02, 0.05, 0.08, 0.15, 0.4, 0.9]


@pytest.mark.parametrize("k", [0.0, 2.0, 20.0])
def test_3d_laplace_helmholtz_against_shell_average(k):
    for r in RADII:
        ref = cf.shell_quadrature_3d(r, SIGMA, k)
        got = complex(cf.potential(3, "laplace" if k == 0 else "helmholtz", k, np.array([r]), SIGMA)[0])
        assert abs(got - ref) <= 1e-11 * abs(ref), (r, got, ref)


def test_2d_laplace_against_circle_average():
    for r in RADII:
        ref = cf.shell_quadrature_2d_laplace(r, SIGMA)
        got = float(cf.u_laplace2d(np.array([r]), SIGMA)[0])
        assert abs(got - ref) <= 1e-11 * abs(ref), (r, got, ref)


def test_biharmonic_against_shell_and_circle_averages():
    for r in RADII:
        for deriv in (False, True):
            ref3 = cf.shell_quadrature_3d_biharmonic(r, SIGMA, deriv)
            got3 = float((cf.du_biharmonic3d if deriv else cf.u_biharmonic3d)(np.array([r]), SIGMA)[0])
            assert abs(got3 - ref3) <= 1e-11 * abs(ref3), ("3d", deriv, r, got3, ref3)
            ref2 = cf.circle_quadrature_2d_biharmonic(r, SIGMA, deriv)
            got2 = float((cf.du_biharmonic2d if deriv else cf.u_biharmonic2d)(np.array([r]), SIGMA)[0])
            assert abs(got2 - ref2) <= 1e-11 * abs(ref2), ("2d", deriv, r, got2, ref2)


def test_biharmonic_3d_printed_form_differs_by_the_missing_exponential():
    """Section 5.1 prints sigma sqrt(2/pi) without e^{-r^2/(2 sigma^2)}: it
    agrees with the shell average only at r = 0 and exceeds it by
    sigma sqrt(2/pi)(1 - e^{-a^2})/(8 pi) elsewhere."""
    from scipy import special as sp
    for r in (0.05, 0.3):
        a = r / (np.sqrt(2) * SIGMA)
        printed = (SIGMA * np.sqrt(2 / np.pi) + sp.erf(a) * (SIGMA ** 2 / r + r)) / (8 * np.pi)
        ref = cf.shell_quadrature_3d_biharmonic(r, SIGMA)
        excess = SIGMA * np.sqrt(2 / np.pi) * (1 - np.exp(-a * a)) / (8 * np.pi)
        assert abs((printed - ref) - excess) <= 1e-12 * ref


def test_2d_biharmonic_brute_force_area_integral():
    """One point against a direct 2D integral of g_b(|x - y|) rho(y) dy in polar
    coordinates about the source (independent of the circle-average formula)."""
    from scipy import integrate
    r = 0.07
    gb = lambda R: -(R * R / (8 * np.pi)) * (np.log(R) - 1.0) if R > 0 else 0.0
    rho = lambda t: np.exp(-t * t / (2 * SIGMA ** 2)) / (2 * np.pi * SIGMA ** 2)
    inner = lambda t: integrate.quad(lambda th: gb(np.sqrt(r * r + t * t - 2 * r * t * np.cos(th))), 0, 2 * np.pi,
                                     limit=200, epsabs=1e-14, epsrel=1e-11)[0]
    ref = integrate.quad(lambda t: rho(t) * t * inner(t), 0, 12 * SIGMA, points=[r], limit=200,
                         epsabs=1e-15, epsrel=1e-10)[0]
    assert abs(float(cf.u_biharmonic2d(np.array([r]), SIGMA)[0]) - ref) <= 1e-8 * abs(ref)
