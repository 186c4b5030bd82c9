"""Pins for the oracle's truncated-kernel transforms (Tables 1 and 2).

Each closed form is checked against the Section 2 radial integral of the
truncated kernel evaluated by adaptive quadrature (a definition independent of
the closed form), at ordinary points, at s = 0, straddling s = k (where the
printed forms are 0/0), and against limits derived by hand.
"""
import math

import numpy as np
import pytest
from scipy import special as sp

from oracle import greens as g

CASES = [
    (3, "laplace", 0.0),
    (3, "helmholtz", 20.0),
    (3, "helmholtz", 2.0),
    (3, "helmholtz", 0.4),      # k L < 1: series region
    (2, "laplace", 0.0),
    (2, "helmholtz", 2.0),
    (2, "helmholtz", 200.0),
    (3, "biharmonic", 0.0),
    (2, "biharmonic", 0.0),
    (3, "laplace_helmholtz", 7.0),
    (2, "laplace_helmholtz", 30.0),
]


def _points(k):
    base = [0.0, 1e-9, 1e-5, 0.01, 0.3, 0.9, 1.7, 3.3, 12.0, 47.5, 131.0]
    if k > 0:
        base += [k, k * (1 - 1e-9), k * (1 + 1e-9), k - 0.004, k + 0.02, 0.5 * k, 1.5 * k, 0.49 * k, 1.51 * k]
    return base


@pytest.mark.parametrize("d,kernel,k", CASES)
def test_closed_form_matches_radial_quadrature(d, kernel, k):
    scale = abs(complex(g.kernel_transform(d, kernel, np.array([0.0]), k)[0]))
    for s in _points(k):
        got = complex(g.kernel_transform(d, kernel, np.array([s]), k)[0])
        ref = g.radial_quadrature(d, kernel, s, k)
        assert abs(got - ref) <= 2e-12 * max(abs(ref), 1e-3 * scale), (s, got, ref)


def test_laplace3d_printed_form_and_limit():
    L = 1.8
    s = np.array([0.2, 1.0, 5.0, 17.0])
    printed = 2 * (np.sin(L * s / 2) / s) ** 2          # Table 1 as printed
    assert np.allclose(g.g_laplace3d(s, L), printed, rtol=1e-14, atol=0)
    assert g.g_laplace3d(np.array([0.0]), L)[0] == pytest.approx(L * L / 2, rel=1e-15)


def test_helmholtz3d_limits_and_laplace_continuity():
    L = 1.8
    for k in (0.7, 3.0, 20.0):
        # s = 0: [e^{ikL}(1 - ikL) - 1]/k^2 ; s = k: (1 - e^{2ikL})/(4k^2) + iL/(2k)
        g0 = (np.exp(1j * k * L) * (1 - 1j * k * L) - 1) / k ** 2
        gk = (1 - np.exp(2j * k * L)) / (4 * k * k) + 1j * L / (2 * k)
        assert abs(g.g_helmholtz3d(np.array([0.0]), k, L)[0] - g0) < 1e-13 * abs(g0)
        assert abs(g.g_helmholtz3d(np.array([k]), k, L)[0] - gk) < 1e-13 * abs(gk)
    # k -> 0 tends to the Laplace transform
    s = np.linspace(0, 30, 61)
    # (the difference is i k int_0^L r sin(sr)/s dr + O(k^2), so linear in k)
    d1 = np.max(np.abs(g.g_helmholtz3d(s, 1e-6, L) - g.g_laplace3d(s, L)))
    d2 = np.max(np.abs(g.g_helmholtz3d(s, 1e-8, L) - g.g_laplace3d(s, L)))
    assert d1 < 1e-6 * L ** 3
    assert d2 == pytest.approx(d1 / 100, rel=1e-3)


def test_helmholtz3d_printed_form_far_from_k():
    L, k = 1.8, 20.0
    s = np.array([1.0, 5.0, 35.0, 80.0])
    printed = (-1 + np.exp(1j * L * k) * (np.cos(L * s) - 1j * (k / s) * np.sin(L * s))) / ((k - s) * (k + s))
    assert np.allclose(g.g_helmholtz3d(s, k, L), printed, rtol=1e-13, atol=0)


def test_laplace2d_printed_form_and_limit():
    L = 1.5
    s = np.array([1.0, 4.0, 33.0])
    printed = (1 - sp.j0(L * s)) / s ** 2 - L * math.log(L) * sp.j1(L * s) / s
    assert np.allclose(g.g_laplace2d(s, L), printed, rtol=1e-13, atol=0)
    g0 = L * L / 4 * (1 - 2 * math.log(L))
    assert g.g_laplace2d(np.array([0.0]), L)[0] == pytest.approx(g0, rel=1e-15)


def test_helmholtz2d_value_at_k_wronskian_limit():
    L = 1.5
    for k in (2.0, 37.0, 200.0):
        x = k * L
        gk = 0.25j * math.pi * L * L * (sp.j0(x) * sp.hankel1(0, x) + sp.j1(x) * sp.hankel1(1, x))
        got = g.g_helmholtz2d(np.array([k]), k, L)[0]
        assert abs(got - gk) < 1e-13 * abs(gk)
        # both sides of the Taylor window join continuously
        w = g.HELM2D_WINDOW
        inside = g.g_helmholtz2d(np.array([k + 0.999999 * w]), k, L)[0]
        outside = g.g_helmholtz2d(np.array([k + 1.000001 * w]), k, L)[0]
        slope = abs(g.g_helmholtz2d(np.array([k + 1.1 * w]), k, L)[0] - outside) / (0.1 * w)
        assert abs(inside - outside) < 1e-12 * abs(gk) + 3e-6 * w * slope


def test_helmholtz2d_printed_form_far_from_k():
    L, k = 1.5, 20.0
    s = np.array([0.5, 7.0, 31.0, 90.0])
    num = 1 + 0.5j * math.pi * L * s * sp.j1(L * s) * sp.hankel1(0, L * k) \
        - 0.5j * math.pi * L * k * sp.j0(L * s) * sp.hankel1(1, L * k)
    assert np.allclose(g.g_helmholtz2d(s, k, L), num / (s * s - k * k), rtol=1e-13, atol=0)


def test_truncated_spectrum_tends_to_free_space_spectrum():
    """Figure 1: away from s = 0 (and s = k) the truncated transforms oscillate
    about the free-space symbol 1/(s^2 - k^2), with an amplitude that decays
    with s."""
    s = np.linspace(30.0, 60.0, 301)
    lap = g.g_laplace3d(s)
    assert np.max(np.abs(lap * s * s - 1.0)) <= 1.0 + 1e-12  # G s^2 - 1 = -cos(Ls)
    assert np.mean(lap * s * s) == pytest.approx(1.0, abs=0.05)
    k = 4.0
    hel = g.g_helmholtz3d(s, k)
    assert np.mean((hel * (s * s - k * k)).real) == pytest.approx(1.0, abs=0.05)


def test_biharmonic_printed_forms_limits_and_series_crossover():
    """Table 1 and Table 2 biharmonic transforms as printed (away from s = 0),
    their s = 0 values (3D: L^4/8; 2D: -(L^4/4)[(log L - 1)/4 - 1/16]) and
    continuity where the oracle switches from the series to the printed form
    (L s = 1)."""
    L3, L2 = 1.8, 1.5
    s = np.array([0.7, 2.0, 9.0, 40.0])
    x = L3 * s
    printed3 = ((2 - x * x) * np.cos(x) + 2 * x * np.sin(x) - 2) / (2 * s ** 4)
    assert np.allclose(g.g_biharmonic3d(s, L3), printed3, rtol=1e-12, atol=0)
    x = L2 * s
    lg = math.log(L2)
    printed2 = ((sp.j0(x) - 1) / s ** 4 - L2 ** 3 * (lg - 1) * sp.j1(x) / (4 * s) + L2 * lg * sp.j1(x) / s ** 3
                - L2 ** 2 * (2 * lg - 1) * sp.j0(x) / (4 * s * s))
    assert np.allclose(g.g_biharmonic2d(s, L2), printed2, rtol=1e-12, atol=0)
    assert g.g_biharmonic3d(np.array([0.0]), L3)[0] == pytest.approx(L3 ** 4 / 8, rel=1e-15)
    assert g.g_biharmonic2d(np.array([0.0]), L2)[0] == pytest.approx(-(L2 ** 4 / 4) * ((lg - 1) / 4 - 1 / 16), rel=1e-15)
    for L, fn in ((L3, g.g_biharmonic3d), (L2, g.g_biharmonic2d)):
        a, b = fn(np.array([(1 - 1e-14) / L, (1 + 1e-14) / L]), L)
        assert abs(a - b) <= 1e-13 * abs(a)


def test_laplace_helmholtz_is_difference_and_vanishes_as_k_to_0():
    """Delta(Delta + k^2): both tables give G_k - G_0; in 3D it tends to 0 with k."""
    s = np.linspace(0, 40, 81)
    for d in (2, 3):
        diff = g.kernel_transform(d, "helmholtz", s, 9.0) - g.kernel_transform(d, "laplace", s, 0.0)
        assert np.array_equal(g.kernel_transform(d, "laplace_helmholtz", s, 9.0), diff)
    small = g.kernel_transform(3, "laplace_helmholtz", s, 1e-4)
    assert np.max(np.abs(small)) < 1e-3


def test_helmholtz2d_near_shell_against_high_precision():
    """The stable evaluation next to s = k, where Table 2's quotient is 0/0,
    against the printed form evaluated with 40 significant digits (mpmath),
    for wavenumbers from kL < 1 to kL = 1500: pointwise relative error below
    2e-13 on both sides of the Taylor window's edge (1.3e-13 at k = 1000 just
    outside it, where the printed form has lost about eps k)."""
    mp = pytest.importorskip("mpmath")
    mp.mp.dps = 40
    L = 1.5
    for k in (0.5, 2.0, 37.0, 200.0, 1000.0):
        ds = np.array([-3.0, -1.0001, -0.9999, -0.3, -1e-2, -1e-4, 0.0, 1e-4, 1e-2, 0.3, 0.9999, 1.0001, 3.0])
        s = k + ds
        s = s[s > 0]
        got = g.g_helmholtz2d(s, k, L)
        x = L * mp.mpf(k)
        H0, H1 = mp.hankel1(0, x), mp.hankel1(1, x)
        for sv, gv in zip(s, got):
            sm = mp.mpf(float(sv))
            if sm == mp.mpf(k):
                exact = 0.25j * mp.pi * L * L * (mp.besselj(0, x) * H0 + mp.besselj(1, x) * H1)
            else:
                num = 1 + 0.5j * mp.pi * L * (sm * mp.besselj(1, L * sm) * H0 - k * mp.besselj(0, L * sm) * H1)
                exact = num / ((sm - k) * (sm + k))
            exact = complex(exact)
            assert abs(gv - exact) <= 2e-13 * abs(exact), (k, sv - k)
