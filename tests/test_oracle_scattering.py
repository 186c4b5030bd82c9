"""Pins for the oracle's Lippmann-Schwinger reference solve (Section 5.3)."""
import numpy as np

from oracle import operator as op
from oracle import scattering as sc
from workloads.scattering import contrast, plane_wave


def test_direct_solution_satisfies_the_equation():
    k = 10.0
    for d, N, name in ((2, 24, "smoothed_disk"), (3, 8, "smoothed_cube"), (2, 20, "luneburg")):
        pl = op.Plan(d, N, "helmholtz", k)
        q, pin = contrast(name, N), plane_wave(d, N, k)
        s = sc.ls_solve_direct(pl, q, pin)
        assert sc.ls_relative_residual(pl, q, pin, s) < 1e-12


def test_born_limit_fixes_sign_and_scale():
    """For a weak contrast eps q the density is sigma = k^2 eps q phi_in + O(eps^2)
    (first Born approximation of -sigma + k^2 q (T sigma) = -k^2 q phi_in)."""
    k, N = 10.0, 16
    pl = op.Plan(2, N, "helmholtz", k)
    pin = plane_wave(2, N, k)
    errs = []
    for eps in (1e-3, 1e-4):
        q = eps * contrast("smoothed_disk", N)
        born = k * k * q * pin
        s = sc.ls_solve_direct(pl, q, pin)
        errs.append(np.linalg.norm(s - born) / np.linalg.norm(born))
    assert errs[1] < 2e-4
    assert 8.0 < errs[0] / errs[1] < 12.0  # first-order remainder


def test_self_convergence_under_refinement():
    """The N and 2N solutions agree on the shared points (2N-grid index 2a + 1)
    to the spectral accuracy the smooth contrast allows."""
    k = 10.0
    sols = {}
    for N in (24, 48):
        pl = op.Plan(2, N, "helmholtz", k)
        sols[N] = sc.ls_solve_direct(pl, contrast("smoothed_disk", N), plane_wave(2, N, k))
    coarse, fine = sols[24], sols[48][1::2, 1::2]
    assert np.linalg.norm(coarse - fine) / np.linalg.norm(fine) < 1e-4
