"""Lippmann-Schwinger reference solutions (Section 5.3), FP64.

Test infrastructure (see the package docstring).

The dual Lippmann-Schwinger equation for the density sigma of the scattered
field phi_s = g_k * sigma is
    A sigma := -sigma + k^2 q (T sigma) = -k^2 q phi_in,
with T the truncated-kernel convolution of an oracle Helmholtz plan.  Here A
is formed densely, column by column from T applied to unit vectors, and the
system is solved by LU (numpy.linalg.solve): slow, exact to rounding, for
small grids only (N^d up to a few thousand unknowns).
"""
from __future__ import annotations

import numpy as np


def ls_rhs(plan, q, phi_in):
    return -(plan.k ** 2) * q * phi_in


def ls_operator(plan, q, sigma):
    """A sigma = -sigma + k^2 q (T sigma)."""
    return -sigma + (plan.k ** 2) * q * plan.apply(sigma)


def ls_dense_matrix(plan, q):
    shape = (plan.N,) * plan.d
    n = int(np.prod(shape))
    A = np.empty((n, n), dtype=np.complex128)
    e = np.zeros(n, dtype=np.complex128)
    for j in range(n):
        e[j] = 1.0
        A[:, j] = ls_operator(plan, q, e.reshape(shape)).ravel()
        e[j] = 0.0
    return A


def ls_solve_direct(plan, q, phi_in):
    """sigma solving A sigma = -k^2 q phi_in exactly (LU)."""
    A = ls_dense_matrix(plan, q)
    sigma = np.linalg.solve(A, ls_rhs(plan, q, phi_in).ravel())
    return sigma.reshape((plan.N,) * plan.d)


def ls_relative_residual(plan, q, phi_in, sigma):
    b = ls_rhs(plan, q, phi_in)
    return float(np.linalg.norm(ls_operator(plan, q, sigma) - b) / np.linalg.norm(b))
