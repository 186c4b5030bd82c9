"""Inputs of the Lippmann-Schwinger scattering examples (Section 5.3).

Analytic contrast functions q(x) and incident fields on the grid x_a =
(a - N/2 + 1)/N of every axis.  These are input definitions only: no part of
the convolution or of the solve.  Axis 0 of an array is the x coordinate, the
direction of the incident plane wave ("propagating to the right").
"""
from __future__ import annotations

import numpy as np

from . import grid_coords

__all__ = ["contrast", "plane_wave", "CONTRASTS"]


def _mesh(d, N):
    x = grid_coords(N)
    return np.meshgrid(*([x] * d), indexing="ij")


def contrast(name: str, N: int) -> np.ndarray:
    """q on the N^d grid (complex128):
      'smoothed_cube' (3D): exp(-((x/0.25)^8 + (y/0.25)^8 + (z/0.25)^8)/2);
      'smoothed_disk' (2D): exp(-(|x|/0.25)^8/2);
      'luneburg' (2D): 1 - (|x|/0.45)^2 inside |x| < 0.45, 0 outside (the lens
        occupies the disk of radius 0.45; outside it the printed expression
        would be negative)."""
    if name == "smoothed_cube":
        X = _mesh(3, N)
        q = np.exp(-0.5 * sum((xx / 0.25) ** 8 for xx in X))
    elif name == "smoothed_disk":
        X = _mesh(2, N)
        r = np.sqrt(X[0] ** 2 + X[1] ** 2)
        q = np.exp(-0.5 * (r / 0.25) ** 8)
    elif name == "luneburg":
        X = _mesh(2, N)
        r = np.sqrt(X[0] ** 2 + X[1] ** 2)
        q = np.where(r < 0.45, 1.0 - (r / 0.45) ** 2, 0.0)
    else:
        raise ValueError(f"unknown contrast {name!r}")
    return q.astype(np.complex128)


CONTRASTS = {"smoothed_cube": 3, "smoothed_disk": 2, "luneburg": 2}


def plane_wave(d: int, N: int, k: float) -> np.ndarray:
    """Incident field exp(i k x) along axis 0 on the N^d grid (complex128)."""
    X = _mesh(d, N)
    return np.exp(1j * k * X[0]).astype(np.complex128)
