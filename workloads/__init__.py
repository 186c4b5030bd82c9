"""Seeded synthetic densities shared by the tests, the benchmark and the oracle.

This module only draws random parameters and evaluates the source density on the
grid.  It contains none of the convolution method's arithmetic: no kernel
spectrum, no FFT, no operator.  Both the FP64 oracle and the GPU library receive
the arrays produced here (the GPU gets them rounded to complex64 for FP32 plans).

Sources are sums of normalised isotropic Gaussians, the paper's analytic test
source (Section 5.1, the Gaussian densities in 3D and 2D), optionally multiplied
by a plane-wave phase exp(i a.x):

    f(x) = exp(i a.x) * sum_j amp_j * rho_{sigma_j}(x - c_j),
    rho_sigma(r) = (2 pi sigma^2)^(-d/2) exp(-r^2 / (2 sigma^2)).

The grid is the paper's (Section 4): h = 1/N and, along every axis, array index
a in [0, N) sits at x_a = (a - N/2 + 1) h, i.e. the integer points
{-N/2+1, ..., N/2} scaled by h.  N must be even.

Random draws use numpy.random.default_rng(seed) (PCG64) in a fixed order:
centres, widths, amplitudes, then the modulation vector.
"""
from __future__ import annotations

from dataclasses import dataclass, field
import math

import numpy as np

__all__ = [
    "GaussianSum",
    "grid_coords",
    "draw_gaussian_sum",
    "evaluate_grid",
    "WORKLOADS",
    "workload",
    "batch_workload",
]


def grid_coords(N: int) -> np.ndarray:
    """Coordinates x_a = (a - N/2 + 1)/N, a = 0..N-1, of one grid axis (N even)."""
    if N % 2:
        raise ValueError("N must be even")
    return (np.arange(N, dtype=np.float64) - (N // 2 - 1)) / N


@dataclass
class GaussianSum:
    d: int
    centers: np.ndarray          # (J, d)
    sigmas: np.ndarray           # (J,)
    amps: np.ndarray             # (J,) real amplitudes
    avec: np.ndarray = field(default=None)  # (d,) plane-wave modulation or None

    @property
    def count(self) -> int:
        return int(self.sigmas.shape[0])


def draw_gaussian_sum(seed: int, d: int, count: int, center_box: float,
                      sigma_range: tuple, mod_max: float = 0.0) -> GaussianSum:
    """Draw `count` Gaussians: centres U[-center_box, center_box]^d, widths
    U[sigma_range], amplitudes N(0,1); if mod_max > 0, a plane-wave vector with a
    uniformly random direction and |a| ~ U[0, mod_max]."""
    rng = np.random.default_rng(seed)
    centers = rng.uniform(-center_box, center_box, size=(count, d))
    sigmas = rng.uniform(sigma_range[0], sigma_range[1], size=count)
    amps = rng.standard_normal(count)
    avec = None
    if mod_max > 0.0:
        direction = rng.standard_normal(d)
        direction /= np.linalg.norm(direction)
        avec = direction * rng.uniform(0.0, mod_max)
    return GaussianSum(d, centers, sigmas, amps, avec)


def evaluate_grid(src: GaussianSum, N: int, window_sigmas: float = 12.0) -> np.ndarray:
    """Evaluate the density on the N^d grid as a C-ordered complex128 array.

    Each Gaussian is separable, so it is formed as an outer product of per-axis
    factors.  Per axis the factor is evaluated only within window_sigmas widths
    of the centre (outside it is below exp(-72) of its peak, under FP64
    resolution of the sum); this bound is part of the input's definition.
    """
    d = src.d
    x = grid_coords(N)
    out = np.zeros((N,) * d, dtype=np.complex128)
    for j in range(src.count):
        sig = float(src.sigmas[j])
        norm = (2.0 * math.pi * sig * sig) ** (-d / 2.0) * float(src.amps[j])
        lo_hi = []
        facs = []
        for ax in range(d):
            c = float(src.centers[j, ax])
            lo = max(0, int(math.floor((c - window_sigmas * sig) * N + (N // 2 - 1))))
            hi = min(N, int(math.ceil((c + window_sigmas * sig) * N + (N // 2 - 1))) + 1)
            if hi <= lo:
                break
            xs = x[lo:hi]
            facs.append(np.exp(-((xs - c) ** 2) / (2.0 * sig * sig)))
            lo_hi.append((lo, hi))
        else:
            block = facs[0] * norm
            for ax in range(1, d):
                block = np.multiply.outer(block, facs[ax])
            sl = tuple(slice(lo, hi) for lo, hi in lo_hi)
            out[sl] += block
    if src.avec is not None:
        phase = None
        for ax in range(d):
            p = np.exp(1j * src.avec[ax] * x)
            shape = [1] * d
            shape[ax] = N
            p = p.reshape(shape)
            phase = p if phase is None else phase * p
        out *= phase
    return out


# Named workloads.  Shapes and value distributions follow the configurations the
# library is measured on; seeds are fixed so every consumer sees the same array.
WORKLOADS = {
    # 3D Laplace, N=32, FP64 plan: 3 Gaussians.
    "laplace3d_n32": dict(d=3, N=32, kernel="laplace", k=0.0, seed=1001, count=3,
                          center_box=0.2, sigma_range=(0.04, 0.08), mod_max=0.0),
    # 3D Helmholtz k=20, N=128 (256^3 padded): 8 modulated Gaussians.
    "helmholtz3d_k20_n128": dict(d=3, N=128, kernel="helmholtz", k=20.0, seed=1002, count=8,
                                 center_box=0.2, sigma_range=(0.03, 0.06), mod_max=10.0),
    # 3D Helmholtz k=20, N=256 (512^3 padded): same recipe at twice the resolution.
    "helmholtz3d_k20_n256": dict(d=3, N=256, kernel="helmholtz", k=20.0, seed=1010, count=8,
                                 center_box=0.2, sigma_range=(0.03, 0.06), mod_max=10.0),
    # 2D, N=4096 (8192^2 padded): 32 Gaussians, Laplace and Helmholtz k=200.
    "laplace2d_n4096": dict(d=2, N=4096, kernel="laplace", k=0.0, seed=1003, count=32,
                            center_box=0.3, sigma_range=(0.005, 0.02), mod_max=0.0),
    "helmholtz2d_k200_n4096": dict(d=2, N=4096, kernel="helmholtz", k=200.0, seed=1003, count=32,
                                   center_box=0.3, sigma_range=(0.005, 0.02), mod_max=0.0),
    # 3D Helmholtz k=150, N=512 (1024^3 padded), potential plus gradient: 256 Gaussians.
    "helmholtz3d_k150_n512": dict(d=3, N=512, kernel="helmholtz", k=150.0, seed=1005, count=256,
                                  center_box=0.3, sigma_range=(0.01, 0.03), mod_max=0.0),
}


def workload(name: str):
    """Return (params, GaussianSum) for a named workload."""
    p = dict(WORKLOADS[name])
    src = draw_gaussian_sum(p["seed"], p["d"], p["count"], p["center_box"],
                            p["sigma_range"], p["mod_max"])
    return p, src


def batch_workload(seed: int = 1004, count: int = 64, sizes=(48, 64, 96, 128)):
    """The mixed batch: `count` 3D densities, N drawn equally from `sizes` and
    shuffled, half Laplace and half Helmholtz with k ~ U[5, 40]; each density is
    a sum of 4 Gaussians (centres U[-0.2,0.2]^3, widths U[0.04,0.08], N(0,1)
    amplitudes).  Returns a list of (params, GaussianSum)."""
    rng = np.random.default_rng(seed)
    Ns = np.repeat(np.asarray(sizes), count // len(sizes))
    rng.shuffle(Ns)
    kinds = np.array(["laplace"] * (count // 2) + ["helmholtz"] * (count - count // 2))
    rng.shuffle(kinds)
    ks = rng.uniform(5.0, 40.0, size=count)
    out = []
    for i in range(count):
        kind = str(kinds[i])
        p = dict(d=3, N=int(Ns[i]), kernel=kind, k=float(ks[i]) if kind == "helmholtz" else 0.0,
                 seed=int(seed * 1000 + i))
        src = draw_gaussian_sum(p["seed"], 3, 4, 0.2, (0.04, 0.08), 0.0)
        out.append((p, src))
    return out
