"""Pins of the oracle's own FFT (oracle/fft.c) against the DFT's definition.

Every length the method transforms is checked: the 2N box lengths of the GPU
path (powers of two, the mixed-radix 96 ... 500 and 3200 ... 12800) and the
P N lattice lengths of the precompute.  The reference is the O(n^2) sum of the
definition (oracle.fft.dft_naive), a different computation from the recursive
factorisation; the bar, 1e-13 of the largest output, is a few hundred times
the rounding of either for these lengths.  Closed-form transforms (an impulse,
a pure exponential) and Parseval's identity pin it without any other DFT.
"""
import numpy as np
import pytest

from oracle import fft as offt
from oracle import operator as op

# 2N of every specialised kernel length, the generic-kernel test lengths,
# and lattice lengths P N (P = 4, 5, 6)
LENGTHS = [2, 3, 4, 5, 6, 7, 8, 10, 12, 14, 20, 21, 24, 28, 30, 32, 40, 48, 60, 64, 70, 80, 96, 100, 112,
           120, 128, 160, 192, 200, 240, 256, 300, 384, 400, 500, 512, 640, 1000, 1024, 1536, 2048, 3200,
           4096, 6400, 8192, 12800]


def rel_max(a, b):
    return np.max(np.abs(a - b)) / max(np.max(np.abs(b)), 1e-300)


@pytest.mark.parametrize("n", LENGTHS)
def test_fft_matches_definition(n):
    rng = np.random.default_rng(n)
    x = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    X = op.fftn(x)
    assert rel_max(X, offt.dft_naive(x, sign=-1)) < 1e-13
    # inverse: the definition with the opposite sign, divided by n
    y = op.ifftn(X)
    assert rel_max(y, offt.dft_naive(X, sign=+1) / n) < 1e-13
    assert rel_max(y, x) < 1e-13


@pytest.mark.parametrize("shape", [(6, 10, 8), (12, 20), (4, 6, 10), (3, 96), (2, 5, 100), (7, 3, 2)])
def test_multi_axis_is_separable_definition(shape):
    rng = np.random.default_rng(len(shape) * 100 + shape[-1])
    x = rng.standard_normal(shape) + 1j * rng.standard_normal(shape)
    ref = x
    for ax in range(x.ndim):
        ref = offt.dft_naive(ref, axis=ax, sign=-1)
    assert rel_max(op.fftn(x), ref) < 1e-13
    back = x
    for ax in range(x.ndim):
        back = offt.dft_naive(back, axis=ax, sign=+1) / x.shape[ax]
    assert rel_max(op.ifftn(x), back) < 1e-13


def test_single_axis_transform():
    rng = np.random.default_rng(5)
    x = rng.standard_normal((4, 30, 6)) + 1j * rng.standard_normal((4, 30, 6))
    assert rel_max(offt.fftn(x, axes=[1]), offt.dft_naive(x, axis=1)) < 1e-13


@pytest.mark.parametrize("n", [96, 500, 512, 8192, 12800])
def test_closed_forms(n):
    # impulse at j0 -> W^{j0 k}; exponential e^{2 pi i m j / n} -> n delta_{k m}
    j0, m = n // 3 + 1, n // 5 + 2
    x = np.zeros(n, complex)
    x[j0] = 1.0
    k = np.arange(n)
    assert np.max(np.abs(op.fftn(x) - np.exp(-2j * np.pi * ((j0 * k) % n) / n))) < 1e-13
    e = np.exp(2j * np.pi * ((m * k) % n) / n)
    ref = np.zeros(n, complex)
    ref[m] = n
    assert np.max(np.abs(op.fftn(e) - ref)) < 1e-12 * n
    # Parseval: sum |X|^2 = n sum |x|^2
    rng = np.random.default_rng(n)
    x = rng.standard_normal(n) + 1j * rng.standard_normal(n)
    X = op.fftn(x)
    assert abs(np.vdot(X, X).real - n * np.vdot(x, x).real) < 1e-12 * n * np.vdot(x, x).real


def test_3d_box_against_definition():
    # a (2N)^3 box of the 3D path (N = 12) and a P N lattice (N = 6, P = 4)
    for shape in [(24, 24, 24), (30, 20, 28)]:
        rng = np.random.default_rng(shape[0])
        x = rng.standard_normal(shape) + 1j * rng.standard_normal(shape)
        ref = x
        for ax in range(3):
            ref = offt.dft_naive(ref, axis=ax)
        assert rel_max(op.fftn(x), ref) < 1e-13


def test_library_cross_check():
    # optional cross-check against scipy's FFT (not a pin: a third party)
    sfft = pytest.importorskip("scipy.fft")
    rng = np.random.default_rng(11)
    x = rng.standard_normal((20, 96, 30)) + 1j * rng.standard_normal((20, 96, 30))
    assert rel_max(op.fftn(x), sfft.fftn(x)) < 1e-14
