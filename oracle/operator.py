"""The discrete volume-integral operator of Section 4, in FP64.

Test infrastructure (see the package docstring).

Notation.  Grid: h = 1/N, N even, array index a in [0, N) at x_a = (a - N/2 + 1) h
(Section 4 places the samples at the integers -N/2+1..N/2 times h).  The
trapezoidal rule of Section 2 runs over a frequency lattice with P = 4 times the
density's resolution (Section 2: a factor 2 for the aperiodic convolution and a
factor 2 for the oscillation of the truncated kernel's transform): M = P N
points per axis, spacing ds = 2 pi / P, s_m = ds * m for signed m in
[-M/2, M/2), taken in FFT order.

The inverse transform (Introduction, eq. `ift`) of G^L F, discretised by the
trapezoidal rule in s and in x, gives phi_{i'} = sum_i T(i' - i) f_i with
    T(n) = M^{-d} sum_m G^L(|s_m|) exp(2 pi i m.n / M)          (1)
because (2 pi)^{-d} ds^d h^d = M^{-d}; T is the response to a unit density at
one grid point (Section 4).  Offsets between points of the N^d grid satisfy
|n_j| <= N - 1, so applying T needs only an aperiodic convolution, i.e. a
(2N)^d circular convolution after zero padding (Section 4):
    Khat(k) = sum_{|n_j| <= N-1} T(n) exp(-2 pi i k.n / (2N))     (2)
    phi     = crop_N( IDFT_2N( Khat * DFT_2N(pad_2N f) ) / (2N)^d ) (3)
The direct route of Section 2, pad to M^d, multiply by G^L(|s_m|), inverse,
crop, is (4); (3) and (4) agree to rounding.
"""
from __future__ import annotations

import math

import numpy as np

from . import fft as _fft
from . import greens

P_DEFAULT = 4


def fftn(a, workers=None):
    """Forward DFT over every axis: the oracle's own FFT (fft.c), pinned to the
    O(n^2) definition at every transform length the method uses."""
    return _fft.fftn(a, workers=workers)


def ifftn(a, workers=None):
    """Inverse DFT over every axis, divided by the number of points."""
    return _fft.ifftn(a, workers=workers)


def grid_coords(N):
    """x_a = (a - N/2 + 1)/N for a = 0..N-1 (Section 4's grid, N even)."""
    if N % 2:
        raise ValueError("N must be even")
    return (np.arange(N, dtype=np.float64) - (N // 2 - 1)) / N


def signed_index(M):
    """Signed integer frequencies of an M-point DFT in FFT order."""
    return np.fft.fftfreq(M, d=1.0 / M)


def lattice_radius(d, M, P=P_DEFAULT):
    """|s_m| on the full M^d lattice, s_m = (2 pi / P) m, FFT order."""
    m = signed_index(M) * (2.0 * math.pi / P)
    sq = np.zeros((M,) * d)
    for ax in range(d):
        shape = [1] * d
        shape[ax] = M
        sq = sq + (m ** 2).reshape(shape)
    return np.sqrt(sq)


def kernel_spectrum(d, N, kernel, k=0.0, L=None, P=P_DEFAULT, h=None):
    """G^L(|s_m|) on the full (P N)^d lattice (Section 2, Tables 1-2).  For the
    convection kernel (Tables 1-2, last row) G_h(s) = G^L_{|h|}(|s - h|), the
    Helmholtz transform at the shifted frequency, which is not radial."""
    M = P * N
    if kernel == "convection":
        h = np.asarray(h, dtype=np.float64)
        m = signed_index(M) * (2.0 * math.pi / P)
        sq = np.zeros((M,) * d)
        for ax in range(d):
            shape = [1] * d
            shape[ax] = M
            sq = sq + ((m - h[ax]) ** 2).reshape(shape)
        return greens.kernel_transform(d, "helmholtz", np.sqrt(sq), float(np.linalg.norm(h)), L)
    return greens.kernel_transform(d, kernel, lattice_radius(d, M, P), k, L)


def operator_T(Ghat, N):
    """Eq. (1): T = M^{-d} IDFT_M(Ghat), returned on the offsets |n_j| <= N-1 as
    an array of shape (2N-1)^d whose centre element is n = 0.  The inverse
    transform ifftn carries the M^{-d} factor."""
    d = Ghat.ndim
    t = ifftn(Ghat)
    idx = np.arange(-(N - 1), N)
    return t[np.ix_(*([idx % Ghat.shape[0]] * d))]


def wrap_2n(T_off, N):
    """Place T(n), |n_j| <= N-1, on the 2N-periodic box (index n mod 2N); the
    one unused offset per axis (n = -N == N mod 2N) is set to zero."""
    d = T_off.ndim
    box = np.zeros((2 * N,) * d, dtype=np.complex128)
    idx = np.arange(-(N - 1), N) % (2 * N)
    box[np.ix_(*([idx] * d))] = T_off
    return box


def kernel_hat_2n(T_off, N):
    """Eq. (2): Khat = DFT_2N of T on the 2N box."""
    return fftn(wrap_2n(T_off, N))


def pad(f, size):
    """Zero-pad an N^d array into size^d, data in the leading corner."""
    out = np.zeros((size,) * f.ndim, dtype=np.complex128)
    out[tuple(slice(0, n) for n in f.shape)] = f
    return out


def crop(a, N):
    return a[(slice(0, N),) * a.ndim]


def apply_2n(f, Khat):
    """Eq. (3): aperiodic convolution with T through the (2N)^d box."""
    N = f.shape[0]
    return crop(ifftn(Khat * fftn(pad(f, 2 * N))), N)


def apply_4n(f, Ghat):
    """Eq. (4), Section 2's direct route: pad to M^d, multiply the density's
    spectrum by G^L on the oversampled lattice, inverse, crop."""
    N = f.shape[0]
    M = Ghat.shape[0]
    return crop(ifftn(Ghat * fftn(pad(f, M))), N)


def spectral_multiplier(d, size, axis, scale):
    """i * scale * (signed frequency along `axis`) on a size^d box, with the
    Nyquist frequency (index size/2) given the value 0."""
    kt = signed_index(size)
    kt[size // 2] = 0.0
    shape = [1] * d
    shape[axis] = size
    return (1j * scale * kt).reshape(shape)


def gradient_2n(f, Khat):
    """Spectral gradient through the 2N box: d_j phi = crop IDFT(i kappa_j Khat
    DFT(pad f)) with kappa_j = pi * k_j (the 2N box has period 2N h = 2), zero at
    the Nyquist index.  The abstract and Section 3 obtain any derivative by
    spectral differentiation at the cost of one more FFT.  Returns (d, N^d)."""
    N = f.shape[0]
    d = f.ndim
    spec = Khat * fftn(pad(f, 2 * N))
    return np.stack([crop(ifftn(spectral_multiplier(d, 2 * N, j, math.pi) * spec), N)
                     for j in range(d)])


def gradient_4n(f, Ghat, P=P_DEFAULT):
    """The same derivative taken on the oversampled lattice: multiply by
    i s_j G^L(|s_m|), s_j = (2 pi / P) m_j (Nyquist zeroed).  An independent
    spectral route used to cross-check gradient_2n."""
    N = f.shape[0]
    d = f.ndim
    M = Ghat.shape[0]
    spec = Ghat * fftn(pad(f, M))
    return np.stack([crop(ifftn(spectral_multiplier(d, M, j, 2.0 * math.pi / P) * spec), N)
                     for j in range(d)])


def apply_direct(f, T_off):
    """phi_{i'} = sum_i T(i' - i) f_i by explicit summation (Section 4's discrete
    convolution written out); O(N^(2d)), for tiny grids only."""
    N = f.shape[0]
    d = f.ndim
    out = np.zeros_like(f, dtype=np.complex128)
    ar = np.arange(N)
    for ip in np.ndindex(*f.shape):
        sl = tuple((ip[ax] - ar) + (N - 1) for ax in range(d))
        out[ip] = np.sum(T_off[np.ix_(*sl)] * f)
    return out


# ---------------------------------------------------------------------------
# Large grids.  The full M^d lattice does not fit in host memory for large N
# (M = 1024 in 3D is 17 GB of complex128), so (1) and (2) are also written as
# sums over one octant.  G^L(|s_m|) depends on |m_j| only, hence the summand of
# (1) pairs m_j with -m_j and per axis
#     sum_{m=-M/2}^{M/2-1} a(m) e^{2 pi i m n/M}
#       = sum_{m=0}^{M/2} w_m a(m) cos(2 pi m n / M),  w_0 = w_{M/2} = 1, else 2,
# applied axis by axis (the partially summed array stays even in the remaining
# axes).  The same evenness of T gives (2) as
#     sum_{n=-(N-1)}^{N-1} T(n) e^{-2 pi i k n/(2N)} = sum_{n=0}^{N-1} v_n T(n) cos(pi k n / N),
# v_0 = 1, else 2, for k in [0, N]; Khat(k) = Khat(2N - k) per axis.

def _cos_matrix(n_out, m_in, period, weights):
    """C[n, m] = weights[m] cos(2 pi (n m mod period) / period)."""
    n = np.arange(n_out, dtype=np.int64)[:, None]
    m = np.arange(m_in, dtype=np.int64)[None, :]
    ph = (n * m) % period
    return np.cos(2.0 * math.pi * ph / period) * weights[None, :]


def _contract_axes(a, mats):
    """Apply mats[j] (shape (out_j, in_j)) along axis j of `a` for every axis."""
    for ax, C in enumerate(mats):
        a = np.moveaxis(np.tensordot(C, a, axes=([1], [ax])), 0, ax)
    return a


def kernel_spectrum_octant(d, N, kernel, k=0.0, L=None, P=P_DEFAULT):
    """G^L(|s_m|) for m in [0, M/2]^d."""
    M = P * N
    m = np.arange(M // 2 + 1, dtype=np.float64) * (2.0 * math.pi / P)
    sq = np.zeros((M // 2 + 1,) * d)
    for ax in range(d):
        shape = [1] * d
        shape[ax] = M // 2 + 1
        sq = sq + (m ** 2).reshape(shape)
    return greens.kernel_transform(d, kernel, np.sqrt(sq), k, L)


def operator_T_octant(G_oct, N, P=P_DEFAULT):
    """Eq. (1) on n in [0, N)^d from the octant of G^L (cosine form above)."""
    d = G_oct.ndim
    M = P * N
    w = np.full(M // 2 + 1, 2.0)
    w[0] = 1.0
    w[-1] = 1.0
    C = _cos_matrix(N, M // 2 + 1, M, w)
    return _contract_axes(G_oct.astype(np.complex128), [C] * d) / float(M) ** d


def kernel_hat_octant(T_oct):
    """Eq. (2) on k in [0, N]^d from the octant of T (cosine form above)."""
    d = T_oct.ndim
    N = T_oct.shape[0]
    v = np.full(N, 2.0)
    v[0] = 1.0
    D = _cos_matrix(N + 1, N, 2 * N, v)
    return _contract_axes(T_oct, [D] * d)


def T_offsets_from_octant(T_oct):
    """Expand T on [0, N)^d to the (2N-1)^d offsets using T(n) = T(|n|)."""
    N = T_oct.shape[0]
    idx = np.abs(np.arange(-(N - 1), N))
    return T_oct[np.ix_(*([idx] * T_oct.ndim))]


def khat_full_from_octant(K_oct):
    """Expand Khat on [0, N]^d to the (2N)^d box using Khat(k) = Khat(2N - k)."""
    N = K_oct.shape[0] - 1
    k = np.arange(2 * N)
    fold = np.minimum(k, 2 * N - k)
    return K_oct[np.ix_(*([fold] * K_oct.ndim))]


def apply_at_points(f, T_oct, points):
    """phi at selected grid points by direct summation sum_i T(i' - i) f_i, with
    T(n) = T_oct(|n_1|, .., |n_d|).  `points` is an (P, d) integer array."""
    N = f.shape[0]
    d = f.ndim
    ar = np.arange(N)
    out = np.empty(len(points), dtype=np.complex128)
    for p, ip in enumerate(points):
        sl = [np.abs(int(ip[ax]) - ar) for ax in range(d)]
        out[p] = np.sum(T_oct[np.ix_(*sl)] * f)
    return out


# ---------------------------------------------------------------------------
# A plan bundles what a convolution needs: the octants of T and of Khat.

class Plan:
    """FP64 oracle plan: T and Khat octants for (d, N, kernel, k, L, P).

    route='full' builds (1) and (2) with full-lattice FFTs (small N);
    route='octant' uses the cosine forms (any N that fits in memory)."""

    def __init__(self, d, N, kernel, k=0.0, L=None, P=P_DEFAULT, route=None, h=None):
        if N % 2 or N < 2:
            raise ValueError("N must be even and >= 2")
        self.d, self.N, self.kernel, self.k, self.P = d, N, kernel, float(k), P
        self.L = greens.L_DEFAULT[d] if L is None else L
        if kernel == "convection":
            # no per-axis symmetry: T on all offsets |n_j| <= N-1 and the full
            # (2N)^d Khat, from full-lattice FFTs
            self.h = np.asarray(h, dtype=np.float64)
            self.k = float(np.linalg.norm(self.h))
            self.route = "full"
            self.Ghat = kernel_spectrum(d, N, kernel, 0.0, self.L, P, self.h)
            self.T_off = operator_T(self.Ghat, N)
            self.Khat = kernel_hat_2n(self.T_off, N)
            self.T_oct = None
            self.K_oct = None
            return
        if route is None:
            route = "full" if (P * N) ** d <= 2 ** 24 else "octant"
        self.route = route
        if route == "full":
            self.Ghat = kernel_spectrum(d, N, kernel, k, self.L, P)
            T_off = operator_T(self.Ghat, N)
            self.T_oct = T_off[(slice(N - 1, None),) * d].copy()
            self.Khat = kernel_hat_2n(T_off, N)
            self.K_oct = self.Khat[(slice(0, N + 1),) * d].copy()
        else:
            self.Ghat = None
            G_oct = kernel_spectrum_octant(d, N, kernel, k, self.L, P)
            self.T_oct = operator_T_octant(G_oct, N, P)
            del G_oct
            self.K_oct = kernel_hat_octant(self.T_oct)
            self.Khat = None

    def khat_full(self):
        if self.Khat is None:
            self.Khat = khat_full_from_octant(self.K_oct)
        return self.Khat

    def apply(self, f):
        return apply_2n(np.asarray(f, dtype=np.complex128), self.khat_full())

    def gradient(self, f):
        return gradient_2n(np.asarray(f, dtype=np.complex128), self.khat_full())

    def apply_at_points(self, f, points):
        return apply_at_points(np.asarray(f, dtype=np.complex128), self.T_oct, points)
