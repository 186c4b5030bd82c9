"""Pins for the oracle's discrete operator (Section 4) and its applications.

Every check compares the oracle with something other than itself: a naive
brute-force sum, the paper's 4N route, the closed-form potentials of Gaussian
sources (Section 5.1), exact algebraic properties (symmetry, linearity,
translation invariance, positivity), or the PDE itself.
"""
import math

import numpy as np
import pytest

from oracle import closed_form as cf
from oracle import greens
from oracle import operator as op
from workloads import grid_coords


def _centered_gaussian(d, N, sigma):
    x = grid_coords(N)
    X = np.meshgrid(*([x] * d), indexing="ij")
    r = np.sqrt(sum(xx ** 2 for xx in X))
    return r, np.exp(-r ** 2 / (2 * sigma ** 2)) / (2 * math.pi * sigma ** 2) ** (d / 2)


def _random_density(rng, d, N, margin=0, real=False):
    f = rng.standard_normal((N,) * d)
    if not real:
        f = f + 1j * rng.standard_normal((N,) * d)
    if margin:
        mask = np.zeros((N,) * d, dtype=bool)
        mask[(slice(margin, N - margin),) * d] = True
        f = np.where(mask, f, 0)
    return f.astype(np.complex128)


@pytest.mark.parametrize("d,N,kernel,k", [(3, 4, "helmholtz", 3.0), (3, 4, "laplace", 0.0),
                                          (2, 8, "helmholtz", 5.0), (2, 6, "laplace", 0.0),
                                          (3, 4, "biharmonic", 0.0), (2, 8, "biharmonic", 0.0),
                                          (3, 4, "laplace_helmholtz", 4.0), (2, 6, "laplace_helmholtz", 9.0)])
def test_T_equals_naive_lattice_sum(d, N, kernel, k):
    """Eq. (1) of the operator module by brute force: M^-d sum_m G e^{2 pi i m.n/M}."""
    plan = op.Plan(d, N, kernel, k, route="full")
    M = 4 * N
    m = op.signed_index(M)
    grids = np.meshgrid(*([m] * d), indexing="ij")
    s = np.sqrt(sum((g * (2 * math.pi / 4)) ** 2 for g in grids))
    G = greens.kernel_transform(d, kernel, s, k)
    for n in [(0,) * d, (1,) + (0,) * (d - 1), tuple(range(1, d + 1)), (N - 1,) * d]:
        ph = sum(g * nn for g, nn in zip(grids, n))
        ref = np.sum(G * np.exp(2j * math.pi * ph / M)) / M ** d
        got = plan.T_oct[tuple(abs(v) for v in n)]
        assert abs(got - ref) < 1e-14 * np.abs(plan.T_oct).max()


@pytest.mark.parametrize("d,N,kernel,k", [(3, 12, "helmholtz", 7.0), (2, 20, "laplace", 0.0),
                                          (2, 16, "helmholtz", 30.0), (3, 10, "laplace", 0.0),
                                          (3, 10, "biharmonic", 0.0), (2, 16, "biharmonic", 0.0),
                                          (2, 16, "laplace_helmholtz", 12.0)])
def test_octant_route_equals_full_lattice_route(d, N, kernel, k):
    full = op.Plan(d, N, kernel, k, route="full")
    octa = op.Plan(d, N, kernel, k, route="octant")
    assert np.max(np.abs(full.T_oct - octa.T_oct)) < 1e-14 * np.max(np.abs(full.T_oct))
    assert np.max(np.abs(full.K_oct - octa.K_oct)) < 1e-13 * np.max(np.abs(full.K_oct))
    assert np.max(np.abs(full.Khat - octa.khat_full())) < 1e-13 * np.max(np.abs(full.Khat))


def test_T_symmetries_and_laplace_reality():
    for d, N, kernel, k in [(3, 8, "helmholtz", 4.0), (3, 8, "laplace", 0.0), (2, 16, "helmholtz", 9.0)]:
        plan = op.Plan(d, N, kernel, k)
        T = op.operator_T(plan.Ghat, N)
        # even in every axis
        for ax in range(d):
            assert np.allclose(T, np.flip(T, axis=ax), rtol=0, atol=1e-15 * np.abs(T).max())
        # symmetric under axis permutations
        assert np.allclose(T, np.swapaxes(T, 0, 1), rtol=0, atol=1e-15 * np.abs(T).max())
        if kernel == "laplace":
            assert np.abs(T.imag).max() < 1e-15 * np.abs(T).max()
            assert np.abs(plan.Khat.imag).max() < 1e-13 * np.abs(plan.Khat).max()


def test_laplace3d_operator_is_positive_semidefinite():
    """G^L_0 >= 0 in 3D, so T is a principal block of a PSD circulant."""
    rng = np.random.default_rng(3)
    N = 12
    plan = op.Plan(3, N, "laplace")
    for _ in range(5):
        f = rng.standard_normal((N, N, N))
        q = np.vdot(f, plan.apply(f)).real
        assert q > 0


def test_T_is_a_mollified_green_function():
    """Figure 2: T(n)/h^3 follows 1/(4 pi |n| h) away from n = 0."""
    N = 32
    h = 1.0 / N
    T = op.Plan(3, N, "laplace").T_oct.real
    for n in (1, 2, 3, 5, 8, 12, 20, 31):
        ratio = T[n, 0, 0] / h ** 3 * 4 * math.pi * n * h
        assert abs(ratio - 1) < (0.06 if n < 8 else 0.015)
        if n >= 5:
            rr = math.hypot(n, n // 2)
            ratio = T[n, n // 2, 0] / h ** 3 * 4 * math.pi * rr * h
            assert abs(ratio - 1) < 0.002
    # the diagonal entry is finite, unlike the naive trapezoidal rule
    assert 0 < T[0, 0, 0] / h ** 3 < 10


@pytest.mark.parametrize("d,N,kernel,k", [(3, 16, "helmholtz", 6.0), (3, 16, "laplace", 0.0),
                                          (2, 48, "helmholtz", 40.0), (2, 40, "laplace", 0.0)])
def test_2n_route_equals_4n_route(d, N, kernel, k):
    """Section 4: after the precomputation a (2N)^d FFT reproduces the (4N)^d route."""
    rng = np.random.default_rng(1)
    plan = op.Plan(d, N, kernel, k, route="full")
    f = _random_density(rng, d, N)
    a = plan.apply(f)
    b = op.apply_4n(f, plan.Ghat)
    assert np.linalg.norm(a - b) / np.linalg.norm(b) < 1e-13


@pytest.mark.parametrize("d,N,kernel,k", [(3, 6, "helmholtz", 5.0), (2, 10, "laplace", 0.0),
                                          (2, 8, "helmholtz", 12.0), (3, 6, "biharmonic", 0.0),
                                          (2, 10, "laplace_helmholtz", 7.0)])
def test_apply_equals_direct_summation(d, N, kernel, k):
    rng = np.random.default_rng(2)
    plan = op.Plan(d, N, kernel, k)
    f = _random_density(rng, d, N)
    T_off = op.T_offsets_from_octant(plan.T_oct)
    direct = op.apply_direct(f, T_off)
    assert np.linalg.norm(plan.apply(f) - direct) / np.linalg.norm(direct) < 1e-14
    pts = np.array([[0] * d, [N - 1] * d, list(range(d))])
    assert np.allclose(plan.apply_at_points(f, pts), direct[tuple(pts.T)], rtol=1e-13, atol=0)


def test_linearity_translation_and_transpose_symmetry():
    rng = np.random.default_rng(4)
    N, s = 16, 3
    plan = op.Plan(3, N, "helmholtz", 8.0)
    f = _random_density(rng, 3, N, margin=s)
    g = _random_density(rng, 3, N)
    a, b = 0.3 - 1.1j, 2.5
    lin = plan.apply(a * f + b * g) - (a * plan.apply(f) + b * plan.apply(g))
    assert np.linalg.norm(lin) < 1e-13 * np.linalg.norm(plan.apply(g))
    # integer shift along axis 1 while the support stays in the grid
    fs = np.zeros_like(f)
    fs[s:] = f[:-s]
    assert np.allclose(plan.apply(fs)[s:], plan.apply(f)[:-s], rtol=0, atol=1e-13 * np.abs(plan.apply(f)).max())
    # T(n) = T(-n): sum g (A f) = sum f (A g) without conjugation
    assert abs(np.sum(g * plan.apply(f)) - np.sum(f * plan.apply(g))) < 1e-12 * abs(np.sum(g * plan.apply(f)))


CONVERGENCE = [
    # (d, kernel, k, N, bound): one Gaussian, sigma = 0.05, centred (Figure 3 set-up, k = 2)
    (3, "laplace", 0.0, 16, 1e-3), (3, "laplace", 0.0, 24, 3e-6), (3, "laplace", 0.0, 32, 5e-9),
    (3, "laplace", 0.0, 48, 1e-14),
    (3, "helmholtz", 2.0, 24, 3e-6), (3, "helmholtz", 2.0, 48, 1e-14),
    (2, "laplace", 0.0, 32, 2e-8), (2, "laplace", 0.0, 64, 1e-14),
    (2, "helmholtz", 2.0, 32, 3e-8), (2, "helmholtz", 2.0, 64, 1e-14),
    # the other kernels of Tables 1-2 (Delta^2 and Delta(Delta + k^2))
    (3, "biharmonic", 0.0, 24, 2e-5), (3, "biharmonic", 0.0, 48, 1e-14),
    (2, "biharmonic", 0.0, 32, 1e-7), (2, "biharmonic", 0.0, 64, 1e-14),
    (3, "laplace_helmholtz", 2.0, 48, 1e-14), (2, "laplace_helmholtz", 20.0, 64, 1e-14),
]


@pytest.mark.parametrize("d,kernel,k,N,bound", CONVERGENCE)
def test_gaussian_source_converges_spectrally_to_closed_form(d, kernel, k, N, bound):
    sigma = 0.05
    r, f = _centered_gaussian(d, N, sigma)
    phi = op.Plan(d, N, kernel, k).apply(f)
    if d == 2 and kernel in ("helmholtz", "laplace_helmholtz"):
        rng = np.random.default_rng(5)
        idx = rng.integers(0, N, size=(12, d))
        rr = r[tuple(idx.T)]
        ref = cf.potential(d, kernel, k, rr, sigma)
        err = np.max(np.abs(phi[tuple(idx.T)] - ref)) / np.max(np.abs(ref))
    else:
        ref = cf.potential(d, kernel, k, r.ravel(), sigma).reshape(r.shape)
        err = np.linalg.norm(phi - ref) / np.linalg.norm(ref)
    assert err < bound


def test_offcentre_gaussian_sum_matches_closed_form():
    """A seeded sum of off-centre Gaussians (3D Helmholtz k = 20).  Widths and
    centres are chosen so the sources are resolved (pi sigma N >= 8) and contained
    (>= 8 sigma from the boundary), so the method's error is below 1e-10."""
    from workloads import draw_gaussian_sum, evaluate_grid
    N = 64
    src = draw_gaussian_sum(77, 3, 3, 0.08, (0.04, 0.05))
    f = evaluate_grid(src, N)
    phi = op.Plan(3, N, "helmholtz", 20.0).apply(f)
    x = grid_coords(N)
    rng = np.random.default_rng(6)
    idx = rng.integers(0, N, size=(200, 3))
    pts = x[idx]
    ref = cf.gaussian_sum_potential(3, "helmholtz", 20.0, src.centers, src.sigmas, src.amps, pts)
    got = phi[tuple(idx.T)]
    assert np.max(np.abs(got - ref)) / np.max(np.abs(ref)) < 1e-10


@pytest.mark.parametrize("d,kernel,k,N", [(3, "laplace", 0.0, 48), (3, "helmholtz", 2.0, 48),
                                          (2, "laplace", 0.0, 64), (2, "helmholtz", 20.0, 64),
                                          (3, "biharmonic", 0.0, 48), (2, "biharmonic", 0.0, 64),
                                          (3, "laplace_helmholtz", 2.0, 48)])
def test_gradient_routes_agree_and_match_closed_form(d, kernel, k, N):
    sigma = 0.05
    r, f = _centered_gaussian(d, N, sigma)
    plan = op.Plan(d, N, kernel, k)
    gB = plan.gradient(f)
    gA = op.gradient_4n(f, plan.Ghat)
    # biharmonic entries grow like |n| h, and G_k - G_0 cancels to k^2/s^4 out
    # of two 1/s^2 terms at large s, so these two carry more rounding
    loose = kernel in ("biharmonic", "laplace_helmholtz")
    assert np.linalg.norm(gA - gB) / np.linalg.norm(gA) < (2e-12 if loose else 2e-13)
    x = grid_coords(N)
    X = np.meshgrid(*([x] * d), indexing="ij")
    pts = np.stack([xx.ravel() for xx in X], 1)
    sel = np.random.default_rng(7).choice(len(pts), 40, replace=False)
    ref = cf.gaussian_sum_gradient(d, kernel, k, np.zeros((1, d)), [sigma], [1.0], pts[sel])
    got = gB.reshape(d, -1)[:, sel]
    assert np.max(np.abs(got - ref)) / np.max(np.abs(ref)) < 1e-12


@pytest.mark.parametrize("d,kernel,k,N", [(3, "laplace", 0.0, 48), (3, "helmholtz", 2.0, 48),
                                          (2, "helmholtz", 20.0, 64), (3, "biharmonic", 0.0, 48),
                                          (2, "biharmonic", 0.0, 64), (3, "laplace_helmholtz", 3.0, 48)])
def test_pde_residual_on_the_box(d, kernel, k, N):
    """phi = g * f solves (Delta + k^2) phi = -f (the sign follows from
    phi = g * f with the outgoing kernel), Delta^2 phi = -f for the biharmonic
    kernel and Delta (Delta + k^2) phi = k^2 f for the tables' g_k - g_0;
    evaluated spectrally on the uncropped 2N-periodic potential and restricted
    to the box."""
    sigma = 0.05
    _, f = _centered_gaussian(d, N, sigma)
    plan = op.Plan(d, N, kernel, k)
    spec = plan.Khat * op.fftn(op.pad(f, 2 * N))
    kap = math.pi * op.signed_index(2 * N)
    K2 = sum((kap ** 2).reshape([-1 if a == b else 1 for b in range(d)]) for a in range(d))
    if kernel == "biharmonic":
        res = op.crop(op.ifftn(K2 * K2 * spec), N) + f
    elif kernel == "laplace_helmholtz":
        res = op.crop(op.ifftn(-K2 * (k * k - K2) * spec), N) - k * k * f
    else:
        res = op.crop(op.ifftn((k * k - K2) * spec), N) + f
    # the fourth-order operators amplify rounding at the top frequencies by
    # |kappa|^4 ~ 5e9 (N = 48); a wrong sign or factor leaves an O(1) residual
    bound = 1e-8 if kernel in ("biharmonic", "laplace_helmholtz") else 1e-12
    assert np.linalg.norm(res) / np.linalg.norm(f) < bound


# ----------------------------------------------- convection kernel (h.grad) --

@pytest.mark.parametrize("d,N,h", [(2, 48, (3.3, -1.7)), (2, 48, (12.0, 5.0)), (3, 48, (2.5, -1.0, 4.0))])
def test_convection_kernel_pde_residual(d, N, h):
    """Tables 1-2, last row: G_h(s) = G_{|h|}(|s - h|) is the transform of
    g_h(x) = e^{i h.x} g_{|h|}(|x|), which satisfies (Delta - 2i h.grad) g_h =
    -delta; phi = g_h * f is checked spectrally on the box."""
    sigma = 0.05
    _, f = _centered_gaussian(d, N, sigma)
    plan = op.Plan(d, N, "convection", h=h)
    spec = plan.Khat * op.fftn(op.pad(f, 2 * N))
    kap = math.pi * op.signed_index(2 * N)
    ks = [kap.reshape([-1 if a == b else 1 for b in range(d)]) for a in range(d)]
    Lop = -sum(kk ** 2 for kk in ks) + 2.0 * sum(hh * kk for hh, kk in zip(h, ks))
    res = op.crop(op.ifftn(Lop * spec), N) + f
    assert np.linalg.norm(res) / np.linalg.norm(f) < 1e-11


@pytest.mark.parametrize("d,N,h", [(2, 8, (2.0, -3.5)), (3, 4, (1.5, 0.5, -2.0))])
def test_convection_T_naive_sum_routes_and_direct_summation(d, N, h):
    rng = np.random.default_rng(11)
    plan = op.Plan(d, N, "convection", h=h)
    M = 4 * N
    m = op.signed_index(M) * (2 * math.pi / 4)
    grids = np.meshgrid(*([m] * d), indexing="ij")
    G = greens.kernel_transform(d, "helmholtz", np.sqrt(sum((g - hh) ** 2 for g, hh in zip(grids, h))),
                                float(np.linalg.norm(h)))
    mi = np.meshgrid(*([op.signed_index(M)] * d), indexing="ij")
    for n in [(0,) * d, (1,) + (0,) * (d - 1), tuple(range(-1, d - 1)), (N - 1,) * d, (-(N - 1),) * d]:
        ref = np.sum(G * np.exp(2j * math.pi * sum(g * nn for g, nn in zip(mi, n)) / M)) / M ** d
        got = plan.T_off[tuple(v + N - 1 for v in n)]
        assert abs(got - ref) < 1e-14 * np.abs(plan.T_off).max()
    f = _random_density(rng, d, N)
    a = plan.apply(f)
    assert np.linalg.norm(a - op.apply_4n(f, plan.Ghat)) / np.linalg.norm(a) < 1e-13
    assert np.linalg.norm(a - op.apply_direct(f, plan.T_off)) / np.linalg.norm(a) < 1e-13
    # not even: T(n) != T(-n) in general
    assert abs(plan.T_off[(N,) * d] - plan.T_off[(N - 2,) * d]) > 1e-6 * np.abs(plan.T_off).max()
