"""GPU: structural properties of the discrete operator of Section 4 on the
device path, each against what the definition phi_{i'} = sum_i T(i' - i) f_i
fixes exactly:

  * the potential of a unit density at one grid point is the operator's
    entries T(i' - i) (the delta response of Section 4): compared element by
    element with the oracle's T and with the plan's own Nystrom entries;
  * an integer shift of a density whose support stays inside the grid shifts
    the potential by the same offset (translation invariance of a discrete
    convolution);
  * sum_i g_i (T f)_i = sum_i f_i (T g)_i (T is even in every axis, so the
    operator is complex symmetric).

Bars: FP64 plans 1e-12, FP32 plans 1e-5 (relative L2 and relative max, as in
the parity tests).
"""
import numpy as np
import pytest

from parity import check  # noqa: E402

pytestmark = pytest.mark.gpu

TOL = {"fp64": 1e-12, "fp32": 1e-5}


def _dev(a, precision):
    import torch
    dt = torch.complex128 if precision == "fp64" else torch.complex64
    return torch.from_numpy(np.ascontiguousarray(a)).to(dtype=dt, device="cuda")


def _T_at(T_oct, a, N):
    """T(i' - a) on the whole grid from the octant T(|n_1|, ..., |n_d|)."""
    d = len(a)
    idx = [np.abs(np.arange(N) - a[ax]) for ax in range(d)]
    return T_oct[np.ix_(*idx)]


CASES = [(3, 16, "helmholtz", 12.0), (3, 24, "laplace", 0.0), (2, 64, "helmholtz", 40.0), (2, 96, "laplace", 0.0),
         (3, 64, "helmholtz", 20.0)]


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("d,N,kernel,k", CASES)
def test_impulse_response_is_the_operator(d, N, kernel, k, precision):
    import torch

    import paper_1604_03155_amd as vg
    from oracle import operator as op
    a = (3, N - 2, N // 2)[:d]
    f = np.zeros((N,) * d, dtype=np.complex128)
    f[a] = 1.0
    p = vg.Plan(d, N, kernel, k, precision=precision, keep_operator=True)
    phi = p.apply(_dev(f, precision))
    torch.cuda.synchronize()
    got = phi.cpu().numpy().astype(np.complex128)
    ref = _T_at(op.Plan(d, N, kernel, k).T_oct, a, N)
    check(got, ref, TOL[precision], f"impulse at {a} vs oracle T")
    # the plan's own Nystrom entries (FP64 on the device for both precisions)
    check(got, _T_at(p.operator_entries(), a, N), TOL[precision], "impulse vs vg_plan_operator_entries")


@pytest.mark.parametrize("precision", ["fp64", "fp32"])
@pytest.mark.parametrize("d,N,kernel,k", [(3, 32, "helmholtz", 15.0), (2, 128, "laplace", 0.0)])
def test_translation_invariance(d, N, kernel, k, precision):
    import torch

    import paper_1604_03155_amd as vg
    rng = np.random.default_rng(31 + N)
    m = N // 2
    f = np.zeros((N,) * d, dtype=np.complex128)
    f[(slice(0, m),) * d] = rng.standard_normal((m,) * d) + 1j * rng.standard_normal((m,) * d)
    s = (5, 3, 7)[:d]
    g = np.roll(f, s, axis=tuple(range(d)))  # support [s, s + m) stays inside the grid
    p = vg.Plan(d, N, kernel, k, precision=precision)
    pf = p.apply(_dev(f, precision)).cpu().numpy().astype(np.complex128)
    pg = p.apply(_dev(g, precision)).cpu().numpy().astype(np.complex128)
    torch.cuda.synchronize()
    shifted = tuple(slice(sj, N) for sj in s)
    unshifted = tuple(slice(0, N - sj) for sj in s)
    check(pg[shifted], pf[unshifted], TOL[precision], f"shift by {s}")


@pytest.mark.parametrize("d,N,kernel,k", [(3, 20, "helmholtz", 9.0), (2, 80, "helmholtz", 30.0)])
def test_operator_is_complex_symmetric(d, N, kernel, k):
    import torch

    import paper_1604_03155_amd as vg
    rng = np.random.default_rng(7 * N)
    f = rng.standard_normal((N,) * d) + 1j * rng.standard_normal((N,) * d)
    g = rng.standard_normal((N,) * d) + 1j * rng.standard_normal((N,) * d)
    p = vg.Plan(d, N, kernel, k, precision="fp64")
    Af = p.apply(_dev(f, "fp64")).cpu().numpy()
    Ag = p.apply(_dev(g, "fp64")).cpu().numpy()
    torch.cuda.synchronize()
    lhs, rhs = np.sum(g * Af), np.sum(f * Ag)
    assert abs(lhs - rhs) <= 1e-12 * max(abs(lhs), np.linalg.norm(g) * np.linalg.norm(Af))
