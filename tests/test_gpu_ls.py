"""GPU: Lippmann-Schwinger solves (Section 5.3) by Bi-CGStab on the device
against the oracle's dense direct solve (small grids), the oracle's FP64
operator (residual of the GPU solution) and self-convergence (larger grids)."""
import sys
import time

import numpy as np
import pytest

from parity import check, rel_l2  # noqa: E402

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()




def _dev(a, precision):
    import torch
    return torch.from_numpy(a).to(torch.complex128 if precision == "fp64" else torch.complex64).cuda().contiguous()


@pytest.mark.parametrize("d,N,name,k,precision,tol,bound", [
    (2, 24, "smoothed_disk", 10.0, "fp64", 1e-13, 1e-10),
    (2, 32, "smoothed_disk", 15.0, "fp64", 1e-13, 1e-10),
    (2, 20, "luneburg", 10.0, "fp64", 1e-13, 1e-10),
    (3, 8, "smoothed_cube", 10.0, "fp64", 1e-13, 1e-10),
    (2, 32, "smoothed_disk", 15.0, "fp32", 1e-6, 1e-4),
])
def test_ls_solve_matches_direct_solve(d, N, name, k, precision, tol, bound):
    import torch

    import paper_1604_03155_amd as vg
    from oracle import operator as op
    from oracle import scattering as sc
    from workloads.scattering import contrast, plane_wave
    say("ls", d, N, name, k, precision)
    q, pin = contrast(name, N), plane_wave(d, N, k)
    ref = sc.ls_solve_direct(op.Plan(d, N, "helmholtz", k), q, pin)
    p = vg.Plan(d, N, "helmholtz", k, precision=precision)
    sigma, info = p.ls_solve(_dev(q, precision), _dev(pin, precision), tol=tol, max_iter=400)
    torch.cuda.synchronize()
    say("  ", info)
    assert info["converged"] == 1 and info["residual"] <= tol
    assert info["matvecs"] <= 2 * info["iterations"]
    check(sigma.cpu().numpy(), ref, bound, "vs direct solve")


def test_ls_large_grids_self_convergence_and_oracle_residual():
    """2D smoothed disk, k = 40 (about six wavelengths across the box):
    the N = 128 and N = 256 solutions agree on shared points, and the N = 128
    GPU solution satisfies the oracle's FP64 equation."""
    import torch

    import paper_1604_03155_amd as vg
    from oracle import operator as op
    from oracle import scattering as sc
    from workloads.scattering import contrast, plane_wave
    k = 40.0
    sols = {}
    for N in (128, 256):
        q, pin = contrast("smoothed_disk", N), plane_wave(2, N, k)
        p = vg.Plan(2, N, "helmholtz", k, precision="fp64")
        t = time.perf_counter()
        sigma, info = p.ls_solve(_dev(q, "fp64"), _dev(pin, "fp64"), tol=1e-12, max_iter=1000)
        torch.cuda.synchronize()
        say("  N", N, info, f"{1e3 * (time.perf_counter() - t):.1f} ms")
        assert info["converged"] == 1
        sols[N] = sigma.cpu().numpy()
    fine = sols[256][1::2, 1::2]
    assert rel_l2(sols[128], fine) <= 1e-6
    q, pin = contrast("smoothed_disk", 128), plane_wave(2, 128, k)
    res = sc.ls_relative_residual(op.Plan(2, 128, "helmholtz", k), q, pin, sols[128])
    say("  oracle residual", res)
    assert res <= 1e-11


def test_ls_3d_smoothed_cube_fp32():
    """3D smoothed cube, k = 20, N = 64, FP32 bulk: converges to 1e-5 and the
    solution satisfies the oracle's FP64 equation at that level."""
    import torch

    import paper_1604_03155_amd as vg
    from oracle import operator as op
    from oracle import scattering as sc
    from workloads.scattering import contrast, plane_wave
    N, k = 64, 20.0
    q, pin = contrast("smoothed_cube", N), plane_wave(3, N, k)
    p = vg.Plan(3, N, "helmholtz", k, precision="fp32")
    ws = torch.empty(p.ls_workspace_size(), dtype=torch.uint8, device="cuda")
    t = time.perf_counter()
    sigma, info = p.ls_solve(_dev(q, "fp32"), _dev(pin, "fp32"), tol=1e-5, max_iter=500, workspace=ws)
    torch.cuda.synchronize()
    say("  3D", info, f"{1e3 * (time.perf_counter() - t):.1f} ms")
    assert info["converged"] == 1
    res = sc.ls_relative_residual(op.Plan(3, N, "helmholtz", k), q, pin, sigma.cpu().numpy())
    say("  oracle residual", res)
    assert res <= 3e-5


def test_ls_rejects_non_helmholtz_plans_and_bad_arguments():
    import paper_1604_03155_amd as vg
    p = vg.Plan(3, 8, "laplace", precision="fp32")
    q = _dev(np.zeros((8, 8, 8), np.complex128), "fp32")
    with pytest.raises(vg.VGError, match="INVALID_ARG"):
        p.ls_solve(q, q)
    h = vg.Plan(3, 8, "helmholtz", 5.0, precision="fp32")
    with pytest.raises(vg.VGError, match="INVALID_ARG"):
        h.ls_solve(q, q, tol=0.0)
    # zero incident field: sigma = 0 at once
    sigma, info = h.ls_solve(q, q)
    assert info["converged"] == 1 and info["iterations"] == 0
    assert float(sigma.abs().max()) == 0.0
