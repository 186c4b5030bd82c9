"""vg_apply_noalloc through the C ABI: the allocation-free apply (workspace in
the library's fixed per-GPU array) against vg_apply with a caller workspace
on the same plan and density.  Both run the same kernels and launches, so the
outputs must agree bit for bit (stricter than the 1e-5 / 1e-12 parity bars).
Two calls in a row, the second on a smaller grid, check that nothing of the
first call's array contents leaks into the second; an oversized plan is
rejected before any launch."""
import ctypes

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


@pytest.fixture(scope="module")
def vg():
    import paper_1604_03155_amd as vg
    return vg


def _density(N, d, seed, dtype):
    from workloads import draw_gaussian_sum, evaluate_grid
    src = draw_gaussian_sum(seed, d, 4, 0.2, (0.04, 0.08), mod_max=8.0)
    return torch.from_numpy(evaluate_grid(src, N)).to(dtype).cuda()


def _run_both(vg, plan, x):
    """(vg_apply output, vg_apply_noalloc output), both called through ctypes."""
    lib = ctypes.CDLL(vg.LIBRARY_PATH)
    lib.vg_apply.argtypes = [ctypes.c_void_p] * 5
    lib.vg_apply.restype = ctypes.c_int
    lib.vg_apply_noalloc.argtypes = [ctypes.c_void_p] * 4
    lib.vg_apply_noalloc.restype = ctypes.c_int
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    ref = torch.full_like(x, float("nan"))
    got = torch.full_like(x, float("nan"))
    ws = plan.new_workspace()
    assert lib.vg_apply(plan.handle, x.data_ptr(), ref.data_ptr(), ws.data_ptr(), stream) == 0
    assert lib.vg_apply_noalloc(plan.handle, x.data_ptr(), got.data_ptr(), stream) == 0
    torch.cuda.synchronize()
    return ref, got


CASES = [
    # (d, N, kernel, k, precision): the first call's grid is the larger one
    [(3, 64, "helmholtz", 20.0, "fp32"), (3, 32, "laplace", 0.0, "fp32")],
    [(3, 128, "helmholtz", 20.0, "fp32"), (3, 48, "helmholtz", 9.0, "fp32")],
    [(3, 96, "laplace", 0.0, "fp64"), (3, 40, "helmholtz", 5.0, "fp64")],
    [(2, 1024, "helmholtz", 200.0, "fp32"), (2, 100, "laplace", 0.0, "fp32")],
]


@pytest.mark.parametrize("case", CASES, ids=lambda c: f"{c[0][0]}d{c[0][1]}-{c[1][0]}d{c[1][1]}-{c[0][4]}")
def test_noalloc_matches_apply_two_calls(vg, case):
    for i, (d, N, kernel, k, prec) in enumerate(case):
        print(f"noalloc: call {i} d={d} N={N} {kernel} k={k} {prec}", flush=True)
        plan = vg.Plan(d, N, kernel, k, precision=prec)
        assert plan.workspace_size() <= 128 << 20
        x = _density(N, d, 40 + i, plan.dtype)
        ref, got = _run_both(vg, plan, x)
        assert torch.isfinite(torch.view_as_real(ref)).all()
        assert torch.equal(torch.view_as_real(got), torch.view_as_real(ref))
        # the binding's method takes the same path
        out = torch.empty_like(x)
        plan.apply_noalloc(x, out)
        torch.cuda.synchronize()
        assert torch.equal(torch.view_as_real(out), torch.view_as_real(ref))


def test_noalloc_in_place(vg):
    plan = vg.Plan(3, 64, "helmholtz", 12.0)
    x = _density(64, 3, 7, plan.dtype)
    ref = plan.apply(x, workspace=plan.new_workspace())
    y = x.clone()
    plan.apply_noalloc(y, y)
    torch.cuda.synchronize()
    assert torch.equal(torch.view_as_real(y), torch.view_as_real(ref))


def test_noalloc_matches_oracle(vg):
    from oracle import operator as op
    N, k = 40, 15.0
    plan = vg.Plan(3, N, "helmholtz", k)
    x = _density(N, 3, 11, plan.dtype)
    out = torch.empty_like(x)
    plan.apply_noalloc(x, out)
    torch.cuda.synchronize()
    ref = op.Plan(3, N, "helmholtz", k).apply(x.cpu().numpy().astype(np.complex128))
    got = out.cpu().numpy().astype(np.complex128)
    assert np.linalg.norm(got - ref) / np.linalg.norm(ref) <= 1e-5
    assert np.max(np.abs(got - ref)) / np.max(np.abs(ref)) <= 1e-5


def test_oversized_plan_is_rejected(vg):
    plan = vg.Plan(3, 160, "laplace", 0.0)
    assert plan.workspace_size() > 128 << 20
    x = torch.zeros((160,) * 3, dtype=plan.dtype, device="cuda")
    with pytest.raises(vg.VGError) as e:
        plan.apply_noalloc(x, torch.empty_like(x))
    assert e.value.code == 2  # VG_ERR_UNSUPPORTED_SIZE
    assert "VG_NOALLOC_WORKSPACE_BYTES" in str(e.value)
