"""GPU: the real-data path (real densities, real kernels) on the half
spectrum, against the FP64 oracle and the complex path (relative L2 and
relative max error, 1e-12 FP64 / 1e-5 FP32)."""
import sys

import numpy as np
import pytest

from parity import check  # noqa: E402

pytestmark = pytest.mark.gpu

FP32_TOL = 1e-5
FP64_TOL = 1e-12


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()




CASES = [(3, 32, "laplace", "fp32"), (3, 64, "biharmonic", "fp32"), (3, 128, "laplace", "fp32"),
         (3, 32, "laplace", "fp64"), (3, 64, "biharmonic", "fp64"), (2, 64, "laplace", "fp32"),
         (2, 256, "biharmonic", "fp32"), (2, 512, "laplace", "fp64"), (2, 1024, "laplace", "fp32"),
         (2, 1024, "biharmonic", "fp64"),
         # mixed-radix lengths (rows of N, columns of 2N with radix-3 / radix-5 stages)
         (3, 100, "laplace", "fp32"), (3, 200, "laplace", "fp32"), (3, 100, "biharmonic", "fp64"),
         (2, 200, "laplace", "fp32"), (2, 3200, "laplace", "fp32")]


@pytest.mark.parametrize("d,N,kernel,precision", CASES)
def test_real_apply_matches_oracle_and_complex_path(d, N, kernel, precision):
    import torch

    import paper_1604_03155_amd as vg
    from oracle import operator as op
    say("real", d, N, kernel, precision)
    rng = np.random.default_rng(700 + N)
    f = rng.standard_normal((N,) * d)
    rdt = torch.float64 if precision == "fp64" else torch.float32
    cdt = torch.complex128 if precision == "fp64" else torch.complex64
    p = vg.Plan(d, N, kernel, precision=precision)
    fr = torch.from_numpy(f).to(rdt).cuda()
    phi = p.apply_real(fr)
    phic = p.apply(fr.to(cdt))
    torch.cuda.synchronize()
    ref = op.Plan(d, N, kernel).apply(f.astype(np.complex128))
    tol = FP64_TOL if precision == "fp64" else FP32_TOL
    assert np.max(np.abs(ref.imag)) <= 1e-12 * np.max(np.abs(ref.real))
    check(phi.cpu().numpy(), ref.real, tol, "vs oracle")
    check(phi.cpu().numpy(), phic.real.cpu().numpy(), tol, "vs complex path")
    # in place
    g = fr.clone()
    p.apply_real(g, out=g)
    torch.cuda.synchronize()
    assert torch.equal(g, phi)


def test_real_apply_rejections():
    import torch

    import paper_1604_03155_amd as vg
    h = vg.Plan(3, 16, "helmholtz", 5.0)
    f = torch.zeros((16, 16, 16), dtype=torch.float32, device="cuda")
    with pytest.raises(vg.VGError, match="INVALID_ARG"):
        h.apply_real(f)
    odd = vg.Plan(3, 30, "laplace")  # row length 30: no specialised kernel
    f30 = torch.zeros((30, 30, 30), dtype=torch.float32, device="cuda")
    with pytest.raises(vg.VGError, match="UNSUPPORTED_SIZE"):
        odd.apply_real(f30)
