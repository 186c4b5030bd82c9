"""Parity measures shared by the GPU tests: a result is compared with its
reference element by element, by two relative errors over all elements,
  rel L2  = ||a - b||_2 / ||b||_2,
  rel max = max_i |a_i - b_i| / max_i |b_i|,
each held to the same bar (1e-5 for FP32 bulk, 1e-12 for the FP64 path).
The norm alone would let an error confined to a small region pass (1e-3 on
one pencil of a 256^3 grid is 1e-5 in L2); the max catches it."""
import sys

import numpy as np


def rel_l2(a, b):
    a, b = np.asarray(a), np.asarray(b)
    return float(np.linalg.norm(a - b) / np.linalg.norm(b))


def rel_max(a, b):
    a, b = np.asarray(a), np.asarray(b)
    return float(np.max(np.abs(a - b)) / np.max(np.abs(b)))


def check(got, ref, tol, what=""):
    """Assert rel L2 <= tol and rel max <= tol; returns (rel L2, rel max)."""
    l2, mx = rel_l2(got, ref), rel_max(got, ref)
    print(f"  parity {what}: rel L2 {l2:.3e}, rel max {mx:.3e} (bar {tol:.0e})", flush=True)
    sys.stdout.flush()
    assert l2 <= tol and mx <= tol, f"{what}: rel L2 {l2:.3e}, rel max {mx:.3e} above {tol:.1e}"
    return l2, mx
