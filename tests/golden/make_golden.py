"""Write the stored oracle fixtures in this folder.

Calls only the oracle (and the seeded input module).  Run from the repository
root:  python tests/golden/make_golden.py
The fixtures guard the oracle against unintended changes: a change to its
arithmetic that moves these values must name the passage of the paper that
justifies it.
"""
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import numpy as np  # noqa: E402

from oracle import operator as op  # noqa: E402


def main():
    out = {}
    for name, (d, N, kernel, k) in {
        "laplace3d_n8": (3, 8, "laplace", 0.0),
        "helmholtz3d_k20_n8": (3, 8, "helmholtz", 20.0),
        "laplace2d_n16": (2, 16, "laplace", 0.0),
        "helmholtz2d_k30_n16": (2, 16, "helmholtz", 30.0),
    }.items():
        plan = op.Plan(d, N, kernel, k, route="full")
        # a few entries of T and of Khat (octant indices)
        idx = [(0,) * d, (1,) + (0,) * (d - 1), tuple(range(1, d + 1)), (N - 1,) * d]
        kidx = [(0,) * d, (N,) * d, tuple(range(2, d + 2))]
        out[name] = {
            "d": d, "N": N, "kernel": kernel, "k": k,
            "T": [[list(i), plan.T_oct[i].real, plan.T_oct[i].imag] for i in idx],
            "Khat": [[list(i), plan.K_oct[i].real, plan.K_oct[i].imag] for i in kidx],
        }
    with open(os.path.join(HERE, "oracle_operator_entries.json"), "w") as fh:
        json.dump(out, fh, indent=1)
        fh.write("\n")


if __name__ == "__main__":
    main()
