"""The oracle against stored fixtures: the paper's printed constants, and
entries of T and Khat written by tests/golden/make_golden.py (which calls only
the oracle) so that any change to the oracle's arithmetic is noticed."""
import json
import os

import numpy as np

from oracle import greens
from oracle import operator as op

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_paper_constants():
    with open(os.path.join(GOLDEN, "paper_constants.json")) as fh:
        c = json.load(fh)
    assert greens.L_DEFAULT[3] == c["truncation_radius"]["3"]["value"]
    assert greens.L_DEFAULT[2] == c["truncation_radius"]["2"]["value"]
    assert op.P_DEFAULT == c["oversampling_factor"]["value"]
    # L exceeds the box diameter sqrt(d), as the truncation argument requires
    assert greens.L_DEFAULT[3] > 3 ** 0.5 and greens.L_DEFAULT[2] > 2 ** 0.5
    # images of the periodised kernel miss the box: P - 1 > L per axis
    assert op.P_DEFAULT - 1 > greens.L_DEFAULT[3]


def test_stored_operator_entries():
    with open(os.path.join(GOLDEN, "oracle_operator_entries.json")) as fh:
        data = json.load(fh)
    for name, e in data.items():
        plan = op.Plan(e["d"], e["N"], e["kernel"], e["k"], route="full")
        for idx, re, im in e["T"]:
            assert abs(plan.T_oct[tuple(idx)] - complex(re, im)) <= 1e-15 * np.abs(plan.T_oct).max(), (name, idx)
        for idx, re, im in e["Khat"]:
            assert abs(plan.K_oct[tuple(idx)] - complex(re, im)) <= 1e-14 * np.abs(plan.K_oct).max(), (name, idx)
