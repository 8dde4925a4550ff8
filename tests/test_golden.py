"""The oracle against the stored brute-force fixtures in tests/golden/."""
import json
import os
from fractions import Fraction

import numpy as np

import oracle

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "bruteforce_small.json")


def load_golden():
    with open(GOLDEN) as f:
        return json.load(f)


def test_oracle_matches_golden():
    for case in load_golden():
        rp = np.array(case["rowptr"], dtype=np.int32)
        ci = np.array(case["colidx"], dtype=np.int32)
        got = oracle.bc_exact(rp, ci)
        for v, frac in enumerate(case["bc"]):
            exact = Fraction(frac)
            assert abs(Fraction(got[v]) - exact) <= Fraction(1, 10 ** 12) * max(1, abs(exact))
        for s in range(case["n"]):
            d, sig = oracle.sssp_counts(rp, ci, s)
            assert d.tolist() == case["d"][s]
            assert [int(x) for x in sig] == case["sigma"][s]
