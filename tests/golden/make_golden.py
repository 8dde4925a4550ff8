"""Writes bruteforce_small.json: exact d, sigma and betweenness (as
fractions, ordered-pair convention) for a few small graphs, computed only by
the all-simple-paths enumeration in oracle/bruteforce.py.

The paper prints no worked example with betweenness values (its only
printed values are top-10 rankings on a dataset that is not available), so
these stored values come from the definition of betweenness evaluated
exactly.  Run from the repository root:  python tests/golden/make_golden.py
"""
import json
import os
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import graphgen as gg  # noqa: E402
from oracle.bruteforce import brute_force  # noqa: E402


def main():
    cases = [
        gg.grid(3, 4),
        gg.hypercube(3),
        gg.diamond_chain(3),
        gg.disjoint_union([gg.cycle(5), gg.star(4), gg.path(1)]),
        gg.erdos_renyi(11, 18, 77),
        gg.barabasi_albert(12, 2, 78),
    ]
    out = []
    for g in cases:
        d, s, bc = brute_force(g.rowptr, g.colidx)
        out.append({
            "name": g.name,
            "n": g.n,
            "rowptr": g.rowptr.tolist(),
            "colidx": g.colidx.tolist(),
            "d": d,
            "sigma": s,
            "bc": [f"{x.numerator}/{x.denominator}" for x in bc],
        })
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "bruteforce_small.json")
    with open(path, "w") as f:
        json.dump(out, f, separators=(",", ":"))
        f.write("\n")
    print("wrote", path)


if __name__ == "__main__":
    main()
