"""Pins of the CPU oracle against exhaustive simple-path enumeration in
exact rationals: every labelled graph on up to 6 vertices, and random graphs
of 6 to 12 vertices (d, sigma and BC all compared)."""
import itertools
import random
from fractions import Fraction

import numpy as np
import pytest

import graphgen as gg
import oracle
from oracle.bruteforce import brute_force


def _check_graph(g):
    d_bf, s_bf, bc_bf = brute_force(g.rowptr, g.colidx)
    bc_or = oracle.bc_exact(g.rowptr, g.colidx)
    for v in range(g.n):
        exact = bc_bf[v]
        assert abs(Fraction(bc_or[v]) - exact) <= Fraction(1, 10 ** 12) * max(1, abs(exact)), (g.name, v)
    for s in range(g.n):
        d, sig = oracle.sssp_counts(g.rowptr, g.colidx, s)
        assert list(d) == d_bf[s]
        assert [int(x) for x in sig] == s_bf[s]


def _all_graphs(n):
    pairs = list(itertools.combinations(range(n), 2))
    for mask in range(1 << len(pairs)):
        es = [p for i, p in enumerate(pairs) if mask >> i & 1]
        u = [a for a, b in es]
        v = [b for a, b in es]
        yield gg.from_edges(n, u, v, f"n{n}_mask{mask}")


@pytest.mark.parametrize("n", [1, 2, 3, 4, 5, 6])
def test_exhaustive_small(n):
    for g in _all_graphs(n):
        _check_graph(g)


@pytest.mark.parametrize("n,count,p", [(6, 60, 0.5), (7, 40, 0.4), (8, 30, 0.35), (9, 15, 0.3),
                                       (10, 8, 0.25), (11, 4, 0.22), (12, 3, 0.2)])
def test_random_small(n, count, p):
    rng = random.Random(1000 + n)
    for _ in range(count):
        es = [(a, b) for a, b in itertools.combinations(range(n), 2) if rng.random() < p]
        g = gg.from_edges(n, [a for a, b in es], [b for a, b in es], f"rand{n}")
        _check_graph(g)


def test_structured_small():
    for g in [gg.grid(3, 3), gg.grid(2, 5), gg.hypercube(3), gg.diamond_chain(3), gg.complete_bipartite(2, 4),
              gg.disjoint_union([gg.cycle(5), gg.path(4), gg.star(3)])]:
        _check_graph(g)
