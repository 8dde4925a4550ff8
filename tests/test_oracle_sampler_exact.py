"""Exact pin of the oracle's pair sampler (section "Heuristics and
Approximation Algorithms": the Riondato-Kornaropoulos estimator needs one
shortest u-v path drawn uniformly at random).

Every random choice of a sample is a value in [0, N) for a range N the
procedure itself computes (the meeting-vertex weight sum, then sigma of each
walk vertex).  The oracle can run a sample on given choices instead of
generator draws, and reports the range of every choice it made, so these
tests walk the whole tree of outcomes of one sample, weigh each leaf by the
product of 1/N over its choices (each choice uniform, the reading of the
multiply-shift reduction), and compare the resulting distribution over paths,
in exact rationals, with the shortest paths found by brute-force simple-path
enumeration: every one of the sigma_uv shortest paths must have probability
exactly 1/sigma_uv, and no other sequence may appear.
"""
import itertools
import random
from collections import defaultdict
from fractions import Fraction

import pytest

import graphgen as gg
import oracle
from oracle.bruteforce import all_pairs_paths


def path_distribution(g, u, v):
    """Exact distribution of the interior (listed from v's side) over every
    outcome of the sampler's choices for the pair (u, v).  None keys an
    unreachable pair."""
    dist = defaultdict(Fraction)
    stack = [[]]
    while stack:
        prefix = stack.pop()
        interior, ranges = oracle.sample_path_given(g.rowptr, g.colidx, u, v, prefix)
        # the first choice past the prefix that has more than one value
        i = len(prefix)
        while i < len(ranges) and ranges[i] == 1:
            i += 1
        if i == len(ranges):
            p = Fraction(1)
            for N in ranges:
                p /= N
            dist[None if interior is None else tuple(interior)] += p
        else:
            base = prefix + [0] * (i - len(prefix))
            stack.extend(base + [x] for x in range(ranges[i]))
    return dict(dist)


def _check_graph(g):
    paths = all_pairs_paths(g.rowptr, g.colidx)
    for u in range(g.n):
        for v in range(g.n):
            if u == v:
                continue
            got = path_distribution(g, u, v)
            if (u, v) not in paths:
                assert got == {None: Fraction(1)}, (g.name, u, v)
                continue
            want = {tuple(reversed(p[1:-1])): Fraction(1, len(paths[(u, v)])) for p in paths[(u, v)]}
            assert got == want, (g.name, u, v)


def _all_graphs(n):
    pairs = list(itertools.combinations(range(n), 2))
    for mask in range(1 << len(pairs)):
        es = [p for i, p in enumerate(pairs) if mask >> i & 1]
        yield gg.from_edges(n, [a for a, b in es], [b for a, b in es], f"n{n}_mask{mask}")


@pytest.mark.parametrize("n", [2, 3, 4, 5])
def test_every_labelled_graph_small(n):
    for g in _all_graphs(n):
        _check_graph(g)


@pytest.mark.parametrize("part", range(8))
def test_every_labelled_graph_n6(part):
    """All 2^15 labelled graphs on 6 vertices, in eight interleaved parts."""
    for mask, g in enumerate(_all_graphs(6)):
        if mask % 8 == part:
            _check_graph(g)


@pytest.mark.parametrize("n,count,p", [(7, 40, 0.4), (8, 30, 0.35), (9, 20, 0.3), (10, 15, 0.3)])
def test_random_graphs(n, count, p):
    rng = random.Random(2000 + n)
    for _ in range(count):
        es = [(a, b) for a, b in itertools.combinations(range(n), 2) if rng.random() < p]
        _check_graph(gg.from_edges(n, [a for a, b in es], [b for a, b in es], f"rand{n}"))


def test_structured_graphs():
    """Many shortest paths and meeting vertices of unequal weight."""
    for g in [gg.grid(3, 4), gg.hypercube(3), gg.complete_bipartite(3, 4), gg.diamond_chain(3), gg.cycle(8),
              gg.disjoint_union([gg.cycle(5), gg.star(4)])]:
        _check_graph(g)


def test_given_choices_reproduce_the_generator():
    """The enumeration runs the same code as a generator-driven sample: the
    generator's own choices, given back explicitly one request at a time,
    give the same path (on pairs with many paths and walks of several steps)."""
    g = gg.grid(4, 5)
    for j in range(40):
        u, v = j % 7, 19 - (j % 5)
        want = oracle.sample_path_uv(g.rowptr, g.colidx, 11, j, u, v)
        vals = []
        while True:
            interior, ranges, keys = oracle.sample_path_given(g.rowptr, g.colidx, u, v, vals, with_keys=True)
            if len(ranges) == len(vals):
                break
            stream, t = keys[len(vals)]
            assert stream in (3, 4, 5)
            vals.append(oracle.bounded(oracle.draw(11, stream, j, t), ranges[len(vals)]))
        assert interior == want
