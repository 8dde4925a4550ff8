"""Pins of the oracle's directed Brandes (out-arc CSR) against path
enumeration, closed forms and the undirected oracle on symmetric inputs."""
from fractions import Fraction

import numpy as np
import pytest
import scipy.sparse as sp
from scipy.sparse.csgraph import shortest_path

import graphgen as gg
import oracle
from oracle import bruteforce as bf

SMALL = [
    lambda: gg.directed_random(9, 20, 1), lambda: gg.directed_random(10, 30, 2), lambda: gg.directed_random(8, 12, 3),
    lambda: gg.directed_from_arcs(6, [0, 0, 1, 2, 3, 4], [1, 2, 3, 3, 4, 5], "diamond-tail"),
    lambda: gg.directed_from_arcs(7, [0, 1, 2, 3, 4, 5, 6, 3], [1, 2, 3, 4, 5, 6, 0, 0], "cycle-chord"),
    lambda: gg.directed_rmat(3, 3, 4),
]


@pytest.mark.parametrize("make", SMALL)
def test_directed_matches_path_enumeration(make):
    """bruteforce follows the adjacency as given, so on an out-arc CSR it
    enumerates directed paths."""
    g = make()
    _, _, ref = bf.brute_force(g.rowptr, g.colidx)
    got = oracle.bc_directed(g.rowptr, g.colidx)
    for v in range(g.n):
        assert abs(Fraction(got[v]) - ref[v]) <= Fraction(1, 10 ** 12) * max(1, abs(ref[v])), (g.name, v)
    sub = [0, g.n - 1, 0]
    got = oracle.bc_directed(g.rowptr, g.colidx, sub, 3.0)
    dep = [Fraction(0)] * g.n
    paths = bf.all_pairs_paths(g.rowptr, g.colidx)
    for s in sub:
        for t in range(g.n):
            for p in paths.get((s, t), []):
                for v in p[1:-1]:
                    dep[v] += Fraction(1, len(paths[(s, t)]))
    for v in range(g.n):
        assert abs(Fraction(got[v]) - 3 * dep[v]) <= Fraction(1, 10 ** 12) * max(1, abs(3 * dep[v]))


@pytest.mark.parametrize("make", [lambda: gg.erdos_renyi(300, 700, 5), lambda: gg.barabasi_albert(400, 3, 6),
                                  lambda: gg.grid(9, 11)])
def test_symmetric_input_equals_undirected(make):
    g = make()
    assert np.allclose(oracle.bc_directed(g.rowptr, g.colidx), oracle.bc_exact(g.rowptr, g.colidx),
                       rtol=1e-12, atol=1e-10)


def test_directed_path_and_cycle_closed_forms():
    n = 30
    p = gg.directed_from_arcs(n, np.arange(n - 1), np.arange(1, n))
    assert np.array_equal(oracle.bc_directed(p.rowptr, p.colidx),
                          np.array([float(v * (n - 1 - v)) for v in range(n)]))
    c = gg.directed_from_arcs(n, np.arange(n), (np.arange(n) + 1) % n)
    assert np.array_equal(oracle.bc_directed(c.rowptr, c.colidx), np.full(n, (n - 1) * (n - 2) / 2.0))


def test_directed_reachability_matches_scipy():
    """A vertex that no other vertex reaches, or that reaches no other
    vertex, lies inside no directed path and scores 0 (reachability from
    scipy's directed distances)."""
    g = gg.directed_rmat(8, 4, 7)
    bc = oracle.bc_directed(g.rowptr, g.colidx)
    a = sp.csr_matrix((np.ones(g.m), g.colidx, g.rowptr), shape=(g.n, g.n))
    dist = shortest_path(a, directed=True, unweighted=True)
    reach_in = np.isfinite(dist).sum(axis=0) - 1    # vertices that reach v
    reach_out = np.isfinite(dist).sum(axis=1) - 1   # vertices v reaches
    assert np.all(bc[(reach_in == 0) | (reach_out == 0)] == 0.0)
    assert (bc > 0).sum() > 0


def test_transpose_helper():
    g = gg.directed_random(50, 200, 8)
    t = gg.transpose(g)
    assert t.m == g.m
    a = sp.csr_matrix((np.ones(g.m), g.colidx, g.rowptr), shape=(g.n, g.n))
    b = sp.csr_matrix((np.ones(t.m), t.colidx, t.rowptr), shape=(g.n, g.n))
    assert (a.T != b).nnz == 0
