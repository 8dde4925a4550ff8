"""Pins of the oracle's closeness (exact, generalised to disconnected
graphs) and Eppstein-Wang sampled closeness: closed forms, networkx's
closeness_centrality (whose default is the same generalisation) and BFS
distances from scipy."""
import networkx as nx
import numpy as np
import pytest
import scipy.sparse as sp
from scipy.sparse.csgraph import shortest_path

import graphgen as gg
import oracle


def _nx(g):
    G = nx.Graph()
    G.add_nodes_from(range(g.n))
    u, v = g.edges()
    G.add_edges_from(zip(u.tolist(), v.tolist()))
    return G


def _dist(g):
    A = sp.csr_matrix((np.ones(g.m), g.colidx, g.rowptr), shape=(g.n, g.n))
    return shortest_path(A, directed=False, unweighted=True)


def test_closed_forms():
    n = 30
    p = gg.path(n)
    want = [(n - 1) / sum(abs(i - j) for j in range(n)) for i in range(n)]
    assert np.allclose(oracle.closeness(p.rowptr, p.colidx), want, rtol=1e-14)
    st = gg.star(20)                     # centre 0, 19 leaves
    c = oracle.closeness(st.rowptr, st.colidx)
    assert c[0] == pytest.approx(1.0) and np.allclose(c[1:], 19 / (1 + 2 * 18))
    k = gg.complete(12)
    assert np.allclose(oracle.closeness(k.rowptr, k.colidx), 1.0)
    iso = gg.disjoint_union([gg.path(1), gg.cycle(5)])
    c = oracle.closeness(iso.rowptr, iso.colidx)
    assert c[0] == 0.0 and np.allclose(c[1:], (4 / 5) * (4 / 6))   # r = 5, n = 6, farness 6


@pytest.mark.parametrize("make", [
    lambda: gg.erdos_renyi(300, 700, 1), lambda: gg.erdos_renyi(400, 300, 2),   # the second is disconnected
    lambda: gg.barabasi_albert(500, 2, 3), lambda: gg.grid(9, 14), lambda: gg.rmat(9, 8, 4),
])
def test_matches_networkx(make):
    g = make()
    ref = nx.closeness_centrality(_nx(g))
    got = oracle.closeness(g.rowptr, g.colidx)
    assert np.allclose(got, [ref[v] for v in range(g.n)], rtol=1e-12, atol=1e-15)


@pytest.mark.parametrize("make", [lambda: gg.barabasi_albert(400, 3, 5), lambda: gg.erdos_renyi(300, 500, 6)])
def test_approx_sums_are_distance_sums(make):
    """The integer sums are sum over the sources of d(s, v) (scipy BFS); with
    every vertex as a source on a connected graph the estimate is exact."""
    g = make()
    D = _dist(g)
    src = gg.sample_sources(g.n, 37, 7)
    est, sums = oracle.closeness_approx(g.rowptr, g.colidx, src)
    Dm = np.where(np.isfinite(D), D, 0.0)
    assert np.array_equal(sums, Dm[src].sum(axis=0).astype(np.int64))
    F = g.n / len(src) * sums
    assert np.allclose(est, np.where(F > 0, (g.n - 1) / np.where(F > 0, F, 1), 0.0), rtol=1e-15)
    if np.isfinite(D).all():
        full, _ = oracle.closeness_approx(g.rowptr, g.colidx, np.arange(g.n))
        assert np.allclose(full, oracle.closeness(g.rowptr, g.colidx), rtol=1e-13)


def test_approx_unbiased_farness():
    """E[n/k * sum d(s, v)] over uniform sources is the farness of v."""
    g = gg.barabasi_albert(200, 2, 8)
    D = _dist(g)
    acc = np.zeros(g.n)
    T = 300
    for t in range(T):
        src = gg.sample_sources(g.n, 10, 100 + t)
        _, sums = oracle.closeness_approx(g.rowptr, g.colidx, src)
        acc += g.n / 10 * sums
    est = acc / T
    far = D.sum(axis=0)
    assert np.max(np.abs(est - far) / far) < 0.05
