"""Pins of the oracle's weighted Brandes (Dijkstra forward phase) against
weighted path enumeration, scipy's Dijkstra distances, unit weights and
small hand-checked cases."""
from fractions import Fraction

import numpy as np
import pytest
import scipy.sparse as sp
from scipy.sparse.csgraph import dijkstra

import graphgen as gg
import oracle
from oracle import bruteforce as bf

SMALL = [
    (lambda: gg.erdos_renyi(9, 14, 3), 3, True), (lambda: gg.grid(3, 3), 2, True),
    (lambda: gg.cycle(8), 4, True), (lambda: gg.complete_bipartite(2, 4), 3, True),
    (lambda: gg.barabasi_albert(9, 2, 5), 5, True), (lambda: gg.directed_random(9, 24, 6), 3, False),
    (lambda: gg.diamond_chain(2), 1, True),
]


@pytest.mark.parametrize("make,wmax,sym", SMALL)
def test_weighted_matches_path_enumeration(make, wmax, sym):
    g = make()
    w = gg.edge_weights(g, wmax, 7, symmetric=sym)
    d, sigma, ref = bf.brute_force_weighted(g.rowptr, g.colidx, w)
    got = oracle.bc_weighted(g.rowptr, g.colidx, w)
    for v in range(g.n):
        assert abs(Fraction(got[v]) - ref[v]) <= Fraction(1, 10 ** 12) * max(1, abs(ref[v])), (g.name, v)
    for s in range(g.n):
        od, osg = oracle.sssp_weighted(g.rowptr, g.colidx, w, s)
        assert list(od) == d[s]
        assert [int(x) for x in osg] == [sigma[s][t] if d[s][t] >= 0 else 0 for t in range(g.n)]


@pytest.mark.parametrize("make,sym", [(lambda: gg.erdos_renyi(400, 1200, 8), True),
                                      (lambda: gg.barabasi_albert(500, 3, 9), True),
                                      (lambda: gg.directed_rmat(9, 6, 10), False)])
def test_weighted_distances_match_scipy(make, sym):
    g = make()
    w = gg.edge_weights(g, 20, 11, symmetric=sym)
    a = sp.csr_matrix((w.astype(np.float64), g.colidx, g.rowptr), shape=(g.n, g.n))
    for s in (0, g.n // 3, g.n - 1):
        ref = dijkstra(a, directed=True, indices=s)
        d, sigma = oracle.sssp_weighted(g.rowptr, g.colidx, w, s)
        reach = np.isfinite(ref)
        assert np.array_equal(d[reach], ref[reach].astype(np.int64))
        assert np.all(d[~reach] == -1) and np.all(sigma[~reach] == 0) and np.all(sigma[reach] >= 1)


@pytest.mark.parametrize("c", [1, 7])
def test_uniform_weights_equal_unweighted(c):
    g = gg.barabasi_albert(600, 3, 12)
    w = np.full(g.m, c, dtype=np.int32)
    assert np.allclose(oracle.bc_weighted(g.rowptr, g.colidx, w), oracle.bc_exact(g.rowptr, g.colidx),
                       rtol=1e-12, atol=1e-10)
    h = gg.directed_rmat(9, 6, 13)
    assert np.allclose(oracle.bc_weighted(h.rowptr, h.colidx, np.full(h.m, c, dtype=np.int32)),
                       oracle.bc_directed(h.rowptr, h.colidx), rtol=1e-12, atol=1e-10)


def test_triangle_detour_and_tie():
    """Edges 0-1 and 1-2 of weight 1 and 0-2 of weight w: with w = 3 both
    ordered pairs (0, 2) and (2, 0) go through 1; with w = 2 half of their
    shortest paths do; with w = 1 none."""
    g = gg.from_edges(3, [0, 1, 0], [1, 2, 2])
    for w02, want in ((3, 2.0), (2, 1.0), (1, 0.0)):
        w = np.array([1 if {u, v} != {0, 2} else w02
                      for u in range(3) for v in g.colidx[g.rowptr[u]:g.rowptr[u + 1]]], dtype=np.int32)
        assert oracle.bc_weighted(g.rowptr, g.colidx, w)[1] == want


def test_weighted_sources_scale_and_errors():
    g = gg.erdos_renyi(200, 500, 14)
    w = gg.edge_weights(g, 9, 15)
    full = oracle.bc_weighted(g.rowptr, g.colidx, w, nthreads=4)
    parts = oracle.bc_weighted(g.rowptr, g.colidx, w, np.arange(0, 100)) + \
        oracle.bc_weighted(g.rowptr, g.colidx, w, np.arange(100, 200), scale=1.0)
    assert np.allclose(full, parts, rtol=1e-12, atol=1e-10)
    assert np.allclose(oracle.bc_weighted(g.rowptr, g.colidx, w, [5, 6], scale=3.0),
                       3.0 * oracle.bc_weighted(g.rowptr, g.colidx, w, [5, 6]), rtol=1e-15)
    bad = w.copy()
    bad[3] = 0
    with pytest.raises(oracle.OracleError):
        oracle.bc_weighted(g.rowptr, g.colidx, bad)
