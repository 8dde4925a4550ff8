"""Pins of the CPU oracle against library routines and invariants that hold
at any size:
  - networkx's betweenness (which counts unordered pairs) times 2;
  - scipy breadth-first distances for d;
  - sum over v of BC(v) = sum over ordered reachable pairs of (d(s,t) - 1);
  - per source, sum of dependencies = sum over t of (d(s,t) - 1);
  - d and sigma symmetric in (s, t); isolated vertices and leaves score 0;
  - source-set form with every vertex and scale 1 equals the exact form;
  - duplicated sources count twice; the scale multiplies.
"""
import networkx as nx
import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.csgraph as csg

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
    return csg.shortest_path(A, method="D", unweighted=True, directed=False)


GRAPHS = [
    lambda: gg.erdos_renyi(300, 900, 11),
    lambda: gg.erdos_renyi(400, 500, 12),     # sparse: several components
    lambda: gg.barabasi_albert(500, 3, 13),
    lambda: gg.rmat(9, 8, 14),
    lambda: gg.chung_lu(600, 2.5, 6.0, 15),
    lambda: gg.disjoint_union([gg.grid(5, 7), gg.star(9), gg.path(1), gg.cycle(8)]),
]


@pytest.mark.parametrize("make", GRAPHS)
def test_networkx_times_two(make):
    g = make()
    ref = nx.betweenness_centrality(_nx(g), normalized=False)
    ref = 2.0 * np.array([ref[i] for i in range(g.n)])
    got = oracle.bc_exact(g.rowptr, g.colidx)
    assert np.allclose(got, ref, rtol=1e-12, atol=1e-9)


@pytest.mark.parametrize("make", GRAPHS)
def test_distance_and_sum_invariants(make):
    g = make()
    D = _dist(g)
    bc = oracle.bc_exact(g.rowptr, g.colidx)
    fin = np.isfinite(D) & (D > 0)
    assert np.isclose(bc.sum(), (D[fin] - 1).sum(), rtol=1e-12)
    deg = g.degrees()
    assert np.all(bc[deg <= 1] == 0)
    for s in [0, g.n // 3, g.n - 1]:
        d, sig = oracle.sssp_counts(g.rowptr, g.colidx, s)
        ref = np.where(np.isfinite(D[s]), D[s], -1).astype(np.int64)
        assert np.array_equal(d.astype(np.int64), ref)
        assert np.all((sig > 0) == (d >= 0))
        dep = oracle.bc_sources(g.rowptr, g.colidx, [s])
        row = D[s][np.isfinite(D[s]) & (D[s] > 0)]
        assert np.isclose(dep.sum(), (row - 1).sum(), rtol=1e-12)


@pytest.mark.parametrize("make", GRAPHS[:3])
def test_symmetry(make):
    g = make()
    picks = [0, 7, 42, g.n - 1]
    res = {s: oracle.sssp_counts(g.rowptr, g.colidx, s) for s in picks}
    for s in picks:
        for t in picks:
            assert res[s][0][t] == res[t][0][s]
            assert res[s][1][t] == res[t][1][s]


def test_sources_forms():
    g = gg.barabasi_albert(300, 2, 21)
    ex = oracle.bc_exact(g.rowptr, g.colidx)
    allsrc = oracle.bc_sources(g.rowptr, g.colidx, np.arange(g.n))
    assert np.array_equal(ex, allsrc)
    a = oracle.bc_sources(g.rowptr, g.colidx, [5, 9])
    b = oracle.bc_sources(g.rowptr, g.colidx, [5, 9, 5], scale=0.5)
    c5 = oracle.bc_sources(g.rowptr, g.colidx, [5])
    assert np.allclose(b, 0.5 * (a + c5), rtol=1e-14)
    assert np.array_equal(oracle.bc_sources(g.rowptr, g.colidx, []), np.zeros(g.n))
    # threaded timing mode: same sums, different addition order
    thr = oracle.bc_sources(g.rowptr, g.colidx, np.arange(g.n), nthreads=4)
    assert np.allclose(thr, ex, rtol=1e-12, atol=1e-9)


def test_vertex_transitive_uniform():
    for g in [gg.cycle(17), gg.hypercube(6), gg.complete(9)]:
        b = oracle.bc_exact(g.rowptr, g.colidx)
        assert np.allclose(b, b[0], rtol=1e-12, atol=1e-12)


def test_work_counts():
    g = gg.disjoint_union([gg.path(4), gg.star(4)])
    # from path end 0: reaches 4 vertices, arcs 1+2+2+1=6, DAG arcs 3, depth 3
    assert oracle.work_counts(g.rowptr, g.colidx, [0]) == (4, 6, 3, 3)
    # from the star centre 4: 4 vertices, 3+3 arcs, 3 DAG arcs, depth 1
    assert oracle.work_counts(g.rowptr, g.colidx, [4]) == (4, 6, 3, 1)


def test_validation_codes():
    g = gg.cycle(5)
    assert oracle.validate(g.rowptr, g.colidx) == 0
    assert oracle.validate(g.rowptr, g.colidx, strict=True) == 0
    bad = g.rowptr.copy()
    bad[2], bad[3] = bad[3], bad[2]
    assert oracle.validate(bad, g.colidx) == oracle.E_INVALID_GRAPH
    bad = g.rowptr.copy()
    bad[0] = 1
    assert oracle.validate(bad, g.colidx) == oracle.E_INVALID_GRAPH
    c = g.colidx.copy()
    c[3] = 5
    assert oracle.validate(g.rowptr, c) == oracle.E_INVALID_GRAPH
    assert oracle.validate(g.rowptr, g.colidx, m=g.m - 1) == oracle.E_INVALID_GRAPH
    # asymmetric / unsorted / self loop are caught only by the strict checks
    c = g.colidx.copy()
    c[0], c[1] = c[1], c[0]
    assert oracle.validate(g.rowptr, c) == 0
    assert oracle.validate(g.rowptr, c, strict=True) == oracle.E_INVALID_GRAPH
    loop = gg.Graph(2, np.array([0, 1, 2], dtype=np.int32), np.array([0, 0], dtype=np.int32))
    assert oracle.validate(loop.rowptr, loop.colidx, strict=True) == oracle.E_INVALID_GRAPH
    with pytest.raises(oracle.OracleError):
        oracle.bc_sources(g.rowptr, g.colidx, [7])
