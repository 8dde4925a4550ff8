"""Pins of the oracle's linear-scaling and bisection estimators
(Geisberger, Sanders and Schultes) and edge betweenness against brute force,
closed forms and invariants computed independently of it (scipy shortest
paths and components)."""
from fractions import Fraction

import numpy as np
import pytest
import scipy.sparse as sp
from scipy.sparse.csgraph import connected_components, shortest_path

import graphgen as gg
import oracle
from oracle import bruteforce as bf


def _csr(g):
    return sp.csr_matrix((np.ones(g.m), g.colidx, g.rowptr), shape=(g.n, g.n))


SMALL = [
    lambda: gg.erdos_renyi(9, 14, 3), lambda: gg.erdos_renyi(10, 12, 4), lambda: gg.barabasi_albert(9, 2, 5),
    lambda: gg.grid(3, 3), lambda: gg.cycle(7), lambda: gg.complete_bipartite(2, 4), lambda: gg.diamond_chain(2),
    lambda: gg.disjoint_union([gg.path(4), gg.cycle(4)]), lambda: gg.star(6),
]


@pytest.mark.parametrize("make", SMALL)
def test_linear_matches_definition_by_enumeration(make):
    g = make()
    for sources in (list(range(g.n)), [0, g.n - 1, g.n // 2], [1, 1]):
        got = oracle.bc_sources_linear(g.rowptr, g.colidx, sources)
        ref = bf.linear_dependencies(g.rowptr, g.colidx, sources)
        for v in range(g.n):
            assert abs(Fraction(got[v]) - ref[v]) <= Fraction(1, 10 ** 12) * max(1, abs(ref[v])), (g.name, v)


@pytest.mark.parametrize("make", SMALL + [lambda: gg.cycle(8), lambda: gg.path(9)])
def test_bisect_matches_definition_by_enumeration(make):
    g = make()
    for sources in (list(range(g.n)), [0, g.n - 1, g.n // 2], [1, 1]):
        got = oracle.bc_sources_bisect(g.rowptr, g.colidx, sources)
        ref = bf.bisection_dependencies(g.rowptr, g.colidx, sources)
        for v in range(g.n):
            assert abs(Fraction(got[v]) - ref[v]) <= Fraction(1, 10 ** 12) * max(1, abs(ref[v])), (g.name, v)


@pytest.mark.parametrize("make", SMALL)
def test_edge_matches_definition_by_enumeration(make):
    g = make()
    ebc, bc = oracle.edge_bc(g.rowptr, g.colidx)
    ref = bf.edge_betweenness(g.rowptr, g.colidx)
    for u in range(g.n):
        for e in range(g.rowptr[u], g.rowptr[u + 1]):
            v = int(g.colidx[e])
            exact = ref[(min(u, v), max(u, v))]
            assert abs(Fraction(ebc[e]) - exact) <= Fraction(1, 10 ** 12) * max(1, abs(exact)), (g.name, u, v)
    _, _, vbc = bf.brute_force(g.rowptr, g.colidx)
    assert np.allclose(bc, [float(x) for x in vbc], rtol=1e-12, atol=1e-12)


MID = [
    lambda: gg.erdos_renyi(400, 900, 11), lambda: gg.barabasi_albert(600, 3, 12), lambda: gg.grid(12, 15),
    lambda: gg.random_tree(500, 13), lambda: gg.disjoint_union([gg.cycle(31), gg.complete(9), gg.path(1)]),
]


@pytest.mark.parametrize("make", MID)
def test_linear_over_all_sources_is_half_of_exact(make):
    """f(x) = x satisfies f(x) + f(1 - x) = 1, so over all ordered pairs each
    path is counted once in total from its two ends: twice the all-source
    linear sum is exact betweenness."""
    g = make()
    lin = oracle.bc_sources_linear(g.rowptr, g.colidx, np.arange(g.n))
    ex = oracle.bc_exact(g.rowptr, g.colidx)
    assert np.allclose(2.0 * lin, ex, rtol=1e-11, atol=1e-9)
    twice = oracle.bc_sources_linear(g.rowptr, g.colidx, np.arange(g.n), scale=2.0, nthreads=4)
    assert np.allclose(twice, ex, rtol=1e-11, atol=1e-9)


@pytest.mark.parametrize("make", MID)
def test_bisect_over_all_sources_is_half_of_exact(make):
    """The bisection weight f (1 above one half, 1/2 at one half, 0 below)
    also satisfies f(x) + f(1 - x) = 1."""
    g = make()
    bis = oracle.bc_sources_bisect(g.rowptr, g.colidx, np.arange(g.n), scale=2.0, nthreads=4)
    assert np.allclose(bis, oracle.bc_exact(g.rowptr, g.colidx), rtol=1e-11, atol=1e-9)


@pytest.mark.parametrize("n", [2, 3, 4, 9, 40])
def test_bisect_single_source_on_a_path(n):
    """Path 0..n-1 from source 0: v lies on the unique path to every t > v;
    it counts fully for v < t < 2v and half for t = 2v."""
    g = gg.path(n)
    got = oracle.bc_sources_bisect(g.rowptr, g.colidx, [0])
    want = [0.0] * n
    for v in range(1, n - 1):
        want[v] = float(sum(1 for t in range(v + 1, n) if t < 2 * v)) + (0.5 if 2 * v <= n - 1 else 0.0)
    assert np.array_equal(got, np.array(want))


def test_bisect_differs_from_linear_and_plain():
    """On a graph with paths of several lengths the three source-set sums are
    pairwise different (a swapped estimator would not pass the GPU parity
    tests unnoticed)."""
    g = gg.barabasi_albert(300, 2, 14)
    src = [0, 7, 99]
    a = oracle.bc_sources(g.rowptr, g.colidx, src)
    b = oracle.bc_sources_linear(g.rowptr, g.colidx, src)
    c = oracle.bc_sources_bisect(g.rowptr, g.colidx, src)
    assert not np.allclose(a, b) and not np.allclose(b, c) and not np.allclose(a, c)


def test_linear_single_source_on_a_path():
    """Path 0..n-1 from source 0: v lies on the paths to every t > v with
    weight v / t, so delta(v) = v * (H(n-1) - H(v))."""
    n = 40
    g = gg.path(n)
    got = oracle.bc_sources_linear(g.rowptr, g.colidx, [0])
    H = np.concatenate([[0.0], np.cumsum(1.0 / np.arange(1, n))])
    want = np.array([v * (H[n - 1] - H[v]) if 0 < v < n - 1 else 0.0 for v in range(n)])
    assert np.allclose(got, want, rtol=1e-13, atol=1e-13)


def test_edge_path_and_tree_closed_forms():
    n = 50
    g = gg.path(n)
    ebc, _ = oracle.edge_bc(g.rowptr, g.colidx)
    for u in range(n - 1):
        e = g.rowptr[u] + (1 if u > 0 else 0)  # arc u -> u+1
        assert g.colidx[e] == u + 1
        assert ebc[e] == pytest.approx(2.0 * (u + 1) * (n - 1 - u), rel=1e-13)
    # any tree: removing edge {u, v} splits it into parts A and B, score 2|A||B|
    t = gg.random_tree(300, 21)
    ebc, _ = oracle.edge_bc(t.rowptr, t.colidx, nthreads=4)
    A = _csr(t).tolil()
    for u in range(0, t.n, 7):
        for e in range(t.rowptr[u], t.rowptr[u + 1]):
            v = int(t.colidx[e])
            cut = A.copy()
            cut[u, v] = 0
            cut[v, u] = 0
            _, lab = connected_components(cut.tocsr(), directed=False)
            a = int(np.sum(lab == lab[u]))
            assert ebc[e] == pytest.approx(2.0 * a * (t.n - a), rel=1e-12)


@pytest.mark.parametrize("make", MID)
def test_edge_sums(make):
    """Every shortest s-t path has d(s,t) edges, so the edge scores sum to
    the sum of distances over ordered reachable pairs; the edges at v carry
    twice v's vertex score plus one unit per pair with v as an endpoint."""
    g = make()
    ebc, bc = oracle.edge_bc(g.rowptr, g.colidx, nthreads=4)
    D = shortest_path(_csr(g), directed=False, unweighted=True)
    reach = np.isfinite(D)
    assert np.sum(ebc) / 2.0 == pytest.approx(float(np.sum(D[reach])), rel=1e-11)
    _, lab = connected_components(_csr(g), directed=False)
    comp = np.bincount(lab)[lab]
    tail = np.repeat(np.arange(g.n), np.diff(g.rowptr))
    inc = np.bincount(tail, weights=ebc, minlength=g.n)
    ex = oracle.bc_exact(g.rowptr, g.colidx)
    assert np.allclose(inc, 2.0 * ex + 2.0 * (comp - 1), rtol=1e-11, atol=1e-9)
    assert np.allclose(bc, ex, rtol=1e-12, atol=1e-12)


def test_edge_sources_scale_and_subsets():
    g = gg.barabasi_albert(300, 2, 31)
    full, _ = oracle.edge_bc(g.rowptr, g.colidx)
    a, _ = oracle.edge_bc(g.rowptr, g.colidx, sources=np.arange(0, 150))
    b, _ = oracle.edge_bc(g.rowptr, g.colidx, sources=np.arange(150, 300))
    assert np.allclose(a + b, full, rtol=1e-12, atol=1e-12)
    s, _ = oracle.edge_bc(g.rowptr, g.colidx, sources=np.arange(0, 150), scale=2.5)
    assert np.allclose(s, 2.5 * a, rtol=1e-14)
    none, vb = oracle.edge_bc(g.rowptr, g.colidx, sources=np.zeros(0, dtype=np.int32))
    assert not none.any() and not vb.any()


def test_edge_needs_reverse_arcs():
    rowptr = np.array([0, 1, 1], dtype=np.int32)   # arc 0 -> 1 without 1 -> 0
    colidx = np.array([1], dtype=np.int32)
    with pytest.raises(oracle.OracleError) as e:
        oracle.edge_bc(rowptr, colidx)
    assert e.value.code == oracle.E_INVALID_GRAPH
