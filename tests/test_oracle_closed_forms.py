"""Pins of the CPU oracle against closed forms (ordered-pair convention).

Each expected value below is derived on paper from the graph's structure,
not by running Brandes' algorithm:
  path P_n      BC(i) = 2 i (n-1-i)
  star S_n      centre (n-1)(n-2), leaves 0
  cycle C_n     (n-1)(n-3)/4 for odd n, (n-2)^2/4 for even n
  K_n           0
  K_{a,b}       side A: b(b-1)/a, side B: a(a-1)/b
  tree T        BC(v) = (n-1)^2 - sum over components C of T-v of |C|^2
  hypercube Q_d BC = d 2^(d-1) - 2^d + 1; sigma(s,t) = Hamming(s,t)!
  grid          sigma(corner, (i,j)) = binomial(i+j, i)
  diamonds      sigma(0, 3k) = 2^k
"""
import math

import numpy as np
import pytest

import graphgen as gg
import oracle


def bc(g):
    return oracle.bc_exact(g.rowptr, g.colidx)


@pytest.mark.parametrize("n", [1, 2, 3, 4, 7, 20])
def test_path(n):
    g = gg.path(n)
    exp = [2 * i * (n - 1 - i) for i in range(n)]
    assert np.array_equal(bc(g), np.array(exp, dtype=float))
    d, s = oracle.sssp_counts(g.rowptr, g.colidx, 0)
    assert list(d) == list(range(n))
    assert all(s == 1)


@pytest.mark.parametrize("n", [2, 3, 5, 11])
def test_star(n):
    g = gg.star(n)
    exp = np.zeros(n)
    exp[0] = (n - 1) * (n - 2)
    assert np.array_equal(bc(g), exp)


@pytest.mark.parametrize("n", [3, 4, 5, 6, 9, 10, 31, 32])
def test_cycle(n):
    g = gg.cycle(n)
    val = (n - 1) * (n - 3) / 4 if n % 2 else (n - 2) ** 2 / 4
    assert np.allclose(bc(g), val, rtol=1e-14, atol=0)
    d, s = oracle.sssp_counts(g.rowptr, g.colidx, 0)
    for t in range(n):
        assert d[t] == min(t, n - t)
        # exactly two shortest paths to the antipode of an even cycle
        assert s[t] == (2 if (n % 2 == 0 and t == n // 2) else 1)


@pytest.mark.parametrize("n", [1, 2, 5, 12])
def test_complete(n):
    g = gg.complete(n)
    assert np.array_equal(bc(g), np.zeros(n))


@pytest.mark.parametrize("a,b", [(1, 1), (1, 5), (2, 3), (4, 4), (3, 7)])
def test_complete_bipartite(a, b):
    g = gg.complete_bipartite(a, b)
    exp = np.array([b * (b - 1) / a] * a + [a * (a - 1) / b] * b)
    assert np.allclose(bc(g), exp, rtol=1e-14, atol=0)
    d, s = oracle.sssp_counts(g.rowptr, g.colidx, 0)
    if a > 1:
        assert d[1] == 2 and s[1] == b  # same side: one path through each vertex of B


def _tree_closed_form(g):
    n = g.n
    adj = [g.colidx[g.rowptr[v]:g.rowptr[v + 1]].tolist() for v in range(n)]
    parent = [-1] * n
    order = [0]
    seen = [False] * n
    seen[0] = True
    for v in order:
        for w in adj[v]:
            if not seen[w]:
                seen[w] = True
                parent[w] = v
                order.append(w)
    size = [1] * n
    for v in reversed(order):
        if parent[v] >= 0:
            size[parent[v]] += size[v]
    out = []
    for v in range(n):
        comps = [size[w] for w in adj[v] if parent[w] == v]
        if parent[v] >= 0:
            comps.append(n - size[v])
        out.append((n - 1) ** 2 - sum(c * c for c in comps))
    return np.array(out, dtype=float)


@pytest.mark.parametrize("n,seed", [(2, 1), (10, 2), (200, 3), (3000, 4)])
def test_random_tree(n, seed):
    g = gg.random_tree(n, seed)
    assert np.allclose(bc(g), _tree_closed_form(g), rtol=1e-12, atol=0)


@pytest.mark.parametrize("d", [1, 2, 3, 5, 7])
def test_hypercube(d):
    g = gg.hypercube(d)
    exp = d * 2 ** (d - 1) - 2 ** d + 1
    assert np.allclose(bc(g), exp, rtol=1e-13, atol=1e-12)
    dist, s = oracle.sssp_counts(g.rowptr, g.colidx, 0)
    for t in range(g.n):
        h = bin(t).count("1")
        assert dist[t] == h
        assert int(s[t]) == math.factorial(h)


def test_hypercube_sigma_limits():
    # Q20: the largest path count is 20! < 2^64; Q21 would need 21! > 2^64
    assert math.factorial(20) < 2 ** 64 < math.factorial(21)
    g = gg.hypercube(20)
    d, s = oracle.sssp_counts(g.rowptr, g.colidx, 0)
    assert int(s[g.n - 1]) == math.factorial(20)


@pytest.mark.parametrize("r,c", [(1, 5), (3, 4), (6, 6)])
def test_grid_sigma(r, c):
    g = gg.grid(r, c)
    d, s = oracle.sssp_counts(g.rowptr, g.colidx, 0)
    for i in range(r):
        for j in range(c):
            assert d[i * c + j] == i + j
            assert int(s[i * c + j]) == math.comb(i + j, i)


def test_grid_overflow_boundary():
    ok = gg.grid(34, 34)
    d, s = oracle.sssp_counts(ok.rowptr, ok.colidx, 0)
    assert int(s[-1]) == math.comb(66, 33) < 2 ** 64
    bad = gg.grid(35, 35)
    assert math.comb(68, 34) >= 2 ** 64
    with pytest.raises(oracle.OracleError) as e:
        oracle.sssp_counts(bad.rowptr, bad.colidx, 0)
    assert e.value.code == oracle.E_SIGMA_OVERFLOW
    with pytest.raises(oracle.OracleError) as e:
        oracle.bc_sources(bad.rowptr, bad.colidx, [0])
    assert e.value.code == oracle.E_SIGMA_OVERFLOW


def test_diamond_chain_overflow_boundary():
    g = gg.diamond_chain(63)
    d, s = oracle.sssp_counts(g.rowptr, g.colidx, 0)
    assert int(s[3 * 63]) == 2 ** 63
    assert d[3 * 63] == 2 * 63
    oracle.bc_sources(g.rowptr, g.colidx, [0, 3 * 63])
    g = gg.diamond_chain(64)
    with pytest.raises(oracle.OracleError) as e:
        oracle.sssp_counts(g.rowptr, g.colidx, 0)
    assert e.value.code == oracle.E_SIGMA_OVERFLOW
    # from the middle joint every count stays below 2^33
    oracle.sssp_counts(g.rowptr, g.colidx, 3 * 32)


def test_diamond_chain_small_bc():
    # k = 1 is the 4-cycle: every vertex lies on one of the two paths between
    # its two neighbours, in both directions: BC = 2 * 1/2 = 1
    g = gg.diamond_chain(1)
    assert np.allclose(bc(g), 1.0)
