"""Pins of the oracle's sampling forms.

  - SplitMix64: the output function matches the published first output of
    SplitMix64 seeded with 0 (0xE220A8397B1DCDAF), and the input generator
    module's independent implementation draws the same numbers;
  - bounded(): range and endpoint properties of multiply-shift reduction;
  - path walk: uniform over the 20 shortest corner-to-corner paths of the
    4x4 grid (chi-square), every sampled path is a shortest path;
  - VD bound: at least the true vertex diameter (networkx), exact on stars;
  - sample size: hand-evaluated values of the Riondato-Kornaropoulos bound;
  - estimator: the epsilon guarantee holds on graphs with known exact BC;
  - source sampling: the n/k-scaled estimator is unbiased (mean over seeds).
"""
import math

import networkx as nx
import numpy as np
import pytest
from scipy.stats import chi2 as chi2_dist

import graphgen as gg
import oracle
from oracle import bruteforce as bf


def test_splitmix64_published_vector():
    assert oracle.mix64(0x9E3779B97F4A7C15) == 0xE220A8397B1DCDAF
    for args in [(0, 0, 0, 0), (1, 2, 3, 4), (2 ** 64 - 1, 3, 10 ** 12, 7)]:
        assert oracle.draw(*args) == gg.draw(*args)


def test_bounded_properties():
    for N in [1, 2, 3, 7, 1000, 2 ** 31 - 1, 2 ** 40 + 3]:
        assert oracle.bounded(0, N) == 0
        assert oracle.bounded(2 ** 64 - 1, N) == N - 1
        prev = 0
        for x in [1, 2 ** 20, 2 ** 40, 2 ** 63, 2 ** 63 + 5, 2 ** 64 - 2]:
            b = oracle.bounded(x, N)
            assert prev <= b < N
            prev = b
    assert oracle.bounded(2 ** 63, 10) == 5


def _is_shortest_path(g, u, v, interior):
    seq = [v] + interior + [u]
    adj = {x: set(g.colidx[g.rowptr[x]:g.rowptr[x + 1]].tolist()) for x in seq}
    for a, b in zip(seq, seq[1:]):
        if b not in adj[a]:
            return False
    d, _ = oracle.sssp_counts(g.rowptr, g.colidx, u)
    return len(seq) - 1 == d[v]


def test_path_walk_uniform_on_grid():
    g = gg.grid(4, 4)
    counts = {}
    N = 6000
    for j in range(N):
        p = tuple(oracle.sample_path_uv(g.rowptr, g.colidx, 99, j, 0, 15))
        counts[p] = counts.get(p, 0) + 1
    assert len(counts) == math.comb(6, 3) == 20
    exp = N / 20
    chi2 = sum((c - exp) ** 2 / exp for c in counts.values())
    assert chi2 < chi2_dist.ppf(0.999, 19)  # 43.82
    for p in list(counts)[:5]:
        assert _is_shortest_path(g, 0, 15, list(p))


@pytest.mark.parametrize("make,u,v", [
    (lambda: gg.grid(3, 5), 0, 14),                       # 15 paths, meeting weights differ
    (lambda: gg.grid(4, 4), 5, 15),
    (lambda: gg.barabasi_albert(12, 2, 8), None, None),   # pair with the most shortest paths
    (lambda: gg.complete_bipartite(3, 4), 0, 1),          # u and v on the same side
])
def test_bidirectional_sampler_uniform_vs_enumeration(make, u, v):
    """Frequencies of the sampled paths of one pair against every shortest
    path enumerated by brute force: chi-square at the 99.9% level."""
    g = make()
    paths = bf.all_pairs_paths(g.rowptr, g.colidx)
    if u is None:
        (u, v), _ = max(paths.items(), key=lambda kv: (len(kv[1]), -kv[0][0], -kv[0][1]))
    want = {tuple(reversed(p[1:-1])) for p in paths[(u, v)]}   # interior from v's side
    assert len(want) >= 3
    N = 1000 * len(want)
    counts = {}
    for j in range(N):
        p = tuple(oracle.sample_path_uv(g.rowptr, g.colidx, 7, j, u, v))
        assert p in want
        counts[p] = counts.get(p, 0) + 1
    assert set(counts) == want
    exp = N / len(want)
    chi2 = sum((c - exp) ** 2 / exp for c in counts.values())
    assert chi2 < chi2_dist.ppf(0.999, len(want) - 1)


def test_bidirectional_sampler_all_pairs_small():
    """Every ordered pair of small random graphs: the sampled interior is a
    shortest path of the brute-force enumeration; unreachable pairs give None."""
    for seed in range(6):
        g = gg.erdos_renyi(9, 9 + seed, 40 + seed)
        paths = bf.all_pairs_paths(g.rowptr, g.colidx)
        for u in range(g.n):
            for v in range(g.n):
                if u == v:
                    continue
                got = oracle.sample_path_uv(g.rowptr, g.colidx, seed, u * g.n + v, u, v)
                if (u, v) not in paths:
                    assert got is None
                else:
                    assert tuple(got) in {tuple(reversed(p[1:-1])) for p in paths[(u, v)]}


def test_sampled_paths_are_shortest():
    g = gg.erdos_renyi(300, 700, 5)
    seen_unreachable = 0
    for j in range(60):
        u, v, interior = oracle.sample_path(g.rowptr, g.colidx, 17, j)
        assert u != v and 0 <= u < g.n and 0 <= v < g.n
        if interior is None:
            seen_unreachable += 1
            continue
        assert _is_shortest_path(g, u, v, interior)


def _true_vd(g):
    G = nx.Graph()
    G.add_nodes_from(range(g.n))
    u, v = g.edges()
    G.add_edges_from(zip(u.tolist(), v.tolist()))
    best = 1
    for comp in nx.connected_components(G):
        if len(comp) > 1:
            best = max(best, nx.diameter(G.subgraph(comp)) + 1)
    return best


@pytest.mark.parametrize("make", [
    lambda: gg.star(10), lambda: gg.path(9), lambda: gg.cycle(12), lambda: gg.grid(5, 6),
    lambda: gg.erdos_renyi(200, 300, 3), lambda: gg.barabasi_albert(300, 2, 4),
    lambda: gg.disjoint_union([gg.star(30), gg.path(12)]),
])
def test_vd_bound_is_upper_bound(make):
    g = make()
    info = oracle.vd_bound(g.rowptr, g.colidx)
    vd = _true_vd(g)
    assert info["vd_ub"] >= vd
    assert info["vd_lb"] <= vd or info["c2"] > 0
    if g.name.startswith("star"):
        assert info["vd_ub"] == 3 and info["x0"] == 0 and info["e1"] == 1
    if g.name.startswith("path"):
        assert info["vd_ub"] == g.n  # capped by the component size


def test_sample_size_values():
    # c = 0.5, eps = 0.01, delta = 0.1: 5000 * (floor(log2(VD-2)) + 1 + ln 10)
    # VD-2 in [4, 7] -> 5000 * (3 + 2.302585...) = 26512.9 -> 26513
    assert oracle.rk_sample_size(0.01, 0.1, 6) == 26513
    assert oracle.rk_sample_size(0.01, 0.1, 9) == 26513
    # VD-2 in [8, 15] -> 5000 * 5.302585 + 5000 = 31512.9 -> 31513
    assert oracle.rk_sample_size(0.01, 0.1, 10) == 31513
    assert oracle.rk_sample_size(0.01, 0.1, 17) == 31513
    # VD <= 3: log term 0 -> 5000 * 3.302585 = 16512.9 -> 16513
    assert oracle.rk_sample_size(0.01, 0.1, 2) == 16513
    assert oracle.rk_sample_size(0.01, 0.1, 3) == 16513
    # eps = 0.05, delta = 0.1, VD-2 in [4,7]: 200 * 5.302585 = 1060.5 -> 1061
    assert oracle.rk_sample_size(0.05, 0.1, 8) == 1061


def test_epsilon_guarantee():
    g = gg.barabasi_albert(120, 2, 8)
    n = g.n
    exact = oracle.bc_exact(g.rowptr, g.colidx) / (n * (n - 1))
    eps, delta = 0.05, 0.1
    fails = 0
    trials = 20
    for seed in range(trials):
        est, cnt, r, vd = oracle.pair_sample(g.rowptr, g.colidx, eps, delta, seed)
        assert r == oracle.rk_sample_size(eps, delta, vd)
        assert np.allclose(est, cnt / r * n * (n - 1))
        if np.max(np.abs(est / (n * (n - 1)) - exact)) > eps:
            fails += 1
    assert fails <= delta * trials


def test_pair_estimate_converges():
    g = gg.grid(4, 5)
    n = g.n
    exact = oracle.bc_exact(g.rowptr, g.colidx)
    cnt = oracle.pair_counts(g.rowptr, g.colidx, 40000, 3)
    est = cnt / 40000 * n * (n - 1)
    assert np.max(np.abs(est - exact)) / (n * (n - 1)) < 0.01


def test_source_sampling_unbiased():
    g = gg.barabasi_albert(80, 2, 9)
    exact = oracle.bc_exact(g.rowptr, g.colidx)
    k, trials = 8, 400
    acc = np.zeros(g.n)
    for seed in range(trials):
        src = gg.sample_sources(g.n, k, 1000 + seed)
        acc += oracle.bc_sources(g.rowptr, g.colidx, src, scale=g.n / k)
    mean = acc / trials
    top = np.argsort(-exact)[:5]
    assert np.allclose(mean[top], exact[top], rtol=0.15)


def test_pairs_uniform_and_distinct():
    g = gg.cycle(4)
    N = 6000
    counts = {}
    for j in range(N):
        u, v, interior = oracle.sample_path(g.rowptr, g.colidx, 5, j)
        assert u != v
        counts[(u, v)] = counts.get((u, v), 0) + 1
        # antipodal pairs of C4 have two paths with one interior vertex each
        if (u - v) % 4 == 2:
            assert len(interior) == 1 and interior[0] in ((u + 1) % 4, (u + 3) % 4)
        else:
            assert interior == []
    assert len(counts) == 12
    exp = N / 12
    chi2 = sum((c - exp) ** 2 / exp for c in counts.values())
    assert chi2 < chi2_dist.ppf(0.999, 11)  # 31.26


def test_pair_counts_threads_agree():
    """The timing mode's contiguous blocks of samples add up to the
    sequential counts exactly."""
    g = gg.barabasi_albert(400, 3, 21)
    one = oracle.pair_counts(g.rowptr, g.colidx, 1500, 8)
    assert one.sum() > 0
    for t in (2, 3, 7):
        assert np.array_equal(oracle.pair_counts(g.rowptr, g.colidx, 1500, 8, nthreads=t), one)
