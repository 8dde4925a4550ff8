"""Input generators: determinism, simplicity and the size statistics the
workloads are specified with."""
import numpy as np
import pytest

import graphgen as gg
import oracle


def _simple(g):
    return oracle.validate(g.rowptr, g.colidx, strict=True) == 0


def test_deterministic_and_seed_sensitive():
    a = gg.erdos_renyi(500, 2000, 7)
    b = gg.erdos_renyi(500, 2000, 7)
    c = gg.erdos_renyi(500, 2000, 8)
    assert a.sha256() == b.sha256() != c.sha256()
    assert gg.rmat(10, 8, 3).sha256() == gg.rmat(10, 8, 3).sha256()
    assert np.array_equal(gg.sample_sources(1000, 50, 2), gg.sample_sources(1000, 50, 2))


@pytest.mark.parametrize("make", [
    lambda: gg.erdos_renyi(2000, 10000, 1), lambda: gg.rmat(12, 16, 2), lambda: gg.chung_lu(5000, 2.5, 20, 3),
    lambda: gg.barabasi_albert(3000, 4, 4), lambda: gg.grid(7, 9), lambda: gg.hypercube(6),
    lambda: gg.diamond_chain(10), lambda: gg.random_tree(500, 5), lambda: gg.complete_bipartite(3, 6),
])
def test_simple_symmetric_sorted(make):
    assert _simple(make())


def test_er_edge_count():
    g = gg.workload_er2000()
    assert g.n == 2000 and g.m == 20000


def test_ba_edge_count():
    g = gg.barabasi_albert(1000, 4, 1)
    assert g.m_undirected == 10 + (1000 - 5) * 4
    assert g.degrees().min() >= 4


def test_sources_distinct_uniform():
    s = gg.sample_sources(100, 100, 4)
    assert sorted(s.tolist()) == list(range(100))
    hits = np.zeros(50)
    for seed in range(2000):
        hits[gg.sample_sources(50, 5, seed)] += 1
    exp = 2000 * 5 / 50
    assert ((hits - exp) ** 2 / exp).sum() < 85.4  # chi-square, 49 dof, 99.9%


def test_rmat_statistics():
    g = gg.rmat(16, 16, 2)
    deg = g.degrees()
    # many isolated vertices (about 29% at scale 16, 38% at scale 20) and the
    # heaviest hub at vertex 0 for these parameters
    assert 0.25 < (deg == 0).mean() < 0.45
    assert deg.argmax() == 0
    assert 0.8 < g.m_undirected / (16 * 2 ** 16) < 0.97


def test_chung_lu_mean_degree():
    g = gg.chung_lu(200000, 2.5, 20.0, 3)
    mean = g.m / g.n
    assert 17.5 < mean < 21.0
    assert g.degrees()[0] == g.degrees().max()


def test_batched_sizes_log_uniform():
    sizes = gg.batched_sizes(512, 1000, 200000, 4)
    assert min(sizes) >= 1000 and max(sizes) <= 200000
    logs = np.log(sizes)
    assert abs(np.median(logs) - 0.5 * (np.log(1000) + np.log(200000))) < 0.5


def test_directed_generators():
    """Directed graphs: rows sorted, no self-loops or duplicate arcs, not
    symmetrised; the transpose holds every arc reversed; deterministic."""
    g = gg.directed_rmat(10, 8, 3)
    assert g.sha256() == gg.directed_rmat(10, 8, 3).sha256() != gg.directed_rmat(10, 8, 4).sha256()
    src = np.repeat(np.arange(g.n), g.degrees())
    assert np.all(src != g.colidx)
    for v in range(g.n):
        row = g.colidx[g.rowptr[v]:g.rowptr[v + 1]]
        assert np.all(np.diff(row) > 0)
    arcs = set(zip(src.tolist(), g.colidx.tolist()))
    assert any((b, a) not in arcs for a, b in arcs)          # not symmetric
    t = gg.transpose(g)
    tsrc = np.repeat(np.arange(t.n), t.degrees())
    assert set(zip(t.colidx.tolist(), tsrc.tolist())) == arcs
    r = gg.directed_random(300, 2000, 9)
    assert r.m <= 2000 and r.sha256() == gg.directed_random(300, 2000, 9).sha256()


def test_edge_weights_symmetric_ranged_deterministic():
    g = gg.barabasi_albert(500, 3, 10)
    w = gg.edge_weights(g, 17, 11)
    assert w.dtype == np.int32 and w.min() >= 1 and w.max() <= 17
    assert np.array_equal(w, gg.edge_weights(g, 17, 11)) and not np.array_equal(w, gg.edge_weights(g, 17, 12))
    src = np.repeat(np.arange(g.n), g.degrees())
    wt = {(int(a), int(b)): int(x) for a, b, x in zip(src, g.colidx, w)}
    assert all(wt[(b, a)] == x for (a, b), x in wt.items())  # both arcs of an edge agree
    d = gg.directed_rmat(8, 4, 13)
    wd = gg.edge_weights(d, 5, 14, symmetric=False)
    assert wd.shape == (d.m,) and wd.min() >= 1 and wd.max() <= 5
    assert len(np.unique(gg.edge_weights(gg.erdos_renyi(2000, 8000, 15), 64, 16))) == 64
