"""Rank agreement of the sampled estimators with exact betweenness (section
"Heuristics and Approximation Algorithms": sampling a small share of the
shortest-path trees still ranks the nodes much like exact betweenness; the
paper's example keeps 8 of the exact top ten, and relative rank errors,
exact rank over approximate rank, stay close to 1).  On power-law graphs
like the paper's router-level network (Barabasi-Albert and R-MAT here), for
the n/k source-sampled estimate with k = 300 sources and for pair sampling
at eps = 0.01: at least 8 of the exact top ten, Spearman's rank correlation
over vertices with nonzero exact score at least 0.9 (0.8 for pairs), and the
median relative rank error of the exact top hundred within [0.75, 1.33]."""
import numpy as np
import pytest
from scipy.stats import spearmanr

import graphgen as gg
import oracle


def _ranks(x):
    order = np.argsort(-x, kind="stable")
    r = np.empty(len(x))
    r[order] = np.arange(1, len(x) + 1)
    return order, r


def rank_agreement(exact, approx):
    """(top-10 overlap, Spearman rho over nonzero exact, median relative rank
    error exact/approx of the exact top 100)."""
    o_ex, r_ex = _ranks(exact)
    o_ap, r_ap = _ranks(approx)
    top10 = len(set(o_ex[:10].tolist()) & set(o_ap[:10].tolist()))
    nz = exact > 0
    rho = spearmanr(exact[nz], approx[nz]).correlation
    top = o_ex[:100]
    return top10, rho, float(np.median(r_ex[top] / r_ap[top]))


GRAPHS = [lambda: gg.barabasi_albert(3000, 3, 5), lambda: gg.rmat(12, 8, 6)]


@pytest.mark.parametrize("make", GRAPHS)
@pytest.mark.parametrize("seed", [0, 1, 2])
def test_source_sampling_ranks_like_exact(make, seed):
    g = make()
    exact = oracle.bc_exact(g.rowptr, g.colidx, nthreads=8)
    src = gg.sample_sources(g.n, 300, 100 + seed)
    approx = oracle.bc_sources(g.rowptr, g.colidx, src, g.n / 300, nthreads=8)
    top10, rho, med = rank_agreement(exact, approx)
    assert top10 >= 8 and rho >= 0.9 and 0.75 <= med <= 1.33, (g.name, top10, rho, med)


@pytest.mark.parametrize("make", GRAPHS)
def test_pair_sampling_ranks_like_exact(make):
    g = make()
    exact = oracle.bc_exact(g.rowptr, g.colidx, nthreads=8)
    est, cnt, r, vd = oracle.pair_sample(g.rowptr, g.colidx, 0.01, 0.1, 3)
    top10, rho, med = rank_agreement(exact, est)
    assert top10 >= 8 and rho >= 0.8, (g.name, top10, rho, med)


def test_rank_agreement_detects_a_shuffle():
    """The measure itself: a random permutation of the exact scores fails
    it, the exact scores pass with full agreement."""
    g = gg.barabasi_albert(3000, 3, 5)
    exact = oracle.bc_exact(g.rowptr, g.colidx, nthreads=8)
    assert rank_agreement(exact, exact) == (10, pytest.approx(1.0), 1.0)
    top10, rho, _ = rank_agreement(exact, np.random.default_rng(1).permutation(exact))
    assert top10 < 8 and rho < 0.5
