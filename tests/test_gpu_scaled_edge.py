"""GPU parity of the linear-scaling and bisection estimators and of edge
betweenness against the oracle, through the C ABI."""
import numpy as np
import pytest
import torch

import graphgen as gg
import oracle
import paper_1403_3005_amd as nk
from nkutil import assert_scores_close, ivec, upload

pytestmark = pytest.mark.gpu


@pytest.fixture(autouse=True)
def _default_tuning():
    nk.nk_set_tuning()
    yield
    nk.nk_set_tuning()


GRAPHS = [
    lambda: gg.path(300), lambda: gg.star(2500), lambda: gg.cycle(257), lambda: gg.grid(20, 27),
    lambda: gg.complete_bipartite(5, 200), lambda: gg.random_tree(3000, 9), lambda: gg.erdos_renyi(2500, 6000, 81),
    lambda: gg.barabasi_albert(4000, 4, 82), lambda: gg.rmat(12, 16, 83),
    lambda: gg.disjoint_union([gg.grid(6, 7), gg.star(50), gg.path(1), gg.cycle(9), gg.complete(5)]),
]


@pytest.mark.parametrize("flags", [0, 4])
@pytest.mark.parametrize("make", GRAPHS)
def test_linear_exact_sources(make, flags):
    """All sources and a sampled set, on the all-in-LDS kernel where the
    graph fits (flags 0) and on the global kernel (flags 4)."""
    nk.nk_set_tuning(flags=flags)
    g = make()
    rp, ci = upload(g)
    got = nk.nk_bc_sources_linear(rp, ci, None, 2.0).cpu().numpy()
    ref = oracle.bc_sources_linear(g.rowptr, g.colidx, np.arange(g.n), 2.0, nthreads=8)
    assert_scores_close(got, ref, g.name + " all")
    k = min(g.n, 97)
    src = gg.sample_sources(g.n, k, 84)
    got = nk.nk_bc_sources_linear(rp, ci, ivec(src), 2.0 * g.n / k).cpu().numpy()
    assert_scores_close(got, oracle.bc_sources_linear(g.rowptr, g.colidx, src, 2.0 * g.n / k), g.name + " sampled")


def test_linear_all_sources_is_half_of_exact_on_gpu():
    g = gg.barabasi_albert(3000, 3, 85)
    rp, ci = upload(g)
    lin = nk.nk_bc_sources_linear(rp, ci, None, 2.0).cpu().numpy()
    assert_scores_close(lin, nk.nk_bc_exact(rp, ci).cpu().numpy(), "2 x linear vs exact")


@pytest.mark.parametrize("block", [256, 1024])
@pytest.mark.parametrize("bu_ratio", [0.0, 1e9])
@pytest.mark.parametrize("bw_ratio", [0.0, 1e9])
def test_linear_launch_variants(block, bu_ratio, bw_ratio):
    """The level weight is applied in both the pull and the push sweep."""
    nk.nk_set_tuning(block=block, bu_ratio=bu_ratio, bw_ratio=bw_ratio, flags=4)
    g = gg.rmat(11, 8, 86)
    src = gg.sample_sources(g.n, 64, 87)
    rp, ci = upload(g)
    got = nk.nk_bc_sources_linear(rp, ci, ivec(src), g.n / 32).cpu().numpy()
    st = nk.nk_last_stats()
    if bw_ratio > 1:
        assert st["levels_bw_push"] > 0
    assert_scores_close(got, oracle.bc_sources_linear(g.rowptr, g.colidx, src, g.n / 32), "linear variant")


def test_linear_rmat14_sampled_relabelled():
    g = gg.rmat(14, 16, 88)
    src = gg.sample_sources(g.n, 256, 89)
    rp, ci = upload(g)
    got = nk.nk_bc_sources_linear(rp, ci, ivec(src), 2.0 * g.n / 256).cpu().numpy()
    assert_scores_close(got, oracle.bc_sources_linear(g.rowptr, g.colidx, src, 2.0 * g.n / 256, nthreads=8),
                        "rmat14 linear")


@pytest.mark.parametrize("make", GRAPHS)
def test_bisect_exact_sources(make):
    """All sources and a sampled set (the bisection sweeps run on the
    global kernel only)."""
    g = make()
    rp, ci = upload(g)
    got = nk.nk_bc_sources_bisect(rp, ci, None, 2.0).cpu().numpy()
    ref = oracle.bc_sources_bisect(g.rowptr, g.colidx, np.arange(g.n), 2.0, nthreads=8)
    assert_scores_close(got, ref, g.name + " all")
    k = min(g.n, 97)
    src = gg.sample_sources(g.n, k, 84)
    got = nk.nk_bc_sources_bisect(rp, ci, ivec(src), 2.0 * g.n / k).cpu().numpy()
    assert_scores_close(got, oracle.bc_sources_bisect(g.rowptr, g.colidx, src, 2.0 * g.n / k), g.name + " sampled")


@pytest.mark.parametrize("bw_ratio", [0.0, 0.1, 1e9])
def test_bisect_sweep_directions(bw_ratio):
    """The truncated sweeps by pull only (ratio 0), by the default choice,
    and by push wherever a level has arcs (ratio 1e9)."""
    nk.nk_set_tuning(bw_ratio=bw_ratio)
    try:
        for g in (gg.rmat(11, 8, 90), gg.barabasi_albert(2500, 2, 91),
                  gg.disjoint_union([gg.grid(9, 13), gg.random_tree(700, 92), gg.path(40)])):
            src = gg.sample_sources(g.n, 80, 93)
            rp, ci = upload(g)
            got = nk.nk_bc_sources_bisect(rp, ci, ivec(src), 2.0 * g.n / 80).cpu().numpy()
            st = nk.nk_last_stats()
            if bw_ratio > 1:
                assert st["levels_bw_push"] > 0
            if bw_ratio == 0.0:
                assert st["levels_bw_push"] == 0
            ref = oracle.bc_sources_bisect(g.rowptr, g.colidx, src, 2.0 * g.n / 80, nthreads=8)
            assert_scores_close(got, ref, f"{g.name} bw_ratio={bw_ratio}")
    finally:
        nk.nk_set_tuning()


@pytest.mark.parametrize("block", [256, 512, 1024])
def test_bisect_block_sizes_deep_graph(block):
    """Cutoff groups of every block size (tiles of block/4 vertices) on a
    graph deep enough for several groups."""
    nk.nk_set_tuning(block=block)
    try:
        g = gg.disjoint_union([gg.barabasi_albert(1500, 2, 94), gg.path(60), gg.grid(5, 40)])
        src = gg.sample_sources(g.n, 120, 95)
        rp, ci = upload(g)
        got = nk.nk_bc_sources_bisect(rp, ci, ivec(src), 2.0 * g.n / 120).cpu().numpy()
        assert nk.nk_last_stats()["block"] == block
        ref = oracle.bc_sources_bisect(g.rowptr, g.colidx, src, 2.0 * g.n / 120, nthreads=8)
        assert_scores_close(got, ref, f"block {block}")
    finally:
        nk.nk_set_tuning()


def test_bisect_all_sources_is_half_of_exact_on_gpu():
    g = gg.barabasi_albert(3000, 3, 85)
    rp, ci = upload(g)
    bis = nk.nk_bc_sources_bisect(rp, ci, None, 2.0).cpu().numpy()
    assert_scores_close(bis, nk.nk_bc_exact(rp, ci).cpu().numpy(), "2 x bisection vs exact")


@pytest.mark.parametrize("block", [256, 1024])
@pytest.mark.parametrize("bu_ratio", [0.0, 1e9])
@pytest.mark.parametrize("bw_ratio", [0.0, 1e9])
def test_bisect_launch_variants(block, bu_ratio, bw_ratio):
    """Output weights in both the pull and the push sweep, truncated sweeps
    after top-down and bottom-up forward levels."""
    nk.nk_set_tuning(block=block, bu_ratio=bu_ratio, bw_ratio=bw_ratio)
    g = gg.rmat(11, 8, 86)
    src = gg.sample_sources(g.n, 64, 87)
    rp, ci = upload(g)
    got = nk.nk_bc_sources_bisect(rp, ci, ivec(src), g.n / 32).cpu().numpy()
    st = nk.nk_last_stats()
    if bw_ratio > 1:
        assert st["levels_bw_push"] > 0
    assert_scores_close(got, oracle.bc_sources_bisect(g.rowptr, g.colidx, src, g.n / 32), "bisect variant")


def test_bisect_rmat14_sampled_relabelled():
    g = gg.rmat(14, 16, 88)
    src = gg.sample_sources(g.n, 256, 89)
    rp, ci = upload(g)
    got = nk.nk_bc_sources_bisect(rp, ci, ivec(src), 2.0 * g.n / 256).cpu().numpy()
    assert_scores_close(got, oracle.bc_sources_bisect(g.rowptr, g.colidx, src, 2.0 * g.n / 256, nthreads=8),
                        "rmat14 bisect")


def test_bisect_edge_cases_and_errors():
    g = gg.cycle(12)
    rp, ci = upload(g)
    out = nk.nk_bc_sources_bisect(rp, ci, torch.zeros(0, dtype=torch.int32, device="cuda:0"), 1.0)
    assert not out.any()
    with pytest.raises(nk.NkError) as e:
        nk.nk_bc_sources_bisect(rp, ci, ivec([0, 12]), 1.0)
    assert e.value.code == nk.NK_E_INVALID_ARG
    got = nk.nk_bc_sources_bisect(rp, ci, ivec([3]), 1.0).cpu().numpy()
    assert_scores_close(got, oracle.bc_sources_bisect(g.rowptr, g.colidx, [3]), "cycle after errors")


@pytest.mark.parametrize("make", GRAPHS)
def test_edge_exact(make):
    g = make()
    rp, ci = upload(g)
    ebc, bc = nk.nk_edge_bc(rp, ci)
    oe, ob = oracle.edge_bc(g.rowptr, g.colidx, nthreads=8)
    assert_scores_close(ebc.cpu().numpy(), oe, g.name + " edges")
    assert_scores_close(bc.cpu().numpy(), ob, g.name + " vertices")


@pytest.mark.parametrize("bw_ratio", [0.0, 0.1, 1e9])
@pytest.mark.parametrize("bu_ratio", [0.0, 16.0, 1e9])
def test_edge_sampled_sources(bu_ratio, bw_ratio):
    """Edge scores with the sweep by pull only, by the default choice, and
    by push wherever a level has arcs (a pushed term lands on the reverse
    arc; both arcs are summed at the end)."""
    nk.nk_set_tuning(bu_ratio=bu_ratio, bw_ratio=bw_ratio)
    g = gg.rmat(13, 16, 90)
    src = gg.sample_sources(g.n, 200, 91)
    rp, ci = upload(g)
    ebc, bc = nk.nk_edge_bc(rp, ci, ivec(src), g.n / 200)
    pushed = nk.nk_last_stats()["levels_bw_push"]
    if bw_ratio == 0.0:
        assert pushed == 0
    if bw_ratio > 1e6:
        assert pushed > 0
    oe, ob = oracle.edge_bc(g.rowptr, g.colidx, src, g.n / 200, nthreads=8)
    assert_scores_close(ebc.cpu().numpy(), oe, "rmat13 edges")
    assert_scores_close(bc.cpu().numpy(), ob, "rmat13 vertices")


def test_edge_edge_cases_and_errors():
    # no arcs
    g = gg.Graph(20, np.zeros(21, dtype=np.int32), np.zeros(0, dtype=np.int32))
    rp, ci = upload(g)
    ebc, bc = nk.nk_edge_bc(rp, ci)
    assert ebc.numel() == 0 and not bc.any()
    # no sources
    g = gg.cycle(12)
    rp, ci = upload(g)
    ebc, bc = nk.nk_edge_bc(rp, ci, torch.zeros(0, dtype=torch.int32, device="cuda:0"))
    assert not ebc.any() and not bc.any()
    # a missing reverse arc
    rowptr = torch.tensor([0, 1, 1], dtype=torch.int32, device="cuda:0")
    colidx = torch.tensor([1], dtype=torch.int32, device="cuda:0")
    with pytest.raises(nk.NkError) as e:
        nk.nk_edge_bc(rowptr, colidx)
    assert e.value.code == nk.NK_E_INVALID_GRAPH
    # sources out of range
    with pytest.raises(nk.NkError) as e:
        nk.nk_edge_bc(rp, ci, ivec([0, 12]))
    assert e.value.code == nk.NK_E_INVALID_ARG
    # the library still works
    ebc, _ = nk.nk_edge_bc(rp, ci)
    assert_scores_close(ebc.cpu().numpy(), oracle.edge_bc(g.rowptr, g.colidx)[0], "cycle after errors")
