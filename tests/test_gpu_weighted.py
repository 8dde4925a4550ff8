"""GPU parity of weighted betweenness (positive integer arc weights) against
the oracle's Dijkstra-based Brandes, through the C ABI."""
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


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.int32)).to("cuda:0")


CASES = [
    (lambda: gg.erdos_renyi(2000, 6000, 41), 3, True), (lambda: gg.erdos_renyi(2000, 6000, 41), 100, True),
    (lambda: gg.barabasi_albert(3000, 3, 42), 5, True), (lambda: gg.grid(20, 27), 2, True),
    (lambda: gg.path(300), 7, True), (lambda: gg.rmat(12, 8, 43), 16, True),
    (lambda: gg.directed_rmat(12, 8, 44), 9, False),
    # weights up to 10^6: distances span more values than the bucket ordering takes (Kahn layers)
    (lambda: gg.erdos_renyi(2000, 6000, 48), 1000000, True), (lambda: gg.rmat(11, 8, 49), 50000, False),
    (lambda: gg.disjoint_union([gg.grid(6, 7), gg.star(50), gg.path(1), gg.cycle(9), gg.complete(5)]), 4, True),
]


@pytest.mark.parametrize("make,wmax,sym", CASES)
def test_weighted_exact_and_sampled(make, wmax, sym):
    g = make()
    w = gg.edge_weights(g, wmax, 45, symmetric=sym)
    rp, ci = upload(g)
    wt = _dev(w)
    got = nk.nk_bc_weighted(rp, ci, wt).cpu().numpy()
    assert_scores_close(got, oracle.bc_weighted(g.rowptr, g.colidx, w, nthreads=8), g.name + " all")
    k = min(g.n, 97)
    src = gg.sample_sources(g.n, k, 46)
    got = nk.nk_bc_weighted(rp, ci, wt, ivec(src), g.n / k).cpu().numpy()
    assert_scores_close(got, oracle.bc_weighted(g.rowptr, g.colidx, w, src, g.n / k), g.name + " sampled")


@pytest.mark.parametrize("sym", [True, False])
def test_weighted_with_and_without_relabelling(sym):
    """Degree relabelling (the default above 256 vertices) carries each
    arc's weight to the renamed arc; flag 2 runs under the caller's ids,
    flag 1 keeps the settled-vertex bitmap in global memory."""
    g = gg.rmat(12, 8, 50) if sym else gg.directed_rmat(12, 8, 51)
    w = gg.edge_weights(g, 12, 52, symmetric=sym)
    rp, ci = upload(g)
    ref = oracle.bc_weighted(g.rowptr, g.colidx, w, nthreads=8)
    for flags in (0, 1, 2, 3):
        nk.nk_set_tuning(flags=flags)
        assert_scores_close(nk.nk_bc_weighted(rp, ci, _dev(w)).cpu().numpy(), ref, f"flags={flags}")
        assert nk.nk_last_stats()["bitmap_lds"] == (0 if flags & 1 else 1)


def test_unit_weights_equal_unweighted_on_gpu():
    g = gg.barabasi_albert(4000, 3, 47)
    rp, ci = upload(g)
    got = nk.nk_bc_weighted(rp, ci, _dev(np.ones(g.m))).cpu().numpy()
    assert_scores_close(got, nk.nk_bc_exact(rp, ci).cpu().numpy(), "unit weights")


@pytest.mark.parametrize("block", [256, 512, 1024])
def test_weighted_block_sizes(block):
    nk.nk_set_tuning(block=block)
    g = gg.rmat(11, 8, 48)
    w = gg.edge_weights(g, 12, 49)
    rp, ci = upload(g)
    src = gg.sample_sources(g.n, 64, 50)
    got = nk.nk_bc_weighted(rp, ci, _dev(w), ivec(src), 1.0).cpu().numpy()
    assert nk.nk_last_stats()["block"] == block
    assert_scores_close(got, oracle.bc_weighted(g.rowptr, g.colidx, w, src), "block variant")


def test_weighted_rmat14_sampled():
    g = gg.rmat(14, 16, 51)
    w = gg.edge_weights(g, 64, 52)
    rp, ci = upload(g)
    src = gg.sample_sources(g.n, 256, 53)
    got = nk.nk_bc_weighted(rp, ci, _dev(w), ivec(src), g.n / 256).cpu().numpy()
    assert_scores_close(got, oracle.bc_weighted(g.rowptr, g.colidx, w, src, g.n / 256, nthreads=8), "rmat14")


def test_weighted_errors():
    g = gg.erdos_renyi(300, 900, 54)
    w = gg.edge_weights(g, 5, 55)
    rp, ci = upload(g)
    bad = w.copy()
    bad[7] = 0
    with pytest.raises(nk.NkError) as e:
        nk.nk_bc_weighted(rp, ci, _dev(bad))
    assert e.value.code == nk.NK_E_INVALID_GRAPH
    with pytest.raises(nk.NkError) as e:
        nk.nk_bc_weighted(rp, ci, _dev(w), ivec([0, 300]))
    assert e.value.code == nk.NK_E_INVALID_ARG
    out = nk.nk_bc_weighted(rp, ci, _dev(w), torch.zeros(0, dtype=torch.int32, device="cuda:0"))
    assert not out.any()
    got = nk.nk_bc_weighted(rp, ci, _dev(w)).cpu().numpy()
    assert_scores_close(got, oracle.bc_weighted(g.rowptr, g.colidx, w), "after errors")
