"""GPU parity of directed betweenness (out-arc CSR, optional in-arc CSR for
bottom-up levels) and of the transpose helper, through the C ABI."""
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


GRAPHS = [
    lambda: gg.directed_random(2000, 9000, 21),
    lambda: gg.directed_rmat(12, 8, 22),
    lambda: gg.directed_from_arcs(300, np.arange(299), np.arange(1, 300), "dpath"),
    lambda: gg.directed_from_arcs(257, np.arange(257), (np.arange(257) + 1) % 257, "dcycle"),
    lambda: gg.directed_from_arcs(3001, np.concatenate([np.zeros(3000), np.arange(1, 3001)]),
                                  np.concatenate([np.arange(1, 3001), (np.arange(1, 3001) * 7) % 3001]), "hub-out"),
]


# flags: 2 keeps the caller's vertex ids (no degree relabelling), 4 turns
# off the all-in-LDS kernel
@pytest.mark.parametrize("flags", [0, 2, 4])
@pytest.mark.parametrize("with_t", [False, True])
@pytest.mark.parametrize("make", GRAPHS)
def test_directed_exact_and_sampled(make, with_t, flags):
    """Every source and a sampled set, with and without the in-arc CSR, on
    the all-in-LDS kernel where the graph fits (flags 0) and on the global
    kernel (flags 4)."""
    nk.nk_set_tuning(flags=flags)
    g = make()
    rp, ci = upload(g)
    trp = tci = None
    if with_t:
        t = gg.transpose(g)
        trp, tci = _dev(t.rowptr), _dev(t.colidx)
    got = nk.nk_bc_directed(rp, ci, None, 1.0, trp, tci).cpu().numpy()
    assert_scores_close(got, oracle.bc_directed(g.rowptr, g.colidx, nthreads=8), g.name + " all")
    k = min(g.n, 97)
    src = gg.sample_sources(g.n, k, 23)
    got = nk.nk_bc_directed(rp, ci, ivec(src), g.n / k, trp, tci).cpu().numpy()
    assert_scores_close(got, oracle.bc_directed(g.rowptr, g.colidx, src, g.n / k), g.name + " sampled")


@pytest.mark.parametrize("bu_ratio", [0.0, 16.0, 1e9])
@pytest.mark.parametrize("block", [256, 1024])
def test_directed_bottom_up_variants(bu_ratio, block):
    """Bottom-up levels over in-arcs (bu_ratio 1e9: every level after the
    first), mixed, and none."""
    nk.nk_set_tuning(block=block, bu_ratio=bu_ratio, flags=4)
    g = gg.directed_rmat(13, 8, 24)
    t = gg.transpose(g)
    rp, ci = upload(g)
    src = gg.sample_sources(g.n, 200, 25)
    got = nk.nk_bc_directed(rp, ci, ivec(src), 1.0, _dev(t.rowptr), _dev(t.colidx)).cpu().numpy()
    st = nk.nk_last_stats()
    if bu_ratio > 1e6:
        assert st["levels_bu"] > 0
    if bu_ratio == 0.0:
        assert st["levels_bu"] == 0
    assert_scores_close(got, oracle.bc_directed(g.rowptr, g.colidx, src), "drmat13 variant")


@pytest.mark.parametrize("bw_ratio", [0.0, 0.1, 1e9])
@pytest.mark.parametrize("flags", [0, 2])
def test_directed_sweep_push_over_in_arcs(bw_ratio, flags):
    """The dependency sweep by pull only, by the default choice, and by push
    over in-arcs wherever a level has arcs, on a graph with many vertices of
    in-degree 0 that have out-arcs (marked unreachable, never pushed to),
    relabelled and not."""
    nk.nk_set_tuning(bw_ratio=bw_ratio, flags=flags | 4)
    g = gg.directed_rmat(12, 6, 27)
    rng = np.random.default_rng(28)
    # 300 extra vertices with out-arcs only
    extra_u = np.repeat(np.arange(g.n, g.n + 300), 3)
    extra_v = rng.integers(0, g.n, extra_u.size)
    src_u, src_v = [], []
    for u in range(g.n):
        for e in range(g.rowptr[u], g.rowptr[u + 1]):
            src_u.append(u)
            src_v.append(int(g.colidx[e]))
    h = gg.directed_from_arcs(g.n + 300, np.concatenate([src_u, extra_u]), np.concatenate([src_v, extra_v]), "drmat12+sources")
    t = gg.transpose(h)
    rp, ci = upload(h)
    src = np.concatenate([gg.sample_sources(g.n, 150, 29), np.arange(g.n, g.n + 20)]).astype(np.int32)
    got = nk.nk_bc_directed(rp, ci, ivec(src), 1.0, _dev(t.rowptr), _dev(t.colidx)).cpu().numpy()
    st = nk.nk_last_stats()
    if bw_ratio > 1e6:
        assert st["levels_bw_push"] > 0
    if bw_ratio == 0.0:
        assert st["levels_bw_push"] == 0
    assert_scores_close(got, oracle.bc_directed(h.rowptr, h.colidx, src, nthreads=8), f"push {bw_ratio} flags {flags}")


def test_symmetric_directed_equals_undirected():
    g = gg.barabasi_albert(4000, 3, 26)
    rp, ci = upload(g)
    nk.nk_set_tuning(flags=4)
    got = nk.nk_bc_directed(rp, ci, None, 1.0, rp, ci).cpu().numpy()
    assert_scores_close(got, nk.nk_bc_exact(rp, ci).cpu().numpy(), "symmetric")


@pytest.mark.parametrize("make", [lambda: gg.directed_rmat(14, 8, 27), lambda: gg.directed_random(5000, 1, 28),
                                  lambda: gg.directed_from_arcs(10, [], [], "no-arcs")])
def test_transpose_matches_host(make):
    g = make()
    rp, ci = upload(g)
    trp, tci = nk.nk_transpose(rp, ci)
    t = gg.transpose(g)
    assert np.array_equal(trp.cpu().numpy(), t.rowptr)
    assert np.array_equal(tci.cpu().numpy(), t.colidx)


def test_directed_rmat14_sampled_with_device_transpose():
    g = gg.directed_rmat(14, 16, 29)
    rp, ci = upload(g)
    trp, tci = nk.nk_transpose(rp, ci)
    src = gg.sample_sources(g.n, 256, 30)
    got = nk.nk_bc_directed(rp, ci, ivec(src), g.n / 256, trp, tci).cpu().numpy()
    assert_scores_close(got, oracle.bc_directed(g.rowptr, g.colidx, src, g.n / 256, nthreads=8), "drmat14")


def test_directed_errors():
    g = gg.directed_random(500, 2000, 31)
    rp, ci = upload(g)
    t = gg.transpose(g)
    trp, tci = _dev(t.rowptr), _dev(t.colidx)
    with pytest.raises(nk.NkError) as e:
        nk.nk_bc_directed(rp, ci, None, 1.0, trp, None)
    assert e.value.code == nk.NK_E_INVALID_ARG
    # in-arc rows of the wrong lengths (the out-arc CSR passed as its own transpose)
    with pytest.raises(nk.NkError) as e:
        nk.nk_bc_directed(rp, ci, None, 1.0, rp, ci)
    assert e.value.code == nk.NK_E_INVALID_GRAPH
    with pytest.raises(nk.NkError) as e:
        nk.nk_bc_directed(rp, ci, ivec([0, 500]), 1.0, trp, tci)
    assert e.value.code == nk.NK_E_INVALID_ARG
    bad = ci.clone()
    bad[0] = 500
    with pytest.raises(nk.NkError) as e:
        nk.nk_transpose(rp, bad)
    assert e.value.code == nk.NK_E_INVALID_GRAPH
    got = nk.nk_bc_directed(rp, ci, None, 1.0, trp, tci).cpu().numpy()
    assert_scores_close(got, oracle.bc_directed(g.rowptr, g.colidx), "after errors")
