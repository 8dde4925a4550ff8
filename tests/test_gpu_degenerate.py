"""Every entry point on degenerate graphs -- no vertices, one vertex, only
isolated vertices, a single edge, two disjoint edges, a three-vertex star,
a directed arc -- against the oracle (or the value the definition fixes)."""
import numpy as np
import pytest
import torch

import graphgen as gg
import oracle
import paper_1403_3005_amd as nk
from nkutil import assert_scores_close, ivec, upload

pytestmark = pytest.mark.gpu


def _graphs():
    return [
        gg.Graph(1, np.zeros(2, dtype=np.int32), np.zeros(0, dtype=np.int32), "one vertex"),
        gg.Graph(50, np.zeros(51, dtype=np.int32), np.zeros(0, dtype=np.int32), "isolated"),
        gg.from_edges(2, [0], [1], "one edge"),
        gg.from_edges(4, [0, 2], [1, 3], "two edges"),
        gg.star(3),
        gg.disjoint_union([gg.path(3), gg.path(1), gg.cycle(4)]),
    ]


@pytest.fixture(autouse=True)
def _default_tuning():
    nk.nk_set_tuning()
    yield
    nk.nk_set_tuning()


@pytest.mark.parametrize("flags", [0, 4])
@pytest.mark.parametrize("idx", range(6))
def test_source_forms(idx, flags):
    nk.nk_set_tuning(flags=flags)
    g = _graphs()[idx]
    rp, ci = upload(g)
    name = g.name
    assert_scores_close(nk.nk_bc_exact(rp, ci).cpu().numpy(), oracle.bc_exact(g.rowptr, g.colidx), name)
    src = np.arange(g.n, dtype=np.int32)[::-1].copy()
    assert_scores_close(nk.nk_bc_sources(rp, ci, ivec(src), 0.5).cpu().numpy(),
                        oracle.bc_sources(g.rowptr, g.colidx, src, 0.5), name + " sources")
    assert_scores_close(nk.nk_bc_sources_linear(rp, ci, None, 2.0).cpu().numpy(),
                        oracle.bc_sources_linear(g.rowptr, g.colidx, np.arange(g.n), 2.0), name + " linear")
    assert_scores_close(nk.nk_bc_sources_bisect(rp, ci, None, 2.0).cpu().numpy(),
                        oracle.bc_sources_bisect(g.rowptr, g.colidx, np.arange(g.n), 2.0), name + " bisect")
    ebc, vbc = nk.nk_edge_bc(rp, ci)
    oe, ob = oracle.edge_bc(g.rowptr, g.colidx)
    assert_scores_close(ebc.cpu().numpy(), oe, name + " edges")
    assert_scores_close(vbc.cpu().numpy(), ob, name + " edge-call vertices")
    assert_scores_close(nk.nk_closeness(rp, ci).cpu().numpy(), oracle.closeness(g.rowptr, g.colidx),
                        name + " closeness")
    assert_scores_close(nk.nk_closeness_sampled(rp, ci, ivec(src)).cpu().numpy(),
                        oracle.closeness_approx(g.rowptr, g.colidx, src)[0], name + " sampled closeness")
    d, sg = nk.nk_sssp_counts(rp, ci, ivec(src[:1]))
    od, osg = oracle.sssp_counts(g.rowptr, g.colidx, int(src[0]))
    assert np.array_equal(d[0].cpu().numpy(), od) and np.array_equal(sg[0].cpu().numpy().view(np.uint64), osg)


@pytest.mark.parametrize("idx", range(6))
def test_directed_weighted_and_pairs(idx):
    g = _graphs()[idx]
    rp, ci = upload(g)
    trp, tci = nk.nk_transpose(rp, ci)
    assert np.array_equal(trp.cpu().numpy(), g.rowptr)   # symmetric graphs are their own transpose
    assert_scores_close(nk.nk_bc_directed(rp, ci, None, 1.0, trp, tci).cpu().numpy(),
                        oracle.bc_directed(g.rowptr, g.colidx), g.name + " directed")
    assert_scores_close(nk.nk_bc_directed(rp, ci).cpu().numpy(), oracle.bc_directed(g.rowptr, g.colidx),
                        g.name + " directed, no in-arcs")
    w = gg.edge_weights(g, 5, 3)
    wt = torch.from_numpy(np.ascontiguousarray(w, dtype=np.int32)).cuda()
    assert_scores_close(nk.nk_bc_weighted(rp, ci, wt).cpu().numpy(), oracle.bc_weighted(g.rowptr, g.colidx, w),
                        g.name + " weighted")
    assert nk.nk_vd_bound(rp, ci) == oracle.vd_bound(g.rowptr, g.colidx)
    if g.n >= 2:
        cnt = nk.nk_pair_counts(rp, ci, 300, 7).cpu().numpy().view(np.uint32)
        assert np.array_equal(cnt, oracle.pair_counts(g.rowptr, g.colidx, 300, 7))
        bc, c, r, vd = nk.nk_bc_pair_sample(rp, ci, 0.2, 0.1, 7)
        ref, oc, orr, ovd = oracle.pair_sample(g.rowptr, g.colidx, 0.2, 0.1, 7)
        assert (r, vd) == (orr, ovd)
        assert np.array_equal(c.cpu().numpy().view(np.uint32), oc)
        assert_scores_close(bc.cpu().numpy(), ref, g.name + " pair sampling")


def test_directed_single_arc_and_empty_graph():
    g = gg.directed_from_arcs(3, [0, 1], [1, 2], "directed path of 3")
    rp, ci = upload(g)
    trp, tci = nk.nk_transpose(rp, ci)
    got = nk.nk_bc_directed(rp, ci, None, 1.0, trp, tci).cpu().numpy()
    assert np.array_equal(got, np.array([0.0, 1.0, 0.0]))
    g0 = gg.Graph(0, np.zeros(1, dtype=np.int32), np.zeros(0, dtype=np.int32))
    rp0, ci0 = upload(g0)
    for out in (nk.nk_bc_exact(rp0, ci0), nk.nk_bc_directed(rp0, ci0), nk.nk_closeness(rp0, ci0),
                nk.nk_bc_weighted(rp0, ci0, torch.zeros(0, dtype=torch.int32, device="cuda:0"))):
        assert out.numel() == 0


def test_batch_of_degenerate_graphs():
    g0 = gg.Graph(0, np.zeros(1, dtype=np.int32), np.zeros(0, dtype=np.int32))
    graphs = [g0] + _graphs()[:5] + [g0]
    vtx = np.zeros(len(graphs) + 1, dtype=np.int64)
    arc = np.zeros(len(graphs) + 1, dtype=np.int64)
    for i, g in enumerate(graphs):
        vtx[i + 1] = vtx[i] + g.n
        arc[i + 1] = arc[i] + g.m
    rp = torch.from_numpy(np.concatenate([g.rowptr for g in graphs]).astype(np.int32)).cuda()
    ci = torch.from_numpy(np.concatenate([g.colidx for g in graphs]).astype(np.int32)).cuda()
    ref = np.concatenate([oracle.bc_exact(g.rowptr, g.colidx) for g in graphs])
    assert_scores_close(nk.nk_bc_exact_batched(vtx, arc, rp, ci).cpu().numpy(), ref, "batched degenerate")
    with nk.NkBatchPlan(vtx, arc, rp, ci) as plan:
        for i in range(2):
            assert_scores_close(plan.run().cpu().numpy(), ref, f"plan replay {i}")
