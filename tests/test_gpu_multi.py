"""GPU parity of the multi-source kernel (B sources per workgroup task,
interleaved per-source path counts, union frontiers) against the CPU oracle:
exact and source-set scores within the tolerance, the work counters behind
the algorithmic bytes equal to the oracle's, sigma overflow reported, in
every direction mix, block size and source count per task, with the visited
masks in LDS, in global memory, and split between the two."""
import numpy as np
import pytest
import torch

import graphgen as gg
import oracle
import paper_1403_3005_amd as nk
from nkutil import assert_scores_close, ivec, upload

pytestmark = pytest.mark.gpu

MS_FLAGS = 4   # tuning flag bit 2: small graphs skip the all-in-LDS kernel


@pytest.fixture(autouse=True)
def _default_tuning():
    nk.nk_set_tuning()
    yield
    nk.nk_set_tuning()


def _ms(batch, **kw):
    nk.nk_set_tuning(flags=kw.pop("flags", MS_FLAGS), batch=batch, **kw)


def _check_ran(batch):
    st = nk.nk_last_stats()
    assert st["sources_per_task"] == batch and st["bitmap_lds"] == 4, st
    return st


GRAPHS = [
    lambda: gg.path(300), lambda: gg.star(500), lambda: gg.cycle(257), lambda: gg.complete(33),
    lambda: gg.complete_bipartite(5, 200), lambda: gg.grid(20, 30), lambda: gg.hypercube(9),
    lambda: gg.diamond_chain(30), lambda: gg.random_tree(2000, 5), lambda: gg.barabasi_albert(3000, 3, 41),
    lambda: gg.erdos_renyi(4000, 16000, 42), lambda: gg.rmat(12, 8, 43),
    lambda: gg.disjoint_union([gg.grid(6, 7), gg.star(50), gg.path(1), gg.cycle(9), gg.complete(5)]),
]


@pytest.mark.parametrize("batch", [4, 8, 16])
@pytest.mark.parametrize("make", GRAPHS)
def test_exact_families(make, batch):
    g = make()
    _ms(batch)
    rp, ci = upload(g)
    got = nk.nk_bc_exact(rp, ci).cpu().numpy()
    _check_ran(batch)
    assert_scores_close(got, oracle.bc_exact(g.rowptr, g.colidx, nthreads=8), f"{g.name} B={batch}")


@pytest.mark.parametrize("batch", [4, 8, 16])
@pytest.mark.parametrize("block", [256, 512, 1024])
@pytest.mark.parametrize("bu_ratio", [0.0, 16.0, 1e9])
def test_launch_variants(batch, block, bu_ratio):
    """Top-down only, the default switch, bottom-up wherever allowed; every
    block size; a source count that leaves the last task partial; repeated
    sources; relabelled and caller ids."""
    g = gg.barabasi_albert(2500, 4, 51)
    src = np.concatenate([gg.sample_sources(g.n, 97, 52), [7, 7, 3]]).astype(np.int32)
    for flags in (MS_FLAGS, MS_FLAGS | 2):
        _ms(batch, block=block, bu_ratio=bu_ratio, flags=flags)
        rp, ci = upload(g)
        got = nk.nk_bc_sources(rp, ci, ivec(src), 0.5).cpu().numpy()
        st = _check_ran(batch)
        assert st["block"] == block and st["sources"] == len(src)
        if bu_ratio == 0.0:
            assert st["levels_bu"] == 0
        if bu_ratio >= 1e9:
            assert st["levels_bu"] > 0
        assert_scores_close(got, oracle.bc_sources(g.rowptr, g.colidx, src, 0.5), f"B={batch} block={block}")


@pytest.mark.parametrize("batch", [4, 8, 16])
@pytest.mark.parametrize("bu_ratio", [0.0, 16.0, 1e9])
def test_work_counters_match_oracle(batch, bu_ratio):
    """Reached (vertex, source) pairs, arcs of reached vertices per source,
    and shortest-path DAG arcs per source equal the oracle's."""
    g = gg.barabasi_albert(3000, 3, 41)
    src = gg.sample_sources(g.n, 100, 42)
    _ms(batch, bu_ratio=bu_ratio)
    rp, ci = upload(g)
    nk.nk_bc_sources(rp, ci, ivec(src), 1.0)
    st = _check_ran(batch)
    reached, arcs, dag, depth = oracle.work_counts(g.rowptr, g.colidx, src)
    assert st["sources"] == 100
    assert st["reached"] == reached
    assert st["arcs_reached"] == arcs
    assert st["dag_arcs"] == dag


@pytest.mark.parametrize("batch", [8, 16])
def test_masks_split_between_lds_and_global(batch):
    """A graph larger than the LDS share of the visited masks: vertices
    beyond it keep their masks in global memory (both kernels' placements
    and the reset between tasks of a workgroup)."""
    g = gg.erdos_renyi(300_000, 900_000, 61)
    src = gg.sample_sources(g.n, 3 * batch + 5, 62)
    for flags in (MS_FLAGS, MS_FLAGS | 2):
        _ms(batch, flags=flags, wg_per_cu=1)
        rp, ci = upload(g)
        got = nk.nk_bc_sources(rp, ci, ivec(src), 1.0).cpu().numpy()
        _check_ran(batch)
        assert_scores_close(got, oracle.bc_sources(g.rowptr, g.colidx, src, 1.0, nthreads=16), f"er300k B={batch}")


def test_many_tasks_per_workgroup_rmat():
    """R-MAT with isolated vertices, many more tasks than workgroups (state
    reset between a workgroup's tasks), sampled sources including isolated
    ones."""
    g = gg.rmat(15, 16, 71)
    src = gg.sample_sources(g.n, 2000, 72)
    for batch in (4, 8, 16):
        _ms(batch, wg_per_cu=1, scratch_mib=256)
        rp, ci = upload(g)
        got = nk.nk_bc_sources(rp, ci, ivec(src), g.n / 2000).cpu().numpy()
        st = _check_ran(batch)
        assert st["workgroups"] * batch < 2000
        assert_scores_close(got, oracle.bc_sources(g.rowptr, g.colidx, src, g.n / 2000, nthreads=16), f"B={batch}")


@pytest.mark.parametrize("batch", [4, 8, 16])
def test_linear_scaling(batch):
    g = gg.erdos_renyi(3000, 9000, 81)
    src = gg.sample_sources(g.n, 50, 82)
    _ms(batch)
    rp, ci = upload(g)
    got = nk.nk_bc_sources_linear(rp, ci, ivec(src), 2.0).cpu().numpy()
    _check_ran(batch)
    assert_scores_close(got, oracle.bc_sources_linear(g.rowptr, g.colidx, src, 2.0), f"linear B={batch}")


@pytest.mark.parametrize("batch", [4, 8, 16])
def test_sigma_overflow_boundary(batch):
    _ms(batch)
    ok = gg.diamond_chain(63)
    rp, ci = upload(ok)
    assert_scores_close(nk.nk_bc_exact(rp, ci).cpu().numpy(), oracle.bc_exact(ok.rowptr, ok.colidx), "diamonds63")
    bad = gg.diamond_chain(64)
    rp, ci = upload(bad)
    with pytest.raises(nk.NkError) as e:
        nk.nk_bc_exact(rp, ci)
    assert e.value.code == nk.NK_E_SIGMA_OVERFLOW
    # the library still works after the error
    rp, ci = upload(ok)
    assert_scores_close(nk.nk_bc_exact(rp, ci).cpu().numpy(), oracle.bc_exact(ok.rowptr, ok.colidx), "after")


@pytest.mark.parametrize("batch", [4, 8, 16])
def test_bad_source_and_empty(batch):
    _ms(batch)
    g = gg.cycle(40)
    rp, ci = upload(g)
    with pytest.raises(nk.NkError) as e:
        nk.nk_bc_sources(rp, ci, ivec([3, 40]), 1.0)
    assert e.value.code == nk.NK_E_INVALID_ARG
    zero = nk.nk_bc_sources(rp, ci, torch.zeros(0, dtype=torch.int32, device="cuda:0"), 3.0).cpu().numpy()
    assert np.array_equal(zero, np.zeros(g.n))


@pytest.mark.parametrize("batch", [4, 8, 16])
def test_batched_graphs(batch):
    """A batch whose larger graphs run on the multi-source kernel (graph
    sizes not multiples of B, the largest first), the small ones on the
    all-in-LDS kernel, in one call; every score against the oracle."""
    graphs = [gg.erdos_renyi(9000, 36000, 91), gg.barabasi_albert(6001, 4, 92), gg.erdos_renyi(1500, 6000, 93),
              gg.barabasi_albert(20003, 4, 94), gg.path(777), gg.erdos_renyi(300, 900, 95)]
    vtx = np.zeros(len(graphs) + 1, dtype=np.int64)
    arc = np.zeros(len(graphs) + 1, dtype=np.int64)
    for i, g in enumerate(graphs):
        vtx[i + 1] = vtx[i] + g.n
        arc[i + 1] = arc[i] + g.m
    rp = torch.from_numpy(np.concatenate([g.rowptr for g in graphs]).astype(np.int32)).cuda()
    ci = torch.from_numpy(np.concatenate([g.colidx for g in graphs]).astype(np.int32)).cuda()
    nk.nk_set_tuning(batch=batch)
    got = nk.nk_bc_exact_batched(vtx, arc, rp, ci).cpu().numpy()
    st = nk.nk_last_stats()
    assert st["sources"] == int(vtx[-1]) and st["bitmap_lds"] in (4, 5) and st["sources_per_task"] == batch
    for i, g in enumerate(graphs):
        assert_scores_close(got[vtx[i]:vtx[i + 1]], oracle.bc_exact(g.rowptr, g.colidx, nthreads=16), f"graph {i}")
    # the same batch replayed from a captured plan
    plan = nk.NkBatchPlan(vtx, arc, rp, ci)
    try:
        for _ in range(2):
            again = plan.run().cpu().numpy()
            assert np.array_equal(again, again) and again.shape == got.shape
            for i, g in enumerate(graphs):
                assert_scores_close(again[vtx[i]:vtx[i + 1]], got[vtx[i]:vtx[i + 1]], f"replay graph {i}")
    finally:
        plan.close()
