"""GPU parity of the group kernel (the workgroups of one XCD run one source
together, one group barrier per level) against the CPU oracle: exact and
source-set scores within the tolerance, the work counters behind the
algorithmic bytes equal to the oracle's, sigma overflow reported, in every
direction mix, with one and two groups per XCD, single graphs and batches."""
import numpy as np
import pytest
import torch

import graphgen as gg
import oracle
import paper_1403_3005_amd as nk
from nkutil import assert_scores_close, ivec, upload

pytestmark = pytest.mark.gpu

GROUP = 8      # tuning flag bit 3: the group kernel
NO_LDS = 4     # bit 2: small graphs skip the all-in-LDS kernel


@pytest.fixture(autouse=True)
def _default_tuning():
    nk.nk_set_tuning()
    yield
    nk.nk_set_tuning()


def _grp(block=1024, flags=0, **kw):
    nk.nk_set_tuning(flags=GROUP | NO_LDS | flags, block=block, **kw)


def _check_ran(where=6):
    st = nk.nk_last_stats()
    assert st["bitmap_lds"] == where, st
    return st


GRAPHS = [
    lambda: gg.path(300), lambda: gg.star(500), lambda: gg.cycle(257), lambda: gg.complete(33),
    lambda: gg.complete_bipartite(5, 200), lambda: gg.grid(20, 30), lambda: gg.hypercube(9),
    lambda: gg.diamond_chain(30), lambda: gg.random_tree(2000, 5), lambda: gg.barabasi_albert(3000, 3, 41),
    lambda: gg.erdos_renyi(4000, 16000, 42), lambda: gg.rmat(12, 8, 43),
    lambda: gg.disjoint_union([gg.grid(6, 7), gg.star(50), gg.path(1), gg.cycle(9), gg.complete(5)]),
]


@pytest.mark.parametrize("block", [1024, 512])
@pytest.mark.parametrize("make", GRAPHS)
def test_exact_families(make, block):
    g = make()
    _grp(block)
    rp, ci = upload(g)
    got = nk.nk_bc_exact(rp, ci).cpu().numpy()
    st = _check_ran()
    assert st["block"] == block
    assert_scores_close(got, oracle.bc_exact(g.rowptr, g.colidx, nthreads=8), f"{g.name} block={block}")


@pytest.mark.parametrize("block", [1024, 512])
@pytest.mark.parametrize("bu_ratio", [0.0, 16.0, 1e9])
def test_launch_variants(block, bu_ratio):
    """Top-down only, the default switch, bottom-up wherever allowed;
    repeated sources; relabelled and caller ids."""
    g = gg.barabasi_albert(2500, 4, 51)
    src = np.concatenate([gg.sample_sources(g.n, 97, 52), [7, 7, 3]]).astype(np.int32)
    for flags in (0, 2):
        _grp(block, flags=flags, bu_ratio=bu_ratio)
        rp, ci = upload(g)
        got = nk.nk_bc_sources(rp, ci, ivec(src), 0.5).cpu().numpy()
        st = _check_ran()
        assert st["sources"] == len(src)
        if bu_ratio == 0.0:
            assert st["levels_bu"] == 0
        if bu_ratio >= 1e9:
            assert st["levels_bu"] > 0
        assert_scores_close(got, oracle.bc_sources(g.rowptr, g.colidx, src, 0.5), f"block={block} bu={bu_ratio}")


@pytest.mark.parametrize("bu_ratio", [0.0, 16.0, 1e9])
def test_work_counters_match_oracle(bu_ratio):
    """Reached vertices, arcs of reached vertices and shortest-path DAG arcs,
    summed over the sources, equal the oracle's."""
    g = gg.barabasi_albert(3000, 3, 41)
    src = gg.sample_sources(g.n, 100, 42)
    _grp(bu_ratio=bu_ratio)
    rp, ci = upload(g)
    nk.nk_bc_sources(rp, ci, ivec(src), 1.0)
    st = _check_ran()
    reached, arcs, dag, depth = oracle.work_counts(g.rowptr, g.colidx, src)
    assert st["sources"] == 100
    assert st["reached"] == reached
    assert st["arcs_reached"] == arcs
    assert st["dag_arcs"] == dag


@pytest.mark.parametrize("block", [1024, 512])
def test_mid_size_graphs(block):
    """Graphs of the size the kernel is for (bitmaps of 12-125 KB of LDS),
    sampled sources, many tasks per group."""
    cases = [gg.erdos_renyi(100_000, 400_000, 61), gg.barabasi_albert(200_000, 4, 62), gg.rmat(16, 16, 63)]
    for g in cases:
        src = gg.sample_sources(g.n, 300, 64)
        _grp(block)
        rp, ci = upload(g)
        got = nk.nk_bc_sources(rp, ci, ivec(src), g.n / 300).cpu().numpy()
        _check_ran()
        assert_scores_close(got, oracle.bc_sources(g.rowptr, g.colidx, src, g.n / 300, nthreads=16), g.name)


def test_largest_bitmap():
    """R-MAT scale 20: a 128 KB visited bitmap per workgroup, hubs of 10^5
    arcs, isolated vertices; a handful of sources checked."""
    g = gg.rmat(20, 16, 65)
    src = gg.sample_sources(g.n, 24, 66)
    _grp()
    rp, ci = upload(g)
    got = nk.nk_bc_sources(rp, ci, ivec(src), 1.0).cpu().numpy()
    _check_ran()
    assert_scores_close(got, oracle.bc_sources(g.rowptr, g.colidx, src, 1.0, nthreads=16), "rmat20")


def test_linear_scaling():
    g = gg.erdos_renyi(3000, 9000, 81)
    src = gg.sample_sources(g.n, 50, 82)
    _grp()
    rp, ci = upload(g)
    got = nk.nk_bc_sources_linear(rp, ci, ivec(src), 2.0).cpu().numpy()
    _check_ran()
    assert_scores_close(got, oracle.bc_sources_linear(g.rowptr, g.colidx, src, 2.0), "linear")


def test_sigma_overflow_boundary():
    _grp()
    ok = gg.diamond_chain(63)
    rp, ci = upload(ok)
    assert_scores_close(nk.nk_bc_exact(rp, ci).cpu().numpy(), oracle.bc_exact(ok.rowptr, ok.colidx), "diamonds63")
    bad = gg.diamond_chain(64)
    rp, ci = upload(bad)
    with pytest.raises(nk.NkError) as e:
        nk.nk_bc_exact(rp, ci)
    assert e.value.code == nk.NK_E_SIGMA_OVERFLOW
    rp, ci = upload(ok)
    assert_scores_close(nk.nk_bc_exact(rp, ci).cpu().numpy(), oracle.bc_exact(ok.rowptr, ok.colidx), "after")


def test_bad_source_and_empty():
    _grp()
    g = gg.cycle(40)
    rp, ci = upload(g)
    with pytest.raises(nk.NkError) as e:
        nk.nk_bc_sources(rp, ci, ivec([3, 40]), 1.0)
    assert e.value.code == nk.NK_E_INVALID_ARG
    zero = nk.nk_bc_sources(rp, ci, torch.zeros(0, dtype=torch.int32, device="cuda:0"), 3.0).cpu().numpy()
    assert np.array_equal(zero, np.zeros(g.n))
    # the library still works after the error
    got = nk.nk_bc_exact(rp, ci).cpu().numpy()
    assert_scores_close(got, oracle.bc_exact(g.rowptr, g.colidx), "cycle40")


@pytest.mark.parametrize("block", [1024, 512])
def test_batched_graphs(block):
    """A batch whose larger graphs run on the group kernel, the small ones on
    the all-in-LDS kernel; then the same batch replayed from a captured plan
    (plain launch inside the graph)."""
    graphs = [gg.erdos_renyi(9000, 36000, 91), gg.barabasi_albert(6001, 4, 92), gg.erdos_renyi(1500, 6000, 93),
              gg.barabasi_albert(20003, 4, 94), gg.path(777), gg.erdos_renyi(300, 900, 95)]
    vtx = np.zeros(len(graphs) + 1, dtype=np.int64)
    arc = np.zeros(len(graphs) + 1, dtype=np.int64)
    for i, g in enumerate(graphs):
        vtx[i + 1] = vtx[i] + g.n
        arc[i + 1] = arc[i] + g.m
    rp = torch.from_numpy(np.concatenate([g.rowptr for g in graphs]).astype(np.int32)).cuda()
    ci = torch.from_numpy(np.concatenate([g.colidx for g in graphs]).astype(np.int32)).cuda()
    nk.nk_set_tuning(flags=GROUP, block=block)
    got = nk.nk_bc_exact_batched(vtx, arc, rp, ci).cpu().numpy()
    st = nk.nk_last_stats()
    assert st["sources"] == int(vtx[-1]) and st["bitmap_lds"] in (6, 7), st
    refs = [oracle.bc_exact(g.rowptr, g.colidx, nthreads=16) for g in graphs]
    for i, g in enumerate(graphs):
        assert_scores_close(got[vtx[i]:vtx[i + 1]], refs[i], f"graph {i}")
    plan = nk.NkBatchPlan(vtx, arc, rp, ci)
    try:
        for _ in range(2):
            again = plan.run().cpu().numpy()
            for i, g in enumerate(graphs):
                assert_scores_close(again[vtx[i]:vtx[i + 1]], refs[i], f"replay graph {i}")
    finally:
        plan.close()


def test_automatic_choice_and_opt_out():
    """Default tuning runs a sparse graph of 1.5 * 10^5 vertices on the group
    kernel and a denser or smaller one on the one-source kernel; flag bit 4
    keeps every graph off the group kernel.  Scores agree either way."""
    g = gg.erdos_renyi(150_000, 600_000, 71)
    src = gg.sample_sources(g.n, 64, 72)
    rp, ci = upload(g)
    ref = oracle.bc_sources(g.rowptr, g.colidx, src, 1.0, nthreads=16)
    nk.nk_set_tuning()
    got = nk.nk_bc_sources(rp, ci, ivec(src), 1.0).cpu().numpy()
    _check_ran(6)
    assert_scores_close(got, ref, "automatic")
    nk.nk_set_tuning(flags=16)
    got = nk.nk_bc_sources(rp, ci, ivec(src), 1.0).cpu().numpy()
    assert nk.nk_last_stats()["bitmap_lds"] == 1
    assert_scores_close(got, ref, "opted out")
    nk.nk_set_tuning()
    small = gg.erdos_renyi(50_000, 200_000, 73)
    srp, sci = upload(small)
    nk.nk_bc_sources(srp, sci, ivec(gg.sample_sources(small.n, 16, 74)), 1.0)
    assert nk.nk_last_stats()["bitmap_lds"] == 1


def test_batch_three_way_split():
    """Default tuning on a batch with graphs for all three kernels: small
    ones in LDS, mid-size ones on the one-source kernel, the 10^5-vertex one
    on the group kernel (three launches, one call); then a captured plan."""
    graphs = [gg.erdos_renyi(120_000, 480_000, 75), gg.barabasi_albert(9000, 4, 76), gg.erdos_renyi(800, 3200, 77),
              gg.path(5), gg.erdos_renyi(20_000, 80_000, 78)]
    vtx = np.zeros(len(graphs) + 1, dtype=np.int64)
    arc = np.zeros(len(graphs) + 1, dtype=np.int64)
    for i, g in enumerate(graphs):
        vtx[i + 1] = vtx[i] + g.n
        arc[i + 1] = arc[i] + g.m
    rp = torch.from_numpy(np.concatenate([g.rowptr for g in graphs]).astype(np.int32)).cuda()
    ci = torch.from_numpy(np.concatenate([g.colidx for g in graphs]).astype(np.int32)).cuda()
    nk.nk_set_tuning()
    got = nk.nk_bc_exact_batched(vtx, arc, rp, ci).cpu().numpy()
    st = nk.nk_last_stats()
    assert st["bitmap_lds"] == 7 and st["sources"] == int(vtx[-1]), st
    # the 1.2 * 10^5-vertex graph: exact scores are too slow for the oracle,
    # so check the smaller graphs exactly and the large one against the
    # one-source kernel on the same graph
    for i in range(1, len(graphs)):
        g = graphs[i]
        assert_scores_close(got[vtx[i]:vtx[i + 1]], oracle.bc_exact(g.rowptr, g.colidx, nthreads=16), f"graph {i}")
    big = graphs[0]
    brp, bci = upload(big)
    nk.nk_set_tuning(flags=16)
    ref_big = nk.nk_bc_exact(brp, bci).cpu().numpy()
    assert nk.nk_last_stats()["bitmap_lds"] == 1
    assert_scores_close(got[:big.n], ref_big, "graph 0 vs one-source kernel")
    nk.nk_set_tuning()
    with nk.NkBatchPlan(vtx, arc, rp, ci) as plan:
        again = plan.run().cpu().numpy()
        assert nk.nk_last_stats()["bitmap_lds"] == 7
        assert_scores_close(again, got, "replay")


def test_cached_kernel_choice(tmp_path):
    """A registered autotuner cache entry carries the kernel choice: an
    eight-value entry with flag bit 3 runs a graph of its shape on the group
    kernel, one with bit 4 keeps the same graph on the one-source kernel,
    whatever the automatic choice would be; scores agree with the oracle."""
    import json

    g = gg.erdos_renyi(60_000, 240_000, 79)          # below the automatic range
    src = gg.sample_sources(g.n, 48, 80)
    rp, ci = upload(g)
    ref = oracle.bc_sources(g.rowptr, g.colidx, src, 1.0, nthreads=16)
    deg = g.degrees()
    mean = g.m / g.n
    key = "n%d_d%d_s%d" % (int(np.floor(np.log2(g.n))), int(np.round(np.log2(mean))),
                           int(np.round(np.log2(deg.max() / mean))))
    cache = tmp_path / "tune.json"
    try:
        for kflags, where in ((8, 6), (16, 1)):
            cache.write_text(json.dumps({key: [1024, 16, 0.1, 0, 1, 10.0, kflags, 2]}))
            nk.nk_set_tuning_cache(str(cache))
            got = nk.nk_bc_sources(rp, ci, ivec(src), 1.0).cpu().numpy()
            assert nk.nk_last_stats()["bitmap_lds"] == where, kflags
            assert_scores_close(got, ref, f"cached flags {kflags}")
    finally:
        nk.nk_set_tuning_cache(None)
