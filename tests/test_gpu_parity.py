"""GPU parity: the HIP path through the C ABI against the CPU oracle on the
same seeded inputs.  d and sigma bit-exact; scores within the tolerance in
tests/nkutil.py."""
import json
import os
from fractions import Fraction

import numpy as np
import pytest
import torch

import graphgen as gg
import oracle
import paper_1403_3005_amd as nk
from nkutil import assert_scores_close, ivec, upload

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "bruteforce_small.json")


@pytest.fixture(autouse=True)
def _default_tuning():
    nk.nk_set_tuning()
    yield
    nk.nk_set_tuning()


def _exact(g):
    rp, ci = upload(g)
    return nk.nk_bc_exact(rp, ci).cpu().numpy()


def _sssp_check(g, sources):
    rp, ci = upload(g)
    d, s = nk.nk_sssp_counts(rp, ci, ivec(sources))
    d = d.cpu().numpy()
    s = s.cpu().numpy().view(np.uint64)
    for i, src in enumerate(sources):
        od, os_ = oracle.sssp_counts(g.rowptr, g.colidx, int(src))
        assert np.array_equal(d[i], od), (g.name, src)
        assert np.array_equal(s[i], os_), (g.name, src)


def test_golden_bruteforce():
    with open(GOLDEN) as f:
        cases = json.load(f)
    for case in cases:
        g = gg.Graph(case["n"], np.array(case["rowptr"], dtype=np.int32), np.array(case["colidx"], dtype=np.int32))
        got = _exact(g)
        for v, frac in enumerate(case["bc"]):
            exact = Fraction(frac)
            assert abs(Fraction(got[v]) - exact) <= Fraction(1, 10 ** 12) * max(1, abs(exact)), (case["name"], v)
        rp, ci = upload(g)
        d, s = nk.nk_sssp_counts(rp, ci, ivec(range(g.n)))
        assert d.cpu().numpy().tolist() == case["d"]
        assert s.cpu().numpy().view(np.uint64).astype(object).tolist() == case["sigma"]


FAMILIES = [
    lambda: gg.path(1), lambda: gg.path(2), lambda: gg.path(700), lambda: gg.star(3000), lambda: gg.cycle(501),
    lambda: gg.cycle(64), lambda: gg.complete(40), lambda: gg.complete_bipartite(7, 300), lambda: gg.grid(30, 40),
    lambda: gg.hypercube(10), lambda: gg.diamond_chain(40), lambda: gg.random_tree(3000, 9),
    lambda: gg.disjoint_union([gg.grid(6, 7), gg.star(50), gg.path(1), gg.cycle(9), gg.complete(5)]),
]


# tuning flag bit 2 turns the all-in-LDS small-graph kernel off, so every
# small graph below runs on both kernels
PATHS = [0, 4]


def _path_check(flags):
    st = nk.nk_last_stats()
    if flags & 4:
        assert st["bitmap_lds"] in (0, 1)
    return st


@pytest.mark.parametrize("flags", PATHS)
@pytest.mark.parametrize("make", FAMILIES)
def test_exact_families(make, flags):
    nk.nk_set_tuning(flags=flags)
    g = make()
    assert_scores_close(_exact(g), oracle.bc_exact(g.rowptr, g.colidx), g.name)
    _path_check(flags)


RANDOM = [
    lambda: gg.erdos_renyi(1500, 4000, 21),
    lambda: gg.erdos_renyi(3000, 2500, 22),  # many components
    lambda: gg.barabasi_albert(4000, 4, 23),
    lambda: gg.rmat(12, 16, 24),
    lambda: gg.chung_lu(5000, 2.5, 20.0, 25),
]


@pytest.mark.parametrize("flags", PATHS)
@pytest.mark.parametrize("make", RANDOM)
def test_exact_random(make, flags):
    nk.nk_set_tuning(flags=flags)
    g = make()
    assert_scores_close(_exact(g), oracle.bc_exact(g.rowptr, g.colidx), g.name)
    _path_check(flags)


@pytest.mark.parametrize("block", [256, 512, 1024])
def test_lds_path_used_and_exact(block):
    """Graphs that fit one workgroup's LDS run on the all-in-LDS kernel at
    every block size; results match the oracle on a tile-spanning hub, a
    700-level path and a random graph."""
    nk.nk_set_tuning(block=block)
    for g in (gg.star(2500), gg.path(700), gg.erdos_renyi(2000, 6000, 71), gg.barabasi_albert(1200, 5, 72)):
        got = _exact(g)
        st = nk.nk_last_stats()
        assert st["bitmap_lds"] == 2 and st["block"] == block, g.name
        assert st["sources"] == g.n
        assert_scores_close(got, oracle.bc_exact(g.rowptr, g.colidx), g.name)
        src = gg.sample_sources(g.n, 37, 73)
        rp, ci = upload(g)
        got = nk.nk_bc_sources(rp, ci, ivec(src), 2.5).cpu().numpy()
        assert_scores_close(got, oracle.bc_sources(g.rowptr, g.colidx, src, 2.5), g.name + " sources")


@pytest.mark.parametrize("make", RANDOM + FAMILIES[2:6])
def test_sssp_bit_exact(make):
    g = make()
    srcs = sorted(set([0, g.n - 1, g.n // 2, g.n // 3, int(np.argmax(g.degrees()))]))
    _sssp_check(g, srcs)


def test_exact_er2000_full():
    """The exact all-sources workload: G(2000, 10000), seed 1."""
    g = gg.workload_er2000()
    assert_scores_close(_exact(g), oracle.bc_exact(g.rowptr, g.colidx), "er2000")
    st = nk.nk_last_stats()
    assert st["sources"] == 2000
    _sssp_check(g, list(range(0, 2000, 97)))


@pytest.mark.parametrize("block", [256, 512, 1024])
@pytest.mark.parametrize("bu_ratio", [0.0, 16.0, 1e9])
@pytest.mark.parametrize("flags", [4, 5, 6])
@pytest.mark.parametrize("bw_ratio", [0.0, 0.1, 1e9])
def test_launch_variants(block, bu_ratio, flags, bw_ratio):
    """Global-memory kernel (the all-in-LDS one is off): every block size,
    forward direction policy (never / default / always bottom-up after the
    first level), backward policy (always pull / default / always push),
    bitmap placement and vertex order (relabelled or as given) gives the
    same result."""
    nk.nk_set_tuning(block=block, bu_ratio=bu_ratio, wg_per_cu=0, flags=flags, bw_ratio=bw_ratio)
    g = gg.rmat(11, 8, 31)
    src = gg.sample_sources(g.n, 64, 32)
    rp, ci = upload(g)
    got = nk.nk_bc_sources(rp, ci, ivec(src), g.n / 64).cpu().numpy()
    st = nk.nk_last_stats()
    assert st["block"] == block and st["bitmap_lds"] == (0 if flags & 1 else 1)
    if bu_ratio == 0.0:
        assert st["levels_bu"] == 0
    if bu_ratio == 1e9:
        assert st["levels_bu"] > 0
    if bw_ratio == 0.0:
        assert st["levels_bw_push"] == 0
    if bw_ratio == 1e9:
        assert st["levels_bw_push"] > 0
    assert_scores_close(got, oracle.bc_sources(g.rowptr, g.colidx, src, g.n / 64), "variant")
    d, s = nk.nk_sssp_counts(rp, ci, ivec(src[:4]))
    for i in range(4):
        od, os_ = oracle.sssp_counts(g.rowptr, g.colidx, int(src[i]))
        assert np.array_equal(d[i].cpu().numpy(), od)
        assert np.array_equal(s[i].cpu().numpy().view(np.uint64), os_)


def test_scratch_cap_shrinks_the_grid():
    """A scratch cap of 8 MiB leaves room for 11 slots of a 16k-vertex graph
    (44 bytes per vertex per slot); results stay exact.  A cap below one
    slot is NK_E_NO_MEMORY.  Pair sampling (68 bytes per vertex per slot)
    honours the cap too."""
    g = gg.rmat(14, 16, 44)
    rp, ci = upload(g)
    src = gg.sample_sources(g.n, 100, 45)
    nk.nk_set_tuning(flags=4, scratch_mib=8)
    got = nk.nk_bc_sources(rp, ci, ivec(src), 1.0).cpu().numpy()
    stride = (g.n + 2 + 63) // 64 * 64
    assert nk.nk_last_stats()["workgroups"] == (8 << 20) // (stride * 44)
    assert_scores_close(got, oracle.bc_sources(g.rowptr, g.colidx, src), "capped")
    cnt = nk.nk_pair_counts(rp, ci, 300, 46).cpu().numpy().view(np.uint32)
    assert nk.nk_last_stats()["workgroups"] <= (8 << 20) // (stride * 68)
    assert np.array_equal(cnt, oracle.pair_counts(g.rowptr, g.colidx, 300, 46))
    nk.nk_set_tuning(flags=4, scratch_mib=0)
    big = gg.rmat(15, 16, 47)
    rp2, ci2 = upload(big)
    nk.nk_set_tuning(flags=4, scratch_mib=1)
    with pytest.raises(nk.NkError) as e:
        nk.nk_bc_sources(rp2, ci2, ivec([0, 1]), 1.0)
    assert e.value.code == nk.NK_E_NO_MEMORY


@pytest.mark.parametrize("flags", PATHS)
@pytest.mark.parametrize("bu_ratio,bw_ratio", [(0.0, 0.1), (16.0, 0.1), (1e9, 1e9), (1e9, 0.0)])
def test_work_counters_match_oracle(flags, bu_ratio, bw_ratio):
    """The counts behind the algorithmic bytes (reached vertices, arcs of
    reached vertices, shortest-path DAG arcs) equal the oracle's in every
    direction mix: top-down only, the benchmark's thresholds, bottom-up and
    push wherever allowed, bottom-up with pull only.  The all-in-LDS kernel
    (flags 0 on this graph) is always top-down and pull."""
    nk.nk_set_tuning(block=0, bu_ratio=bu_ratio, bw_ratio=bw_ratio, flags=flags)
    g = gg.barabasi_albert(3000, 3, 41)
    src = gg.sample_sources(g.n, 100, 42)
    rp, ci = upload(g)
    got = nk.nk_bc_sources(rp, ci, ivec(src), 1.0).cpu().numpy()
    st = nk.nk_last_stats()
    reached, arcs, dag, depth = oracle.work_counts(g.rowptr, g.colidx, src)
    assert st["sources"] == 100
    assert st["reached"] == reached
    assert st["arcs_reached"] == arcs
    assert st["dag_arcs"] == dag
    assert st["levels_td"] + st["levels_bu"] == depth + 100  # one extra (empty) expansion per source
    lds = st["bitmap_lds"] == 2
    assert lds == (flags == 0)
    if bu_ratio == 0.0 or lds:
        assert st["arcs_fwd"] == arcs and st["levels_bu"] == 0
    else:
        assert st["levels_bu"] > 0
    if bw_ratio >= 1e9 and not lds:
        assert st["levels_bw_push"] > 0
    if bw_ratio == 0.0:
        assert st["levels_bw_push"] == 0
    assert_scores_close(got, oracle.bc_sources(g.rowptr, g.colidx, src), "counters run")


def test_sources_forms_and_duplicates():
    g = gg.barabasi_albert(2000, 2, 51)
    rp, ci = upload(g)
    src = [5, 9, 5, 1999, 0]
    got = nk.nk_bc_sources(rp, ci, ivec(src), 0.25).cpu().numpy()
    assert_scores_close(got, oracle.bc_sources(g.rowptr, g.colidx, src, 0.25), "dups")
    allsrc = nk.nk_bc_sources(rp, ci, ivec(range(g.n)), 1.0).cpu().numpy()
    assert_scores_close(allsrc, _exact(g), "all-vs-exact")
    zero = nk.nk_bc_sources(rp, ci, torch.zeros(0, dtype=torch.int32, device="cuda:0"), 3.0).cpu().numpy()
    assert np.array_equal(zero, np.zeros(g.n))


def test_rmat14_sampled_sources():
    g = gg.rmat(14, 16, 2)
    src = gg.sample_sources(g.n, 512, 2)
    rp, ci = upload(g)
    got = nk.nk_bc_sources(rp, ci, ivec(src), g.n / 512).cpu().numpy()
    assert_scores_close(got, oracle.bc_sources(g.rowptr, g.colidx, src, g.n / 512), "rmat14")


def test_edge_cases():
    # isolated vertices only
    g = gg.Graph(50, np.zeros(51, dtype=np.int32), np.zeros(0, dtype=np.int32))
    assert np.array_equal(_exact(g), np.zeros(50))
    # a single vertex
    g1 = gg.Graph(1, np.zeros(2, dtype=np.int32), np.zeros(0, dtype=np.int32))
    assert np.array_equal(_exact(g1), np.zeros(1))
    # empty graph
    g0 = gg.Graph(0, np.zeros(1, dtype=np.int32), np.zeros(0, dtype=np.int32))
    rp, ci = upload(g0)
    assert nk.nk_bc_exact(rp, ci).numel() == 0


def test_invalid_graph_and_args():
    g = gg.cycle(100)
    bad = g.colidx.copy()
    bad[7] = 100
    rp = torch.from_numpy(g.rowptr).cuda()
    with pytest.raises(nk.NkError) as e:
        nk.nk_bc_exact(rp, torch.from_numpy(bad).cuda())
    assert e.value.code == nk.NK_E_INVALID_GRAPH
    badrp = g.rowptr.copy()
    badrp[10] = badrp[11] + 1
    with pytest.raises(nk.NkError) as e:
        nk.nk_bc_exact(torch.from_numpy(badrp).cuda(), torch.from_numpy(g.colidx).cuda())
    assert e.value.code == nk.NK_E_INVALID_GRAPH
    rp, ci = upload(g)
    with pytest.raises(nk.NkError) as e:
        nk.nk_bc_sources(rp, ci, ivec([3, 100]), 1.0)
    assert e.value.code == nk.NK_E_INVALID_ARG
    with pytest.raises(nk.NkError) as e:
        nk.nk_validate_graph(rp, torch.from_numpy(np.ascontiguousarray(g.colidx[::-1])).cuda(), strict=True)
    assert e.value.code == nk.NK_E_INVALID_GRAPH
    nk.nk_validate_graph(rp, ci, strict=True)
    # the library still works after errors
    assert_scores_close(_exact(g), oracle.bc_exact(g.rowptr, g.colidx), "after-errors")


def test_sigma_overflow_boundary():
    ok = gg.diamond_chain(63)
    assert_scores_close(_exact(ok), oracle.bc_exact(ok.rowptr, ok.colidx), "diamonds63")
    _sssp_check(ok, [0, 3 * 63])
    bad = gg.diamond_chain(64)
    rp, ci = upload(bad)
    with pytest.raises(nk.NkError) as e:
        nk.nk_bc_exact(rp, ci)
    assert e.value.code == nk.NK_E_SIGMA_OVERFLOW
    with pytest.raises(nk.NkError) as e:
        nk.nk_sssp_counts(rp, ci, ivec([0]))
    assert e.value.code == nk.NK_E_SIGMA_OVERFLOW
    # sources whose counts stay below 2^64 succeed on the same graph
    got = nk.nk_bc_sources(rp, ci, ivec([96, 97]), 1.0).cpu().numpy()
    assert_scores_close(got, oracle.bc_sources(bad.rowptr, bad.colidx, [96, 97]), "diamonds64-mid")
    for rows, fits in [(34, True), (35, False)]:
        grid = gg.grid(rows, rows)
        rp, ci = upload(grid)
        if fits:
            _sssp_check(grid, [0])
        else:
            with pytest.raises(nk.NkError) as e:
                nk.nk_bc_sources(rp, ci, ivec([0]), 1.0)
            assert e.value.code == nk.NK_E_SIGMA_OVERFLOW


def test_repeat_calls_deterministic_integers():
    g = gg.rmat(12, 16, 61)
    rp, ci = upload(g)
    src = ivec(gg.sample_sources(g.n, 256, 62))
    a = nk.nk_bc_sources(rp, ci, src, 1.0).cpu().numpy()
    b = nk.nk_bc_sources(rp, ci, src, 1.0).cpu().numpy()
    assert_scores_close(a, b, "repeat")
    d1, s1 = nk.nk_sssp_counts(rp, ci, src[:8])
    d2, s2 = nk.nk_sssp_counts(rp, ci, src[:8])
    assert torch.equal(d1, d2) and torch.equal(s1, s2)


# ----------------------------------------------------------- pair sampling --

@pytest.mark.parametrize("make", [
    lambda: gg.star(40), lambda: gg.path(30), lambda: gg.grid(12, 15), lambda: gg.erdos_renyi(800, 1200, 71),
    lambda: gg.barabasi_albert(1500, 2, 72), lambda: gg.disjoint_union([gg.star(30), gg.path(25), gg.cycle(7)]),
    lambda: gg.chung_lu(20000, 2.5, 20.0, 73),
])
def test_vd_bound_matches_oracle(make):
    g = make()
    rp, ci = upload(g)
    assert nk.nk_vd_bound(rp, ci) == oracle.vd_bound(g.rowptr, g.colidx)


def _broom_graph():
    """A hub with 12,000 leaves, every 40th leaf tied into a sparse random
    graph of 50,000 vertices and 150,000 edges: the sweep from the hub takes
    top-down levels whose arcs span several tiles of 2048, the first one all
    from a single vertex."""
    er = gg.erdos_renyi(50000, 150000, 74)
    a, b = er.edges()
    leaves = np.arange(1, 12001)
    u = np.concatenate([np.zeros(12000, dtype=np.int64), leaves[::40], a + 12001])
    v = np.concatenate([leaves, 12001 + (leaves[::40] * 7919) % 50000, b + 12001])
    return gg.from_edges(62001, u, v, "broom")


def test_vd_bound_balanced_top_down():
    g = _broom_graph()
    rp, ci = upload(g)
    info = nk.nk_vd_bound(rp, ci)
    assert info == oracle.vd_bound(g.rowptr, g.colidx)
    assert info["x0"] == 0


def _deferred_bottom_up_graph():
    """A graph whose breadth-first sweep from the hub takes a bottom-up
    step in which an unreached vertex of degree 301 finds its only frontier
    neighbour after its first 256 arcs (the wave-per-vertex pass), plus a
    second component of 350 vertices."""
    edges = [(0, 10000 + i) for i in range(1000)]            # hub 0, level 1 at ids 10000..10999
    edges += [(5000, 2000 + i) for i in range(300)]          # vertex 5000: 300 leaves with low ids ...
    edges.append((5000, 10999))                              # ... then its frontier neighbour
    edges += [(20000 + i, 20001 + i) for i in range(349)]    # a path of 350 vertices elsewhere
    u, v = zip(*edges)
    return gg.from_edges(20400, np.array(u), np.array(v), "deferred-bottom-up")


def test_vd_bound_deferred_bottom_up():
    g = _deferred_bottom_up_graph()
    rp, ci = upload(g)
    info = nk.nk_vd_bound(rp, ci)
    assert info == oracle.vd_bound(g.rowptr, g.colidx)
    assert info["c2"] == 350 and info["e1"] == 3


@pytest.mark.parametrize("make,r,seed", [
    (lambda: gg.grid(8, 9), 3000, 5), (lambda: gg.erdos_renyi(600, 1500, 81), 2000, 6),
    (lambda: gg.barabasi_albert(2000, 3, 82), 1500, 7), (lambda: gg.rmat(11, 16, 83), 1000, 8),
    (lambda: gg.hypercube(9), 800, 9),
])
def test_pair_counts_bit_exact(make, r, seed):
    g = make()
    rp, ci = upload(g)
    got = nk.nk_pair_counts(rp, ci, r, seed).cpu().numpy().view(np.uint32)
    ref = oracle.pair_counts(g.rowptr, g.colidx, r, seed)
    assert np.array_equal(got, ref)


def test_pair_record_block_reused_across_sizes():
    """Pair launches reuse the previous launch's record block without a
    fill when it is left all unreached.  Betweenness calls in between leave
    dirty pool blocks of other sizes behind; every pair result, on graphs
    growing and shrinking, stays bit-exact."""
    nk.nk_shutdown()
    graphs = [gg.rmat(10, 8, 91), gg.rmat(12, 8, 92), gg.rmat(13, 8, 93), gg.rmat(11, 8, 94), gg.rmat(13, 16, 95)]
    big = gg.rmat(14, 16, 96)
    brp, bci = upload(big)
    for i, g in enumerate(graphs):
        nk.nk_bc_sources(brp, bci, ivec(gg.sample_sources(big.n, 300 + 100 * i, 97)), 1.0)
        rp, ci = upload(g)
        for seed in (98, 99):
            got = nk.nk_pair_counts(rp, ci, 700, seed + i).cpu().numpy().view(np.uint32)
            assert np.array_equal(got, oracle.pair_counts(g.rowptr, g.colidx, 700, seed + i)), (g.name, seed)


def test_sample_paths_bit_exact():
    g = gg.barabasi_albert(3000, 2, 91)
    rp, ci = upload(g)
    uv, ln, path = nk.nk_sample_paths(rp, ci, 11, 100, 64, 32)
    uv, ln, path = uv.cpu().numpy(), ln.cpu().numpy(), path.cpu().numpy()
    for i in range(64):
        u, v, interior = oracle.sample_path(g.rowptr, g.colidx, 11, 100 + i)
        assert (uv[i, 0], uv[i, 1]) == (u, v)
        if interior is None:
            assert ln[i] == -1
        else:
            assert ln[i] == len(interior)
            assert path[i, :ln[i]].tolist() == interior


@pytest.mark.parametrize("make,eps,seed", [
    (lambda: gg.barabasi_albert(400, 2, 101), 0.05, 3), (lambda: gg.grid(10, 10), 0.08, 4),
    (lambda: gg.disjoint_union([gg.erdos_renyi(300, 500, 102), gg.path(40)]), 0.06, 5),
])
def test_pair_sample_matches_oracle(make, eps, seed):
    g = make()
    rp, ci = upload(g)
    bc, cnt, r, vd = nk.nk_bc_pair_sample(rp, ci, eps, 0.1, seed)
    obc, ocnt, orr, ovd = oracle.pair_sample(g.rowptr, g.colidx, eps, 0.1, seed)
    assert (r, vd) == (orr, ovd)
    assert np.array_equal(cnt.cpu().numpy().view(np.uint32), ocnt)
    assert_scores_close(bc.cpu().numpy(), obc, "pair-bc")


# ----------------------------------------------------------------- batched --

def _batched_inputs(graphs):
    vtx = np.zeros(len(graphs) + 1, dtype=np.int64)
    arc = np.zeros(len(graphs) + 1, dtype=np.int64)
    for i, g in enumerate(graphs):
        vtx[i + 1] = vtx[i] + g.n
        arc[i + 1] = arc[i] + g.m
    rp = np.concatenate([g.rowptr for g in graphs]).astype(np.int32)
    ci = np.concatenate([g.colidx for g in graphs]).astype(np.int32) if arc[-1] else np.zeros(0, np.int32)
    return vtx, arc, torch.from_numpy(rp).cuda(), torch.from_numpy(ci).cuda()


@pytest.mark.parametrize("flags", PATHS)
def test_batched_small_mixed(flags):
    nk.nk_set_tuning(flags=flags)
    sizes = gg.batched_sizes(24, 50, 3000, 111)
    graphs = []
    for i, n in enumerate(sizes):
        graphs.append(gg.erdos_renyi(n, 4 * n, 200 + i) if i % 2 == 0 else gg.barabasi_albert(n, 4, 200 + i))
    graphs.insert(5, gg.Graph(1, np.zeros(2, dtype=np.int32), np.zeros(0, dtype=np.int32)))
    graphs.insert(9, gg.path(2))
    vtx, arc, rp, ci = _batched_inputs(graphs)
    got = nk.nk_bc_exact_batched(vtx, arc, rp, ci).cpu().numpy()
    for i, g in enumerate(graphs):
        assert_scores_close(got[vtx[i]:vtx[i + 1]], oracle.bc_exact(g.rowptr, g.colidx), f"graph {i}")
    assert nk.nk_last_stats()["sources"] == int(vtx[-1])


def test_batched_split_between_kernels():
    """A batch holding graphs on both sides of the LDS limit: the small ones
    run on the all-in-LDS kernel, the large ones on the global kernel, in
    one call."""
    graphs = [gg.erdos_renyi(900, 3600, 131), gg.barabasi_albert(9000, 4, 132), gg.path(3),
              gg.erdos_renyi(12000, 48000, 133), gg.star(700)]
    vtx, arc, rp, ci = _batched_inputs(graphs)
    got = nk.nk_bc_exact_batched(vtx, arc, rp, ci).cpu().numpy()
    st = nk.nk_last_stats()
    assert st["bitmap_lds"] == 3 and st["sources"] == int(vtx[-1])
    for i, g in enumerate(graphs):
        assert_scores_close(got[vtx[i]:vtx[i + 1]], oracle.bc_exact(g.rowptr, g.colidx, nthreads=8), f"graph {i}")


def test_pair_isolated_targets():
    """Pairs whose target (or source) is an isolated vertex add nothing."""
    g = gg.disjoint_union([gg.star(20), gg.path(1), gg.path(1), gg.path(1), gg.cycle(6)])
    rp, ci = upload(g)
    got = nk.nk_pair_counts(rp, ci, 5000, 12).cpu().numpy().view(np.uint32)
    assert np.array_equal(got, oracle.pair_counts(g.rowptr, g.colidx, 5000, 12))
    uv, ln, path = nk.nk_sample_paths(rp, ci, 12, 0, 200, 8)
    for i in range(200):
        u, v, interior = oracle.sample_path(g.rowptr, g.colidx, 12, i)
        assert ln[i].item() == (-1 if interior is None else len(interior))


def test_autotune_picks_a_valid_tuning(tmp_path):
    g = gg.rmat(12, 16, 121)
    rp, ci = upload(g)
    src = ivec(gg.sample_sources(g.n, 64, 122))
    before = nk.nk_get_tuning()
    cache = str(tmp_path / "tune.json")
    best = nk.nk_autotune(rp, ci, src, cache)
    assert nk.nk_get_tuning() == before  # unchanged
    assert best["block"] in (256, 512, 1024)
    deg = g.degrees()
    assert nk.nk_tuning_lookup(cache, g.n, g.m, int(deg.max())) == best
    nk.nk_set_tuning(**best)
    got = nk.nk_bc_sources(rp, ci, src, 1.0).cpu().numpy()
    assert_scores_close(got, oracle.bc_sources(g.rowptr, g.colidx, src.cpu().numpy()), "tuned")


def _retune_cache(path, **fields):
    """Rewrites every entry of an autotuner cache with the given fields."""
    order = ["block", "bu_ratio", "bw_ratio", "wg_per_cu", "batch"]
    with open(path) as f:
        c = json.load(f)
    for k, v in c.items():
        for name, val in fields.items():
            v[order.index(name)] = val
    with open(path, "w") as f:
        json.dump(c, f)


def test_cached_tuning_applies_without_set_tuning(tmp_path):
    """A registered cache entry is picked up by nk_bc_sources, the batched
    plan and the server for graphs of its shape (no nk_set_tuning), results
    match the oracle; graphs of other shapes, and all graphs once the cache
    is unregistered, run under the global tuning."""
    g = gg.barabasi_albert(20000, 4, 123)
    rp, ci = upload(g)
    src = gg.sample_sources(g.n, 96, 124)
    cache = str(tmp_path / "tune.json")
    nk.nk_autotune(rp, ci, ivec(src[:32]), cache)
    # a distinctive entry: 256-thread workgroups, the multi-source kernel with 8 sources per task
    _retune_cache(cache, block=256, batch=8, bu_ratio=0.0)
    nk.nk_set_tuning(flags=4)
    try:
        nk.nk_set_tuning_cache(cache)
        got = nk.nk_bc_sources(rp, ci, ivec(src), 2.0).cpu().numpy()
        st = nk.nk_last_stats()
        assert st["block"] == 256 and st["sources_per_task"] == 8 and st["bitmap_lds"] == 4 and st["levels_bu"] == 0
        assert_scores_close(got, oracle.bc_sources(g.rowptr, g.colidx, src, 2.0, nthreads=8), "cached tuning")
        # another shape: the global tuning
        other = gg.erdos_renyi(3000, 6000, 125)
        orp, oci = upload(other)
        nk.nk_bc_sources(orp, oci, ivec([1, 2, 3]), 1.0)
        assert nk.nk_last_stats()["sources_per_task"] == 1
        # the batched plan: its large graph has the cached shape
        vtx = np.array([0, other.n, other.n + g.n], dtype=np.int64)
        arc = np.array([0, other.m, other.m + g.m], dtype=np.int64)
        brp = torch.from_numpy(np.concatenate([other.rowptr, g.rowptr]).astype(np.int32)).cuda()
        bci = torch.from_numpy(np.concatenate([other.colidx, g.colidx]).astype(np.int32)).cuda()
        with nk.NkBatchPlan(vtx, arc, brp, bci) as plan:
            out = plan.run().cpu().numpy()
            st = nk.nk_last_stats()
            assert st["sources_per_task"] == 8 and st["block"] == 256
        assert_scores_close(out[other.n:], oracle.bc_exact(g.rowptr, g.colidx, nthreads=16), "batched, cached")
        assert_scores_close(out[:other.n], oracle.bc_exact(other.rowptr, other.colidx), "batched, other")
        # the server: a graph added while the cache is registered
        with nk.NkServer(16 << 30, slots=2) as sv:
            gid = sv.add_graph(rp, ci)
            t = sv.submit(gid, sources=src)
            scores, _ = sv.wait(t)
        assert_scores_close(scores, oracle.bc_sources(g.rowptr, g.colidx, src, g.n / len(src), nthreads=8), "server")
        nk.nk_set_tuning_cache(None)
        nk.nk_bc_sources(rp, ci, ivec(src), 2.0)
        assert nk.nk_last_stats()["sources_per_task"] == 1
    finally:
        nk.nk_set_tuning_cache(None)
        nk.nk_set_tuning()
