"""Parity at the workloads' full sizes, in the launch configuration bench.py
times, on outputs the oracle can compute one by one and on properties that
hold at any size."""
import numpy as np
import pytest
import torch

import graphgen as gg
import oracle
import paper_1403_3005_amd as nk
from nkutil import assert_scores_close, ivec, upload

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def rmat20():
    g, src = gg.workload_rmat20(2)
    rp, ci = upload(g)
    return g, src, rp, ci


def test_rmat20_sampled_sources_vs_oracle(rmat20):
    """Full R-MAT-20 graph: scores of the first 6 benchmark sources against
    the oracle, and d / sigma of 4 sources bit for bit."""
    g, src, rp, ci = rmat20
    nk.nk_set_tuning()
    few = src[:6]
    got = nk.nk_bc_sources(rp, ci, ivec(few), g.n / 4096).cpu().numpy()
    assert_scores_close(got, oracle.bc_sources(g.rowptr, g.colidx, few, g.n / 4096), "rmat20 6 sources")
    pick = [int(s) for s in src[:40] if g.rowptr[s + 1] > g.rowptr[s]][:4]
    d, s = nk.nk_sssp_counts(rp, ci, ivec(pick))
    for i, v in enumerate(pick):
        od, os_ = oracle.sssp_counts(g.rowptr, g.colidx, v)
        assert np.array_equal(d[i].cpu().numpy(), od)
        assert np.array_equal(s[i].cpu().numpy().view(np.uint64), os_)


def test_rmat20_strided_512_sources_vs_oracle(rmat20):
    """Every eighth benchmark source (512 of the 4096) in the benchmark's
    launch form (256 workgroups of 1024 threads, bottom-up and push levels
    on): twice as many sources as workgroups, so slots run further sources
    on state the previous one left, and two calls in a row; every score
    against the oracle."""
    g, src, rp, ci = rmat20
    nk.nk_set_tuning()
    part = np.ascontiguousarray(src[::8])
    ref = oracle.bc_sources(g.rowptr, g.colidx, part, g.n / 4096, nthreads=16)
    for call in range(2):
        got = nk.nk_bc_sources(rp, ci, ivec(part), g.n / 4096).cpu().numpy()
        st = nk.nk_last_stats()
        assert st["workgroups"] == 256 and st["block"] == 1024, st
        assert st["levels_bu"] > 0 and st["levels_bw_push"] > 0, st
        assert_scores_close(got, ref, f"rmat20 strided sources, call {call}")


def test_rmat20_all_4096_sources_sum_invariant(rmat20):
    """The benchmark call itself (4096 sources, scale n/4096): the scores sum
    to scale x sum over sources and reached t of (d(s,t) - 1), with d from
    the inspection call in chunks; the work counters match their own sums."""
    g, src, rp, ci = rmat20
    nk.nk_set_tuning()
    scale = g.n / 4096
    bc = nk.nk_bc_sources(rp, ci, ivec(src), scale)
    st = nk.nk_last_stats()
    total = float(bc.sum().item())
    acc = 0.0
    reached = 0
    for c0 in range(0, 4096, 256):
        d, _ = nk.nk_sssp_counts(rp, ci, ivec(src[c0:c0 + 256]))
        pos = d[d > 0].to(torch.float64)
        acc += float((pos - 1.0).sum().item())
        reached += int((d >= 0).sum().item())
        del d
    assert abs(total - scale * acc) <= 1e-9 * scale * acc
    assert st["reached"] == reached and st["sources"] == 4096
    assert bc.min().item() >= 0.0


@pytest.fixture(scope="module")
def chunglu4m():
    g = gg.workload_chung_lu4m(3)
    rp, ci = upload(g)
    return g, rp, ci


def test_chunglu4m_vd_bound_and_r(chunglu4m):
    g, rp, ci = chunglu4m
    info = nk.nk_vd_bound(rp, ci)
    assert info == oracle.vd_bound(g.rowptr, g.colidx)
    assert nk.nk_rk_sample_size(0.01, 0.1, info["vd_ub"]) == oracle.rk_sample_size(0.01, 0.1, info["vd_ub"])


def test_chunglu4m_sampled_pairs_bit_exact(chunglu4m):
    """The first samples of the benchmark's sequence (seed 3): pairs, paths
    and counts identical to the oracle's."""
    g, rp, ci = chunglu4m
    uv, ln, path = nk.nk_sample_paths(rp, ci, 3, 0, 6, 64)
    for j in range(6):
        u, v, interior = oracle.sample_path(g.rowptr, g.colidx, 3, j)
        assert (int(uv[j, 0]), int(uv[j, 1])) == (u, v)
        if interior is None:
            assert int(ln[j]) == -1
        else:
            assert int(ln[j]) == len(interior)
            assert path[j, :len(interior)].cpu().tolist() == interior
    got = nk.nk_pair_counts(rp, ci, 10, 3).cpu().numpy().view(np.uint32)
    assert np.array_equal(got, oracle.pair_counts(g.rowptr, g.colidx, 10, 3))


def test_chunglu4m_full_sample_bit_exact(chunglu4m):
    """The benchmark call itself (eps 0.01, delta 0.1, seed 3: r = 31,513
    samples on 512 slots of 256 threads with one record per vertex), twice,
    so the second call runs on the per-vertex records the first left (reused
    without a fill); then with hashed records per slot (the samples that
    could outgrow them rerun with one record per vertex): all counts
    identical to the oracle's over the whole sample."""
    g, rp, ci = chunglu4m
    nk.nk_set_tuning()
    _, cnt0, r, vd = nk.nk_bc_pair_sample(rp, ci, 0.01, 0.1, 3)
    assert r == oracle.rk_sample_size(0.01, 0.1, vd)
    ref = oracle.pair_counts(g.rowptr, g.colidx, r, 3, nthreads=16)
    assert np.array_equal(cnt0.cpu().numpy().view(np.uint32), ref)
    _, cnt1, r1, _ = nk.nk_bc_pair_sample(rp, ci, 0.01, 0.1, 3)
    assert r1 == r and np.array_equal(cnt1.cpu().numpy().view(np.uint32), ref)
    nk.nk_set_tuning(flags=64)
    try:
        _, cnt2, r2, _ = nk.nk_bc_pair_sample(rp, ci, 0.01, 0.1, 3)
    finally:
        nk.nk_set_tuning()
    assert r2 == r and np.array_equal(cnt2.cpu().numpy().view(np.uint32), ref)


def test_batched_with_50k_vertex_graphs():
    """A batch holding an ER and a BA graph of 5e4 vertices (mean degree 8,
    the batched workload's generators) beside small graphs, in one call:
    every score of every graph against the oracle."""
    graphs = [gg.erdos_renyi(50_000, 200_000, 811), gg.barabasi_albert(50_000, 4, 812),
              gg.erdos_renyi(1500, 6000, 813), gg.barabasi_albert(4000, 4, 814), gg.erdos_renyi(9000, 36000, 815)]
    vtx = np.zeros(len(graphs) + 1, dtype=np.int64)
    arc = np.zeros(len(graphs) + 1, dtype=np.int64)
    for i, g in enumerate(graphs):
        vtx[i + 1] = vtx[i] + g.n
        arc[i + 1] = arc[i] + g.m
    rp = torch.from_numpy(np.concatenate([g.rowptr for g in graphs]).astype(np.int32)).cuda()
    ci = torch.from_numpy(np.concatenate([g.colidx for g in graphs]).astype(np.int32)).cuda()
    nk.nk_set_tuning()
    got = nk.nk_bc_exact_batched(vtx, arc, rp, ci).cpu().numpy()
    assert nk.nk_last_stats()["sources"] == int(vtx[-1])
    for i, g in enumerate(graphs):
        assert_scores_close(got[vtx[i]:vtx[i + 1]], oracle.bc_exact(g.rowptr, g.colidx, nthreads=16), f"graph {i}")


def test_batched_c4_sized_graphs():
    """Graphs drawn from the batched workload's size distribution (n up to
    2e4 here so the oracle runs them all) in one launch."""
    sizes = [n for n in gg.batched_sizes(512, 1000, 200_000, 4) if n <= 20_000][:10]
    graphs = []
    for i, n in enumerate(sizes):
        gs = gg.draw(4, 61, i, 0)
        graphs.append(gg.erdos_renyi(n, 4 * n, gs) if i % 2 == 0 else gg.barabasi_albert(n, 4, gs))
    vtx = np.zeros(len(graphs) + 1, dtype=np.int64)
    arc = np.zeros(len(graphs) + 1, dtype=np.int64)
    for i, g in enumerate(graphs):
        vtx[i + 1] = vtx[i] + g.n
        arc[i + 1] = arc[i] + g.m
    rp = torch.from_numpy(np.concatenate([g.rowptr for g in graphs])).cuda()
    ci = torch.from_numpy(np.concatenate([g.colidx for g in graphs])).cuda()
    got = nk.nk_bc_exact_batched(vtx, arc, rp, ci).cpu().numpy()
    for i, g in enumerate(graphs):
        assert_scores_close(got[vtx[i]:vtx[i + 1]], oracle.bc_exact(g.rowptr, g.colidx, nthreads=8), f"graph {i}")


def test_rmat20_directed_sampled_vs_oracle():
    """The directed benchmark graph (R-MAT-20 draws as arcs, 16.1M arcs) with
    its device-built in-arc CSR, in the benchmark's launch form: the first 6
    benchmark sources against the oracle."""
    g = gg.directed_rmat(20, 16, 2)
    src = gg.sample_sources(g.n, 4096, 2)
    rp, ci = upload(g)
    trp, tci = nk.nk_transpose(rp, ci)
    nk.nk_set_tuning()
    few = src[:6]
    got = nk.nk_bc_directed(rp, ci, ivec(few), g.n / 4096, trp, tci).cpu().numpy()
    assert_scores_close(got, oracle.bc_directed(g.rowptr, g.colidx, few, g.n / 4096, nthreads=6), "drmat20")


def test_rmat20_weighted_sampled_vs_oracle(rmat20):
    """The weighted benchmark workload (R-MAT-20, edge weights 1..64): the
    first 6 benchmark sources against the oracle's Dijkstra Brandes."""
    g, src, rp, ci = rmat20
    w = gg.edge_weights(g, 64, 2)
    wt = torch.from_numpy(w).to("cuda:0")
    nk.nk_set_tuning()
    few = src[:6]
    got = nk.nk_bc_weighted(rp, ci, wt, ivec(few), g.n / 4096).cpu().numpy()
    assert_scores_close(got, oracle.bc_weighted(g.rowptr, g.colidx, w, few, g.n / 4096, nthreads=6), "wrmat20")


def test_batched512_first_launch_group_at_full_size():
    """The batched workload's first launch group exactly as the benchmark
    builds and runs it (64 graphs of the 512, one call): the graphs the
    oracle finishes quickly against it, the largest graph by the identity
    sum of scores = sum over sources s and reached t != s of (d(s, t) - 1)
    with distances from the inspection call (bit-exact against the oracle
    elsewhere), every score non-negative."""
    sizes = gg.batched_sizes(512, 1000, 200_000, 4)[:64]
    graphs = []
    for i, n in enumerate(sizes):
        gs = gg.draw(4, 61, i, 0)
        graphs.append(gg.erdos_renyi(n, 4 * n, gs) if i % 2 == 0 else gg.barabasi_albert(n, 4, gs))
    vtx = np.zeros(len(graphs) + 1, dtype=np.int64)
    arc = np.zeros(len(graphs) + 1, dtype=np.int64)
    for i, g in enumerate(graphs):
        vtx[i + 1] = vtx[i] + g.n
        arc[i + 1] = arc[i] + g.m
    rp = torch.from_numpy(np.concatenate([g.rowptr for g in graphs]).astype(np.int32)).cuda()
    ci = torch.from_numpy(np.concatenate([g.colidx for g in graphs]).astype(np.int32)).cuda()
    nk.nk_set_tuning()
    got = nk.nk_bc_exact_batched(vtx, arc, rp, ci).cpu().numpy()
    assert nk.nk_last_stats()["sources"] == int(vtx[-1])
    assert got.min() >= 0.0
    small = [i for i, g in enumerate(graphs) if g.n <= 2500]
    assert small
    for i in small:
        g = graphs[i]
        assert_scores_close(got[vtx[i]:vtx[i + 1]], oracle.bc_exact(g.rowptr, g.colidx, nthreads=8), f"graph {i}")
    big = max(range(len(graphs)), key=lambda i: graphs[i].n)
    g = graphs[big]
    grp, gci = upload(g)
    acc = 0.0
    for c0 in range(0, g.n, 512):
        src = np.arange(c0, min(g.n, c0 + 512), dtype=np.int32)
        d, _ = nk.nk_sssp_counts(grp, gci, ivec(src))
        pos = d[d > 0].to(torch.float64)
        acc += float((pos - 1.0).sum().item())
        del d
    total = float(got[vtx[big]:vtx[big + 1]].sum())
    assert abs(total - acc) <= 1e-9 * acc, (g.n, total, acc)
