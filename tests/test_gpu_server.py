"""Serving: results through the server equal the CPU oracle's (and the
direct calls'), each request gives the same result alone and inside a
concurrent mix, admission respects the HBM budget, and graphs can be added
while requests run."""
import numpy as np
import pytest

import graphgen as gg
import oracle
import paper_1403_3005_amd as nk
from paper_1403_3005_amd.serving import replay
from nkutil import assert_scores_close, ivec, upload

pytestmark = pytest.mark.gpu

GIB = 1 << 30


def _pool():
    return [gg.rmat(13, 16, 501), gg.barabasi_albert(20000, 4, 502), gg.rmat(15, 16, 503), gg.erdos_renyi(3000, 9000, 504)]


def _oracle_request(g, rq):
    """The oracle's answer to one request: scores of the k listed sources
    scaled by n/k, or pair-sampling scores (counts / r * n(n-1))."""
    if "sources" in rq:
        k = len(rq["sources"])
        return oracle.bc_sources(g.rowptr, g.colidx, rq["sources"], g.n / k, nthreads=16), None
    est, cnt, r, vd = oracle.pair_sample(g.rowptr, g.colidx, rq["eps"], rq["delta"], rq["seed"])
    return est, (cnt, r)


def test_server_matches_oracle():
    """Every request of a mixed stream over the pool against the CPU oracle:
    source requests within the score tolerance, pair requests with counts
    identical to the oracle's (recovered from the scores and the oracle's r)."""
    pool = _pool()
    with nk.NkServer(64 * GIB, slots=4) as sv:
        ids = [sv.add_graph(*upload(g)) for g in pool]
        reqs = gg.request_stream(30, 1000.0, [g.n for g in pool], seed=19)
        assert {("sources" in rq) for rq in reqs} == {True, False}
        results, _ = replay(sv, ids, reqs)
        for rq, (scores, lat) in zip(reqs, results):
            g = pool[rq["graph"]]
            ref, pair = _oracle_request(g, rq)
            if pair is None:
                assert_scores_close(scores, ref, f"request {rq['id']} vs oracle")
            else:
                cnt, r = pair
                scale = g.n * (g.n - 1) / r
                assert np.array_equal(np.rint(scores / scale).astype(np.int64), cnt.astype(np.int64)), rq["id"]
                assert_scores_close(scores, ref, f"pair request {rq['id']} vs oracle")


def test_add_graph_while_requests_run():
    """Graphs added while requests are in flight: earlier requests finish
    with the oracle's scores and the new graphs serve requests too."""
    pool = _pool()
    with nk.NkServer(64 * GIB, slots=4) as sv:
        ids = [sv.add_graph(*upload(pool[0]))]
        tickets = []
        for i in range(8):
            src = gg.sample_sources(pool[0].n, 256, 900 + i)
            tickets.append((0, src, sv.submit(ids[0], sources=src)))
            if i < 3:
                ids.append(sv.add_graph(*upload(pool[i + 1])))
        for gi in range(1, 4):
            src = gg.sample_sources(pool[gi].n, 64, 950 + gi)
            tickets.append((gi, src, sv.submit(ids[gi], sources=src)))
        for gi, src, t in tickets:
            scores, _ = sv.wait(t)
            g = pool[gi]
            ref = oracle.bc_sources(g.rowptr, g.colidx, src, g.n / len(src), nthreads=16)
            assert_scores_close(scores, ref, f"graph {gi}")


def test_server_matches_direct_calls():
    pool = _pool()
    with nk.NkServer(64 * GIB, slots=4) as sv:
        ids = [sv.add_graph(*upload(g)) for g in pool]
        reqs = gg.request_stream(20, 1000.0, [g.n for g in pool], seed=9)
        results, _ = replay(sv, ids, reqs)
        for rq, (scores, lat) in zip(reqs, results):
            g = pool[rq["graph"]]
            rp, ci = upload(g)
            if "sources" in rq:
                k = len(rq["sources"])
                ref = nk.nk_bc_sources(rp, ci, ivec(rq["sources"]), g.n / k).cpu().numpy()
                assert_scores_close(scores, ref, f"request {rq['id']}")
            else:
                ref, cnt, r, vd = nk.nk_bc_pair_sample(rp, ci, rq["eps"], rq["delta"], rq["seed"])
                assert np.array_equal(scores, ref.cpu().numpy()), rq["id"]
            assert lat > 0
        st = sv.stats()
        assert st["completed"] == 20 and st["failed"] == 0
        assert st["p99_ms"] >= st["p50_ms"] > 0


def test_alone_equals_mix():
    pool = _pool()
    with nk.NkServer(64 * GIB, slots=4) as sv:
        ids = [sv.add_graph(*upload(g)) for g in pool]
        reqs = gg.request_stream(24, 1e6, [g.n for g in pool], seed=11)  # all arrive at once
        alone = []
        for rq in reqs:
            res, _ = replay(sv, ids, [dict(rq, t=0.0)])
            alone.append(res[0][0])
        sv.reset_stats()
        mixed, _ = replay(sv, ids, reqs)
        assert sv.stats()["max_inflight"] > 1  # requests really overlapped
        for rq, a, (b, _) in zip(reqs, alone, mixed):
            if "sources" in rq:
                assert_scores_close(b, a, f"request {rq['id']}")
            else:
                assert np.array_equal(a, b)


def test_budget_admission():
    g = gg.rmat(14, 16, 601)
    rp, ci = upload(g)
    with nk.NkServer(1 << 20, slots=2) as sv:  # 1 MiB: the graph itself does not fit
        with pytest.raises(nk.NkError) as e:
            sv.add_graph(rp, ci)
        assert e.value.code == nk.NK_E_BUDGET
    # room for the graph (about 2 MiB) and one running request (its grid
    # shrinks until the per-workgroup scratch fits: about 46 MiB at 64
    # workgroups): requests run one at a time
    with nk.NkServer(80 << 20, slots=4) as sv:
        gid = sv.add_graph(rp, ci)
        reqs = [{"id": i, "t": 0.0, "graph": 0, "seed": i, "sources": gg.sample_sources(g.n, 128, 700 + i)}
                for i in range(6)]
        results, _ = replay(sv, [gid], reqs)
        for rq, (scores, _) in zip(reqs, results):
            ref = nk.nk_bc_sources(rp, ci, ivec(rq["sources"]), g.n / 128).cpu().numpy()
            assert_scores_close(scores, ref, "budgeted")
        assert sv.stats()["max_inflight"] == 1
    with nk.NkServer(2 << 20, slots=2) as sv:
        small = gg.path(100)
        gid = sv.add_graph(*upload(small))
        big = gg.rmat(15, 16, 602)
        with pytest.raises(nk.NkError):
            sv.add_graph(*upload(big))


def test_server_argument_errors():
    g = gg.cycle(50)
    with nk.NkServer(GIB, slots=1) as sv:
        gid = sv.add_graph(*upload(g))
        with pytest.raises(nk.NkError):
            sv.submit(gid + 5, sources=np.array([1], dtype=np.int32))
        with pytest.raises(nk.NkError):
            sv.submit(gid, eps=1.5)
        with pytest.raises(nk.NkError):
            sv.submit(gid, sources=np.array([60], dtype=np.int32))
        t = sv.submit(gid, sources=np.array([1, 2], dtype=np.int32))
        scores, _ = sv.wait(t)
        assert scores.shape == (50,)
