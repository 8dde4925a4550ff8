"""The batched exact run captured once into a HIP graph and replayed: every
replay, with the program's own eager work and synchronisations between
replays, equals the eager batched call within the score tolerance."""
import numpy as np
import pytest
import torch

import graphgen as gg
import oracle
import paper_1403_3005_amd as nk
from nkutil import assert_scores_close, upload

pytestmark = pytest.mark.gpu


def _batch(graphs):
    vtx = np.zeros(len(graphs) + 1, dtype=np.int64)
    arc = np.zeros(len(graphs) + 1, dtype=np.int64)
    for i, g in enumerate(graphs):
        vtx[i + 1] = vtx[i] + g.n
        arc[i + 1] = arc[i] + g.m
    rp = torch.from_numpy(np.concatenate([g.rowptr for g in graphs]).astype(np.int32)).cuda()
    ci = torch.from_numpy(np.concatenate([g.colidx for g in graphs]).astype(np.int32)).cuda()
    return vtx, arc, rp, ci


def _graphs():
    return [gg.erdos_renyi(900, 3600, 141), gg.barabasi_albert(9000, 4, 142), gg.path(3),
            gg.erdos_renyi(12000, 48000, 143), gg.star(700),
            gg.Graph(1, np.zeros(2, dtype=np.int32), np.zeros(0, dtype=np.int32)), gg.barabasi_albert(500, 4, 144)]


def test_batch_plan_replays_match_eager():
    nk.nk_set_tuning()
    graphs = _graphs()
    vtx, arc, rp, ci = _batch(graphs)
    eager = nk.nk_bc_exact_batched(vtx, arc, rp, ci).cpu().numpy()
    for i, g in enumerate(graphs):
        assert_scores_close(eager[vtx[i]:vtx[i + 1]], oracle.bc_exact(g.rowptr, g.colidx, nthreads=8), f"graph {i}")
    other = gg.rmat(12, 8, 145)
    orp, oci = upload(other)
    ref_other = nk.nk_bc_exact(orp, oci).cpu().numpy()
    with nk.NkBatchPlan(vtx, arc, rp, ci) as plan:
        for r in range(4):
            got = plan.run().cpu().numpy()
            st = nk.nk_last_stats()
            assert st["sources"] == int(vtx[-1]) and st["bitmap_lds"] == 3
            assert_scores_close(got, eager, f"replay {r}")
            # eager work between replays: another library call on the same
            # device (it reuses pooled scratch), torch kernels, a sync
            assert_scores_close(nk.nk_bc_exact(orp, oci).cpu().numpy(), ref_other, f"eager call after replay {r}")
            x = torch.arange(100000, device="cuda:0", dtype=torch.float64)
            assert float(x.sum().item()) == 4999950000.0
            torch.cuda.synchronize()


def test_batch_plan_reads_current_graph_contents_and_reports_errors():
    graphs = [gg.erdos_renyi(2000, 8000, 146), gg.barabasi_albert(6000, 3, 147)]
    vtx, arc, rp, ci = _batch(graphs)
    with nk.NkBatchPlan(vtx, arc, rp, ci) as plan:
        good = plan.run().cpu().numpy()
        saved = ci[5].item()
        ci[5] = 2000  # out of range for graph 0
        with pytest.raises(nk.NkError) as e:
            plan.run()
        assert e.value.code == nk.NK_E_INVALID_GRAPH
        ci[5] = saved
        assert_scores_close(plan.run().cpu().numpy(), good, "after the repaired graph")
    eager = nk.nk_bc_exact_batched(vtx, arc, rp, ci).cpu().numpy()
    assert_scores_close(good, eager, "plan vs eager")


def test_batch_plan_empty_and_bad_arguments():
    vtx = np.zeros(3, dtype=np.int64)
    arc = np.zeros(3, dtype=np.int64)
    rp = torch.zeros(2, dtype=torch.int32, device="cuda:0")
    ci = torch.zeros(0, dtype=torch.int32, device="cuda:0")
    with nk.NkBatchPlan(vtx, arc, rp, ci) as plan:
        assert plan.run().numel() == 0
    with pytest.raises(nk.NkError):
        nk.NkBatchPlan(np.array([1, 2], dtype=np.int64), np.array([0, 0], dtype=np.int64), rp, ci)


def test_batch_plan_launch_progress_finish():
    """The run in halves on a stream of its own: progress is read while the
    run goes on (never decreasing, never above the total), reaches every
    source once the launch has completed, and finish returns the eager
    scores; a second launch before finishing is refused."""
    nk.nk_set_tuning()
    graphs = _graphs() + [gg.erdos_renyi(60000, 240000, 148)]
    vtx, arc, rp, ci = _batch(graphs)
    eager = nk.nk_bc_exact_batched(vtx, arc, rp, ci).cpu().numpy()
    stream = torch.cuda.Stream()
    with nk.NkBatchPlan(vtx, arc, rp, ci) as plan:
        for r in range(2):
            plan.launch(stream)
            with pytest.raises(nk.NkError):
                plan.launch(stream)
            seen = []
            for _ in range(200000):
                done, total, finished = plan.progress()
                assert total == int(vtx[-1]) and 0 <= done <= total
                seen.append(done)
                if finished:
                    break
            assert finished and seen == sorted(seen)
            done, total, _ = plan.progress()
            assert done == total
            got = plan.finish(stream).cpu().numpy()
            assert nk.nk_last_stats()["sources"] == total
            assert_scores_close(got, eager, f"launched run {r}")
        with pytest.raises(nk.NkError):
            plan.finish(stream)
