"""Calls of different kinds back to back on one device, each checked
against the oracle: pooled scratch passes from one kind to the next with
whatever the previous call left in it (DAG-arc bits, cutoff vectors, pair
records, push accumulators), so a kernel that read state it did not write
would show here."""
import numpy as np
import pytest
import torch

import graphgen as gg
import oracle
import paper_1403_3005_amd as nk
from nkutil import assert_scores_close, ivec, upload

pytestmark = pytest.mark.gpu


def _dev(a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.int32)).to("cuda:0")


def test_mixed_call_sequence():
    nk.nk_set_tuning()
    a = gg.rmat(12, 8, 60)
    b = gg.barabasi_albert(5000, 3, 61)
    d = gg.directed_rmat(12, 8, 62)
    wa = gg.edge_weights(a, 20, 63)
    ra, ca = upload(a)
    rb, cb = upload(b)
    rd, cd = upload(d)
    sa = gg.sample_sources(a.n, 90, 64)
    sb = gg.sample_sources(b.n, 90, 65)
    refs = {
        "weighted": oracle.bc_weighted(a.rowptr, a.colidx, wa, sa, 1.0, nthreads=8),
        "bisect": oracle.bc_sources_bisect(a.rowptr, a.colidx, sa, 1.0, nthreads=8),
        "edge": oracle.edge_bc(b.rowptr, b.colidx, sb, 1.0, nthreads=8),
        "directed": oracle.bc_directed(d.rowptr, d.colidx, sa % d.n, 1.0, nthreads=8),
        "plain": oracle.bc_sources(b.rowptr, b.colidx, sb, 1.0, nthreads=8),
        "pairs": oracle.pair_sample(a.rowptr, a.colidx, 0.05, 0.1, 66),
    }
    trd, tcd = nk.nk_transpose(rd, cd)
    for rnd in range(2):
        for kind in ("weighted", "pairs", "bisect", "edge", "directed", "weighted", "plain", "bisect"):
            if kind == "weighted":
                got = nk.nk_bc_weighted(ra, ca, _dev(wa), ivec(sa)).cpu().numpy()
                assert_scores_close(got, refs[kind], f"{kind} round {rnd}")
            elif kind == "bisect":
                got = nk.nk_bc_sources_bisect(ra, ca, ivec(sa), 1.0).cpu().numpy()
                assert_scores_close(got, refs[kind], f"{kind} round {rnd}")
            elif kind == "edge":
                ebc, bc = nk.nk_edge_bc(rb, cb, ivec(sb), 1.0)
                assert_scores_close(ebc.cpu().numpy(), refs[kind][0], f"{kind} edges round {rnd}")
                assert_scores_close(bc.cpu().numpy(), refs[kind][1], f"{kind} vertices round {rnd}")
            elif kind == "directed":
                got = nk.nk_bc_directed(rd, cd, ivec(sa % d.n), 1.0, trd, tcd).cpu().numpy()
                assert_scores_close(got, refs[kind], f"{kind} round {rnd}")
            elif kind == "plain":
                got = nk.nk_bc_sources(rb, cb, ivec(sb), 1.0).cpu().numpy()
                assert_scores_close(got, refs[kind], f"{kind} round {rnd}")
            else:
                bc, cnt, r, vd = nk.nk_bc_pair_sample(ra, ca, 0.05, 0.1, 66)
                obc, ocnt, orr, ovd = refs[kind]
                assert (r, vd) == (orr, ovd)
                assert np.array_equal(cnt.cpu().numpy().view(np.uint32), ocnt)
                assert_scores_close(bc.cpu().numpy(), obc, f"pairs round {rnd}")
