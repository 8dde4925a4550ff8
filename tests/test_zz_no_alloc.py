"""The allocation-free source-set entry point (nk_bc_sources_noalloc)
against nk_bc_sources, through the C ABI: two calls in a row on one device,
the second with a smaller input, so the second runs on the fixed scratch
the first left behind; the all-in-LDS path, the persistent kernel with its
per-workgroup state in the fixed scratch (bitmap in LDS and in HBM), and a
graph too large for it."""
import numpy as np
import pytest
import torch

import graphgen as gg
import oracle
import paper_1403_3005_amd as nk
from nkutil import assert_scores_close, ivec, upload

pytestmark = pytest.mark.gpu


def _both(g, src, scale):
    rp, ci = upload(g)
    sv = ivec(src)
    ref = nk.nk_bc_sources(rp, ci, sv, scale).cpu().numpy()
    bc = torch.full((g.n,), -1.0, dtype=torch.float64, device="cuda:0")
    got = nk.nk_bc_sources_noalloc(rp, ci, sv, scale, bc=bc).cpu().numpy()
    return got, ref, nk.nk_last_stats()


@pytest.mark.parametrize("flags", [0, 1])
def test_noalloc_matches_nk_bc_sources_twice(flags):
    """Persistent kernel (bitmap in LDS, or in the fixed scratch with flag
    bit 0): a large call, then a smaller one."""
    nk.nk_set_tuning(flags=flags)
    try:
        big = gg.rmat(16, 16, 71)
        src = gg.sample_sources(big.n, 700, 72)
        got, ref, st = _both(big, src, big.n / 700)
        assert st["bitmap_lds"] == (0 if flags else 1) and st["workgroups"] > 1 and st["sources"] == 700
        assert_scores_close(got, ref, "first call")
        assert_scores_close(got, oracle.bc_sources(big.rowptr, big.colidx, src, big.n / 700, nthreads=8),
                            "first call vs oracle")
        small = gg.barabasi_albert(30000, 3, 73)
        src2 = gg.sample_sources(small.n, 300, 74)
        got2, ref2, st2 = _both(small, src2, 2.0)
        assert st2["sources"] == 300
        assert_scores_close(got2, ref2, "second call")
    finally:
        nk.nk_set_tuning()


def test_noalloc_lds_path_and_degenerate_inputs():
    g = gg.erdos_renyi(1200, 4000, 75)
    got, ref, st = _both(g, np.arange(g.n, dtype=np.int32), 1.0)
    assert st["bitmap_lds"] == 2
    assert_scores_close(got, ref, "all-in-LDS")
    rp, ci = upload(g)
    zero = nk.nk_bc_sources_noalloc(rp, ci, torch.zeros(0, dtype=torch.int32, device="cuda:0"), 3.0).cpu().numpy()
    assert np.array_equal(zero, np.zeros(g.n))
    with pytest.raises(nk.NkError) as e:
        nk.nk_bc_sources_noalloc(rp, ci, ivec([0, g.n]), 1.0)
    assert e.value.code == nk.NK_E_INVALID_ARG
    # a valid call right after the error still matches
    got, ref, _ = _both(g, [5, 7, 5], 0.5)
    assert_scores_close(got, ref, "after error")


def test_noalloc_rejects_a_graph_beyond_its_scratch():
    """3.5e6 isolated vertices: one workgroup's state exceeds the fixed
    scratch; the call fails with NK_E_BUDGET before any launch."""
    n = 3_500_000
    rp = torch.zeros(n + 1, dtype=torch.int32, device="cuda:0")
    ci = torch.zeros(0, dtype=torch.int32, device="cuda:0")
    with pytest.raises(nk.NkError) as e:
        nk.nk_bc_sources_noalloc(rp, ci, ivec([0, 1]), 1.0)
    assert e.value.code == nk.NK_E_BUDGET
    assert "no-allocation scratch" in str(e.value)
