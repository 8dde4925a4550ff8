"""Pair sampling with hashed per-slot records (tuning flag bit 6; used by
itself only where records per vertex would leave too few slots): sample
pairs, paths and counts bit-identical to the records-per-vertex kernel
(flag bit 5) and to the CPU oracle, including samples that could outgrow the
table and run again with one record per vertex."""
import numpy as np
import pytest

import graphgen as gg
import oracle
import paper_1403_3005_amd as nk
from nkutil import upload

pytestmark = pytest.mark.gpu

DIRECT = 32    # tuning flag bit 5: one record per vertex
HASHED = 64    # bit 6: hashed records


@pytest.fixture(autouse=True)
def _default_tuning():
    nk.nk_set_tuning()
    yield
    nk.nk_set_tuning()


def _paths(rp, ci, seed, count, flags):
    nk.nk_set_tuning(flags=flags)
    uv, ln, path = nk.nk_sample_paths(rp, ci, seed, 0, count, 64)
    st = nk.nk_last_stats()
    return uv.cpu().numpy(), ln.cpu().numpy(), path.cpu().numpy(), st


def _check_against_oracle(g, seed, uv, ln, path, count):
    for j in range(count):
        u, v, interior = oracle.sample_path(g.rowptr, g.colidx, seed, j)
        assert (int(uv[j, 0]), int(uv[j, 1])) == (u, v), j
        if interior is None:
            assert int(ln[j]) == -1, j
        else:
            # a path longer than the 64 output entries reports -2 and its
            # first 64 interior vertices
            assert int(ln[j]) == (len(interior) if len(interior) <= 64 else -2), j
            k = min(len(interior), 64)
            assert path[j, :k].tolist() == interior[:k], j


def test_hashed_records_match_direct_and_oracle():
    g = gg.erdos_renyi(300_000, 1_200_000, 201)
    rp, ci = upload(g)
    h = _paths(rp, ci, 7, 300, HASHED)
    d = _paths(rp, ci, 7, 300, DIRECT)
    assert h[3]["pair_deferred"] == 0 and d[3]["pair_deferred"] == 0
    for a, b in zip(h[:3], d[:3]):
        assert np.array_equal(a, b)
    _check_against_oracle(g, 7, *h[:3], 40)
    # counts over a larger sample, both record layouts, twice (the second
    # call reuses the tables the first left free)
    ref = oracle.pair_counts(g.rowptr, g.colidx, 3000, 7, nthreads=16)
    for flags in (HASHED, HASHED, DIRECT, 0):
        nk.nk_set_tuning(flags=flags)
        got = nk.nk_pair_counts(rp, ci, 3000, 7).cpu().numpy().view(np.uint32)
        assert np.array_equal(got, ref), flags


def test_samples_that_outgrow_the_table():
    """A 2.8 * 10^5-vertex preferential-attachment graph plus a 40,000-cycle:
    pairs on the cycle (searches of up to 20,000 levels) and pairs across
    the two components (the cycle side explores all of it) list more than
    half a table and run again with one record per vertex; results do not
    depend on which launch ran a sample."""
    g = gg.disjoint_union([gg.barabasi_albert(280_000, 3, 202), gg.cycle(40_000)])
    rp, ci = upload(g)
    h = _paths(rp, ci, 11, 48, HASHED)
    d = _paths(rp, ci, 11, 48, DIRECT)
    assert h[3]["pair_deferred"] > 0 and d[3]["pair_deferred"] == 0
    assert h[3]["sources"] == 48
    for a, b in zip(h[:3], d[:3]):
        assert np.array_equal(a, b)
    _check_against_oracle(g, 11, *h[:3], 48)
    ref = oracle.pair_counts(g.rowptr, g.colidx, 48, 11)
    nk.nk_set_tuning(flags=HASHED)
    got = nk.nk_pair_counts(rp, ci, 48, 11).cpu().numpy().view(np.uint32)
    assert np.array_equal(got, ref)
