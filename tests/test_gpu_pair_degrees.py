"""Pair sampling keeps each vertex's degree in its per-vertex record, filled
once per record block and refreshed on the device when a later call brings
other row pointers.  These tests alternate graphs that share the record
layout (same vertex count, or vertex counts of the same padded stride),
including a graph written over the previous one's row-pointer buffer in
place, and check every call's samples and counts against the CPU oracle:
a block that kept stale degrees would choose other search sides and grow
other levels, which changes paths and counts."""
import numpy as np
import pytest

import graphgen as gg
import oracle
import paper_1403_3005_amd as nk
from nkutil import upload

pytestmark = pytest.mark.gpu

DIRECT = 32    # tuning flag bit 5: one record per vertex


@pytest.fixture(autouse=True)
def _default_tuning():
    nk.nk_set_tuning(flags=DIRECT)
    yield
    nk.nk_set_tuning()


def _check(g, rp, ci, seed, count=60, r=400):
    uv, ln, path = (t.cpu().numpy() for t in nk.nk_sample_paths(rp, ci, seed, 0, count, 64))
    for j in range(count):
        u, v, interior = oracle.sample_path(g.rowptr, g.colidx, seed, j)
        assert (int(uv[j, 0]), int(uv[j, 1])) == (u, v), j
        if interior is None:
            assert int(ln[j]) == -1, j
        else:
            assert int(ln[j]) == (len(interior) if len(interior) <= 64 else -2), j
            k = min(len(interior), 64)
            assert path[j, :k].tolist() == interior[:k], j
    got = nk.nk_pair_counts(rp, ci, r, seed).cpu().numpy()
    ref = oracle.pair_counts(g.rowptr, g.colidx, r, seed, nthreads=8)
    assert np.array_equal(got, ref)


def test_graphs_of_one_layout_in_turn():
    # 5000 and 4995 vertices pad to the same record stride
    a = gg.chung_lu(5000, 2.3, 8.0, 11)
    b = gg.erdos_renyi(5000, 30_000, 12)
    c = gg.barabasi_albert(4995, 3, 13)
    for g in (a, b, a, c, b, c):
        rp, ci = upload(g)
        _check(g, rp, ci, 21)


def test_row_pointers_rewritten_in_place():
    a = gg.erdos_renyi(6000, 24_000, 31)
    b = gg.chung_lu(6000, 2.2, 6.0, 32)
    rp, ci = upload(a)
    _check(a, rp, ci, 5)
    # the same device buffer now holds the other graph's row pointers
    rpb, cib = upload(b)
    rp.copy_(rpb)
    _check(b, rp, cib, 5)
    rp.copy_(upload(a)[0])
    _check(a, rp, ci, 5)


def test_after_hash_tables():
    # tables (flag bit 6) and record blocks never share a pooled block
    g = gg.erdos_renyi(300_000, 1_200_000, 41)
    h = gg.erdos_renyi(300_000, 900_000, 42)
    rpg, cig = upload(g)
    rph, cih = upload(h)
    nk.nk_set_tuning(flags=64)
    a = [t.cpu().numpy() for t in nk.nk_sample_paths(rpg, cig, 3, 0, 200, 64)]
    nk.nk_set_tuning(flags=DIRECT)
    b = [t.cpu().numpy() for t in nk.nk_sample_paths(rph, cih, 3, 0, 200, 64)]
    c = [t.cpu().numpy() for t in nk.nk_sample_paths(rpg, cig, 3, 0, 200, 64)]
    for x, y in zip(a, c):
        assert np.array_equal(x, y)
    for j in range(30):
        u, v, interior = oracle.sample_path(h.rowptr, h.colidx, 3, j)
        assert (int(b[0][j, 0]), int(b[0][j, 1])) == (u, v), j
        if interior is not None and len(interior) <= 64:
            assert b[2][j, :len(interior)].tolist() == interior, j
