"""Pair sampling probes the level that may end a search: only the meeting
vertices are written when it does, and the full level runs otherwise (also
whenever the deepest level's path counts sum to 2^64 or more, so that an
overflowing count is still caught).  Layered graphs -- complete bipartite
joins between consecutive layers of 16 vertices, path counts multiplying
by 16 per layer -- take samples through every case: searches that meet on
the first level, deep searches whose level sums pass 2^64 (the full level
runs and the counts stay exact, or overflow and are reported), and meeting
products past 2^64.  Each sample runs alone and is compared with the CPU
oracle: the same pair and interior vertices, or an overflow on both."""
import numpy as np
import pytest

import graphgen as gg
import oracle
import paper_1403_3005_amd as nk
from nkutil import upload

pytestmark = pytest.mark.gpu


def layered(layers: int, width: int = 16) -> gg.Graph:
    us, vs = [], []
    for i in range(layers - 1):
        for a in range(width):
            for b in range(width):
                us.append(i * width + a)
                vs.append((i + 1) * width + b)
    return gg.from_edges(layers * width, us, vs, f"layered{layers}x{width}")


@pytest.fixture(autouse=True)
def _default_tuning():
    nk.nk_set_tuning()
    yield
    nk.nk_set_tuning()


@pytest.mark.parametrize("layers", [6, 17, 24, 40])
def test_layered_samples_one_by_one(layers):
    g = layered(layers)
    rp, ci = upload(g)
    over = 0
    for j in range(48):
        try:
            ref = oracle.sample_path(g.rowptr, g.colidx, 9, j)
        except oracle.OracleError as e:
            assert e.code == oracle.E_SIGMA_OVERFLOW
            ref = None
        if ref is None:
            over += 1
            with pytest.raises(nk.NkError) as e:
                nk.nk_sample_paths(rp, ci, 9, j, 1, 64)
            assert e.value.code == nk.NK_E_SIGMA_OVERFLOW, j
            continue
        u, v, interior = ref
        uv, ln, path = (t.cpu().numpy() for t in nk.nk_sample_paths(rp, ci, 9, j, 1, 64))
        assert (int(uv[0, 0]), int(uv[0, 1])) == (u, v), j
        assert interior is not None
        assert int(ln[0]) == len(interior), j
        assert path[0, :len(interior)].tolist() == interior, j
    # the short graphs never overflow; the long ones do for far pairs
    assert (over == 0) == (layers <= 17)


def test_layered_counts_match_oracle():
    # every sample of the 17-layer graph fits (at most 16^15 paths)
    g = layered(17)
    rp, ci = upload(g)
    got = nk.nk_pair_counts(rp, ci, 600, 4).cpu().numpy()
    ref = oracle.pair_counts(g.rowptr, g.colidx, 600, 4, nthreads=8)
    assert np.array_equal(got, ref)


def chain_fan_hub() -> gg.Graph:
    """63 diamonds in series (2^63 paths end to end), 64 leaves on the last
    joint, one more vertex on each leaf, the first of those joined to a hub
    with 1000 pendant vertices.  A pair (early chain vertex, pendant) grows
    the chain side all the way: its level of leaves holds 64 counts of up
    to 2^63 each (a sum past 2^64, no count past it), so the next levels
    run in full, and the sample still succeeds."""
    k = 63
    us, vs = [], []
    for i in range(k):
        a, x, y, b = 3 * i, 3 * i + 1, 3 * i + 2, 3 * i + 3
        us += [a, a, x, y]
        vs += [x, y, b, b]
    end = 3 * k
    leaf0, far0, hub = end + 1, end + 65, end + 129
    for i in range(64):
        us += [end, leaf0 + i]
        vs += [leaf0 + i, far0 + i]
    us.append(far0)
    vs.append(hub)
    for i in range(1000):
        us.append(hub)
        vs.append(hub + 1 + i)
    return gg.from_edges(hub + 1001, us, vs, "chain-fan-hub")


def test_level_sums_past_2_64_run_in_full():
    g = chain_fan_hub()
    rp, ci = upload(g)
    count = 3000
    uv, ln, path = (t.cpu().numpy() for t in nk.nk_sample_paths(rp, ci, 12, 0, count, 64))
    deep = 0
    for j in range(count):
        u, v, interior = oracle.sample_path(g.rowptr, g.colidx, 12, j)
        assert (int(uv[j, 0]), int(uv[j, 1])) == (u, v), j
        assert int(ln[j]) == (len(interior) if len(interior) <= 64 else -2), j
        k = min(len(interior), 64)
        assert path[j, :k].tolist() == interior[:k], j
        if min(u, v) <= 12 and max(u, v) > 3 * 63 + 129:
            deep += 1
    assert deep >= 5
    got = nk.nk_pair_counts(rp, ci, count, 12).cpu().numpy()
    ref = oracle.pair_counts(g.rowptr, g.colidx, count, 12, nthreads=8)
    assert np.array_equal(got, ref)
