"""GPU parity of exact and Eppstein-Wang sampled closeness against the
oracle, through the C ABI."""
import numpy as np
import pytest
import torch

import graphgen as gg
import oracle
import paper_1403_3005_amd as nk
from nkutil import ivec, upload

pytestmark = pytest.mark.gpu

RTOL = 1e-14   # both sides reduce exact integer distance sums, then a few FP64 operations


@pytest.fixture(autouse=True)
def _default_tuning():
    nk.nk_set_tuning()
    yield
    nk.nk_set_tuning()


GRAPHS = [
    lambda: gg.path(500), lambda: gg.star(3000), lambda: gg.grid(30, 41), lambda: gg.complete(40),
    lambda: gg.erdos_renyi(3000, 2500, 91),                              # many components
    lambda: gg.barabasi_albert(5000, 3, 92), lambda: gg.rmat(13, 16, 93),
    lambda: gg.disjoint_union([gg.cycle(9), gg.path(1), gg.star(40), gg.complete(6)]),
]


@pytest.mark.parametrize("make", GRAPHS)
@pytest.mark.parametrize("block", [256, 1024])
def test_closeness_exact(make, block):
    nk.nk_set_tuning(block=block)
    g = make()
    rp, ci = upload(g)
    got = nk.nk_closeness(rp, ci).cpu().numpy()
    ref = oracle.closeness(g.rowptr, g.colidx)
    assert np.allclose(got, ref, rtol=RTOL, atol=0.0), g.name


@pytest.mark.parametrize("make", GRAPHS)
@pytest.mark.parametrize("bu_ratio", [0.0, 16.0, 1e9])
def test_closeness_sampled(make, bu_ratio):
    nk.nk_set_tuning(bu_ratio=bu_ratio)
    g = make()
    rp, ci = upload(g)
    k = min(g.n, 61)
    src = gg.sample_sources(g.n, k, 94)
    got = nk.nk_closeness_sampled(rp, ci, ivec(src)).cpu().numpy()
    ref, _ = oracle.closeness_approx(g.rowptr, g.colidx, src)
    assert np.allclose(got, ref, rtol=RTOL, atol=0.0), g.name


def test_closeness_edge_cases():
    g = gg.Graph(7, np.zeros(8, dtype=np.int32), np.zeros(0, dtype=np.int32))
    rp, ci = upload(g)
    assert not nk.nk_closeness(rp, ci).any()
    g = gg.cycle(20)
    rp, ci = upload(g)
    assert not nk.nk_closeness_sampled(rp, ci, torch.zeros(0, dtype=torch.int32, device="cuda:0")).any()
    with pytest.raises(nk.NkError) as e:
        nk.nk_closeness_sampled(rp, ci, ivec([0, 20]))
    assert e.value.code == nk.NK_E_INVALID_ARG
    # path counts far beyond 2^64 are no error for closeness
    big = gg.grid(40, 40)
    rp, ci = upload(big)
    assert np.allclose(nk.nk_closeness(rp, ci).cpu().numpy(), oracle.closeness(big.rowptr, big.colidx), rtol=RTOL)
