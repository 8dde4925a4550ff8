"""Shared helpers for the GPU tests: device upload and the score tolerance.

Scores: |got - ref| <= 1e-12 * |ref|, or <= 1e-9 where |ref| < 1e-3 (the
GPU sums dependencies in a different order than the oracle; every term is
non-negative, so the relative rounding error stays near (degree + depth)
* 2^-53).  Distances, path counts and sample counts must match exactly.
"""
import numpy as np
import torch

RTOL = 1e-12
ATOL_NEAR_ZERO = 1e-9


def dev():
    return torch.device("cuda:0")


def upload(g):
    d = dev()
    rp = torch.from_numpy(np.ascontiguousarray(g.rowptr, dtype=np.int32)).to(d)
    ci = torch.from_numpy(np.ascontiguousarray(g.colidx, dtype=np.int32)).to(d)
    if ci.numel() == 0:
        ci = torch.zeros(0, dtype=torch.int32, device=d)
    return rp, ci


def ivec(x):
    return torch.tensor(np.asarray(x, dtype=np.int32), dtype=torch.int32, device=dev())


def assert_scores_close(got, ref, what=""):
    got = np.asarray(got, dtype=np.float64)
    ref = np.asarray(ref, dtype=np.float64)
    assert got.shape == ref.shape, (what, got.shape, ref.shape)
    err = np.abs(got - ref)
    ok = (err <= RTOL * np.abs(ref)) | ((np.abs(ref) < 1e-3) & (err <= ATOL_NEAR_ZERO))
    if not ok.all():
        i = int(np.argmax(~ok))
        raise AssertionError(f"{what}: {int((~ok).sum())} scores off, first v={i} got={got[i]!r} ref={ref[i]!r}")
