"""The C-ABI library loads on a machine without a GPU and exports every
function include/nk_bc.h declares; host-side argument checks and the sample
size formula need no device."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "nk_bc.h")


def declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(nk_[a-z_0-9]+)\s*\(", text)))


def test_header_declares_core_calls():
    names = declared()
    for need in ["nk_bc_exact", "nk_bc_sources", "nk_bc_pair_sample", "nk_sssp_counts", "nk_bc_exact_batched",
                 "nk_last_error", "nk_vd_bound"]:
        assert need in names


def test_library_exports_every_declared_symbol():
    import paper_1403_3005_amd as nk
    lib = nk.load()
    raw = ctypes.CDLL(nk._lib.LIB_PATH)
    for name in declared():
        assert hasattr(raw, name), name
    assert nk.nk_version().startswith("nkbc")


def test_binding_covers_header():
    import paper_1403_3005_amd._lib as L
    assert set(L.EXPORTS) == set(declared())


def test_host_argument_checks():
    import paper_1403_3005_amd as nk
    lib = nk.load()
    vp = ctypes.c_void_p
    assert lib.nk_bc_exact(vp(0), vp(0), -1, 0, vp(0), vp(0)) == nk.NK_E_INVALID_ARG
    assert b"negative" in lib.nk_last_error()
    assert lib.nk_bc_exact(vp(0), vp(0), 0, 0, vp(0), vp(0)) == nk.NK_OK  # n = 0: nothing to do
    assert lib.nk_bc_exact(vp(0), vp(0), 5, 0, vp(0), vp(0)) == nk.NK_E_INVALID_ARG  # rowptr NULL
    assert lib.nk_bc_sources(vp(8), vp(8), 5, 10, vp(0), 3, 1.0, vp(8), vp(0)) == nk.NK_E_INVALID_ARG
    assert lib.nk_bc_exact(vp(8), vp(8), 5, 2 ** 31, vp(8), vp(0)) == nk.NK_E_INVALID_ARG
    r = ctypes.c_int64(0)
    v = ctypes.c_int32(0)
    assert lib.nk_bc_pair_sample(vp(8), vp(8), 5, 10, 0.0, 0.1, 1, vp(8), vp(0), ctypes.byref(r), ctypes.byref(v),
                                 vp(0)) == nk.NK_E_INVALID_ARG
    assert lib.nk_bc_pair_sample(vp(8), vp(8), 5, 10, 0.1, 1.0, 1, vp(8), vp(0), ctypes.byref(r), ctypes.byref(v),
                                 vp(0)) == nk.NK_E_INVALID_ARG
    assert lib.nk_bc_exact_batched(-1, None, None, vp(0), vp(0), vp(0), vp(0)) == nk.NK_E_INVALID_ARG


def test_tuning_roundtrip():
    import paper_1403_3005_amd as nk
    old = nk.nk_get_tuning()
    nk.nk_set_tuning(block=512, bu_ratio=2.0, wg_per_cu=1, flags=1, bw_ratio=0.5, scratch_mib=64, batch=8, group=4)
    assert nk.nk_get_tuning() == {"block": 512, "bu_ratio": 2.0, "wg_per_cu": 1, "flags": 1, "bw_ratio": 0.5,
                                  "scratch_mib": 64, "batch": 8, "group": 4}
    with pytest.raises(nk.NkError):
        nk.nk_set_tuning(block=300)
    with pytest.raises(nk.NkError):
        nk.nk_set_tuning(batch=3)
    with pytest.raises(nk.NkError):
        nk.nk_set_tuning(scratch_mib=-1)
    with pytest.raises(nk.NkError):
        nk.nk_set_tuning(group=3)
    nk.nk_set_tuning(**old)


@pytest.mark.parametrize("eps,delta,vd", [(0.01, 0.1, 6), (0.01, 0.1, 10), (0.05, 0.1, 8), (0.02, 0.05, 40),
                                          (0.3, 0.5, 1), (0.01, 0.1, 1000000)])
def test_sample_size_matches_oracle(eps, delta, vd):
    import oracle
    import paper_1403_3005_amd as nk
    assert nk.nk_rk_sample_size(eps, delta, vd) == oracle.rk_sample_size(eps, delta, vd)
    assert nk.nk_rk_sample_size(1.5, delta, vd) == -1


def test_tuning_cache_lookup(tmp_path):
    """The autotuner's cache format and bucket key (host logic, no GPU)."""
    import paper_1403_3005_amd as nk
    path = tmp_path / "tune.json"
    # n = 2^20, 31.4M arcs (mean degree ~30 -> 2^5), max degree 65k (skew 2^11)
    path.write_text('{\n  "n20_d5_s11": [1024, 16, 0.1, 455.5],\n  "n10_d3_s1": [256, 2, 0, 1.0]\n}\n')
    t = nk.nk_tuning_lookup(str(path), 1 << 20, 31399850, 64562)
    assert t["block"] == 1024 and t["bu_ratio"] == 16.0 and abs(t["bw_ratio"] - 0.1) < 1e-6
    t = nk.nk_tuning_lookup(str(path), 2000, 20000, 25)
    assert t["block"] == 256 and t["bu_ratio"] == 2.0 and t["bw_ratio"] == 0.0
    with pytest.raises(nk.NkError):
        nk.nk_tuning_lookup(str(path), 100, 300, 10)


def test_tuning_cache_formats_and_registration(tmp_path):
    """Cache entries of six values and of the older four read back (host
    only); registering a missing file is refused, None unregisters."""
    import json

    import paper_1403_3005_amd as nk
    path = tmp_path / "c.json"
    # n = 1000 (floor log2 = 9), m = 8000 (mean 8: log2 3), max degree 64 (ratio 8: log2 3)
    path.write_text(json.dumps({"n9_d3_s3": [256, 2, 0.25, 1, 8, 1.5], "n10_d3_s3": [512, 8, 0.1, 3.5]}))
    t = nk.nk_tuning_lookup(str(path), 1000, 8000, 64)
    assert (t["block"], t["bu_ratio"], t["bw_ratio"], t["wg_per_cu"], t["batch"]) == (256, 2.0, 0.25, 1, 8)
    t = nk.nk_tuning_lookup(str(path), 1500, 12000, 64)
    assert (t["block"], t["bu_ratio"], t["wg_per_cu"], t["batch"]) == (512, 8.0, 0, 0)
    # eight values: the kernel choice (flag bits 3 and 4) and workgroups per
    # source; other flag bits stay the caller's
    path8 = tmp_path / "c8.json"
    path8.write_text(json.dumps({"n17_d3_s3": [1024, 16, 0.1, 0, 1, 120.5, 8, 4],
                                 "n16_d3_s3": [1024, 16, 0.1, 0, 1, 80.0, 16, 0]}))
    old = nk.nk_get_tuning()
    try:
        nk.nk_set_tuning(flags=2 | 16)
        t = nk.nk_tuning_lookup(str(path8), 200_000, 1_600_000, 64)
        assert (t["flags"], t["group"], t["batch"]) == (2 | 8, 4, 1)
        nk.nk_set_tuning(flags=2 | 8)
        t = nk.nk_tuning_lookup(str(path8), 100_000, 800_000, 64)
        assert (t["flags"], t["group"]) == (2 | 16, 0)
    finally:
        nk.nk_set_tuning(**old)
    with pytest.raises(nk.NkError):
        nk.nk_tuning_lookup(str(path), 100000, 800000, 64)
    with pytest.raises(nk.NkError):
        nk.nk_set_tuning_cache(str(tmp_path / "missing.json"))
    nk.nk_set_tuning_cache(str(path))
    nk.nk_set_tuning_cache(None)
