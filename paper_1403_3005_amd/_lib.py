"""ctypes binding of libnkbc.so: the C ABI of include/nk_bc.h under the same
names.  Argument marshalling only -- every step of the computation runs in
the library's HIP kernels.  PyTorch provides device memory and the stream.

Device arrays are torch tensors on the current HIP device:
  rowptr, colidx, sources  int32, contiguous;
  bc                       float64;
  sigma                    int64 tensor holding uint64 bit patterns;
  counts                   int32 tensor holding uint32 counts.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np
import torch  # loads the HIP runtime the library binds to

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libnkbc.so")
_lib = None

NK_OK = 0
NK_E_INVALID_ARG = -1
NK_E_INVALID_GRAPH = -2
NK_E_SIGMA_OVERFLOW = -3
NK_E_NO_MEMORY = -4
NK_E_HIP = -5
NK_E_BUDGET = -6
NK_E_TIMEOUT = -7
NK_E_INTERNAL = -8

EXPORTS = [
    "nk_last_error", "nk_version", "nk_shutdown", "nk_validate_graph", "nk_bc_exact", "nk_bc_sources",
    "nk_bc_sources_noalloc",
    "nk_bc_sources_linear", "nk_bc_sources_bisect", "nk_bc_directed", "nk_bc_weighted", "nk_transpose", "nk_edge_bc", "nk_closeness", "nk_closeness_sampled",
    "nk_sssp_counts", "nk_vd_bound", "nk_rk_sample_size", "nk_bc_pair_sample", "nk_pair_counts",
    "nk_sample_paths", "nk_bc_exact_batched", "nk_batch_plan_create", "nk_batch_plan_run", "nk_batch_plan_destroy",
    "nk_batch_plan_launch", "nk_batch_plan_progress", "nk_batch_plan_finish",
    "nk_last_stats", "nk_set_tuning", "nk_get_tuning",
    "nk_server_create", "nk_server_add_graph", "nk_server_submit", "nk_server_wait", "nk_server_poll",
    "nk_server_stats", "nk_server_reset_stats", "nk_server_destroy", "nk_autotune", "nk_tuning_lookup",
    "nk_set_tuning_cache",
]


class NkError(RuntimeError):
    def __init__(self, code: int, message: str):
        super().__init__(f"nk status {code}: {message}")
        self.code = code


class NkTuning(ctypes.Structure):
    _fields_ = [("block", ctypes.c_int32), ("bu_ratio", ctypes.c_float), ("wg_per_cu", ctypes.c_int32),
                ("flags", ctypes.c_int32), ("bw_ratio", ctypes.c_float), ("scratch_mib", ctypes.c_int32),
                ("batch", ctypes.c_int32), ("group", ctypes.c_int32)]


def load():
    """Loads libnkbc.so; raises if it was not built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_1403_3005_amd.build.build()")
    lib = ctypes.CDLL(LIB_PATH)
    c = ctypes
    vp, i32p, i64p = c.c_void_p, c.POINTER(c.c_int32), c.POINTER(c.c_int64)
    g = [vp, vp, c.c_int32, c.c_int64]
    sig = {
        "nk_last_error": (c.c_char_p, []),
        "nk_version": (c.c_char_p, []),
        "nk_shutdown": (None, []),
        "nk_validate_graph": (c.c_int32, g + [c.c_int32, vp]),
        "nk_bc_exact": (c.c_int32, g + [vp, vp]),
        "nk_bc_sources": (c.c_int32, g + [vp, c.c_int32, c.c_double, vp, vp]),
        "nk_bc_sources_noalloc": (c.c_int32, g + [vp, c.c_int32, c.c_double, vp, vp]),
        "nk_bc_sources_linear": (c.c_int32, g + [vp, c.c_int32, c.c_double, vp, vp]),
        "nk_bc_sources_bisect": (c.c_int32, g + [vp, c.c_int32, c.c_double, vp, vp]),
        "nk_bc_directed": (c.c_int32, [vp, vp, vp, vp, c.c_int32, c.c_int64, vp, c.c_int32, c.c_double, vp, vp]),
        "nk_transpose": (c.c_int32, g + [vp, vp, vp]),
        "nk_bc_weighted": (c.c_int32, [vp, vp, vp, c.c_int32, c.c_int64, vp, c.c_int32, c.c_double, vp, vp]),
        "nk_edge_bc": (c.c_int32, g + [vp, c.c_int32, c.c_double, vp, vp, vp]),
        "nk_closeness": (c.c_int32, g + [vp, vp]),
        "nk_closeness_sampled": (c.c_int32, g + [vp, c.c_int32, vp, vp]),
        "nk_sssp_counts": (c.c_int32, g + [vp, c.c_int32, vp, vp, vp]),
        "nk_vd_bound": (c.c_int32, g + [i32p, vp]),
        "nk_rk_sample_size": (c.c_int64, [c.c_double, c.c_double, c.c_int32]),
        "nk_bc_pair_sample": (c.c_int32, g + [c.c_double, c.c_double, c.c_uint64, vp, vp, i64p, i32p, vp]),
        "nk_pair_counts": (c.c_int32, g + [c.c_int64, c.c_uint64, vp, vp]),
        "nk_sample_paths": (c.c_int32, g + [c.c_uint64, c.c_int64, c.c_int32, c.c_int32, vp, vp, vp, vp]),
        "nk_bc_exact_batched": (c.c_int32, [c.c_int32, i64p, i64p, vp, vp, vp, vp]),
        "nk_batch_plan_create": (c.c_int32, [c.c_int32, i64p, i64p, vp, vp, vp, c.POINTER(vp)]),
        "nk_batch_plan_run": (c.c_int32, [vp, vp]),
        "nk_batch_plan_launch": (c.c_int32, [vp, vp]),
        "nk_batch_plan_progress": (c.c_int32, [vp, i64p, i64p, i32p]),
        "nk_batch_plan_finish": (c.c_int32, [vp, vp]),
        "nk_batch_plan_destroy": (None, [vp]),
        "nk_last_stats": (c.c_int32, [i64p]),
        "nk_set_tuning": (c.c_int32, [c.POINTER(NkTuning)]),
        "nk_get_tuning": (c.c_int32, [c.POINTER(NkTuning)]),
        "nk_server_create": (c.c_int32, [c.c_size_t, c.c_int32, c.POINTER(vp)]),
        "nk_server_add_graph": (c.c_int32, [vp, vp, vp, c.c_int32, c.c_int64, i32p]),
        "nk_server_submit": (c.c_int32, [vp, c.c_int32, i32p, c.c_int32, c.c_double, c.c_double, c.c_uint64,
                                         c.POINTER(c.c_double), i64p]),
        "nk_server_wait": (c.c_int32, [vp, c.c_int64, c.c_double, c.POINTER(c.c_double)]),
        "nk_server_poll": (c.c_int32, [vp, c.c_int64, i32p]),
        "nk_server_stats": (c.c_int32, [vp, c.POINTER(c.c_double)]),
        "nk_server_reset_stats": (c.c_int32, [vp]),
        "nk_server_destroy": (None, [vp]),
        "nk_autotune": (c.c_int32, g + [vp, c.c_int32, c.c_char_p, c.POINTER(NkTuning), vp]),
        "nk_tuning_lookup": (c.c_int32, [c.c_char_p, c.c_int32, c.c_int64, c.c_int64, c.POINTER(NkTuning)]),
        "nk_set_tuning_cache": (c.c_int32, [c.c_char_p]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def _check(code: int):
    if code != NK_OK:
        msg = load().nk_last_error().decode(errors="replace")
        raise NkError(code, msg)


def _stream(stream):
    if stream is None:
        return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    if isinstance(stream, torch.cuda.Stream):
        return ctypes.c_void_p(stream.cuda_stream)
    return ctypes.c_void_p(int(stream))


def _dev(t, dtype, name):
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a device tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must have dtype {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return ctypes.c_void_p(t.data_ptr())


def _graph(rowptr, colidx):
    rp = _dev(rowptr, torch.int32, "rowptr")
    ci = _dev(colidx, torch.int32, "colidx")
    n = rowptr.numel() - 1
    m = colidx.numel()
    return rp, ci, n, m


def nk_version() -> str:
    return load().nk_version().decode()


def nk_shutdown():
    load().nk_shutdown()


def nk_validate_graph(rowptr, colidx, strict: bool = False, stream=None):
    rp, ci, n, m = _graph(rowptr, colidx)
    _check(load().nk_validate_graph(rp, ci, n, m, 1 if strict else 0, _stream(stream)))


def nk_bc_exact(rowptr, colidx, bc=None, stream=None):
    rp, ci, n, m = _graph(rowptr, colidx)
    if bc is None:
        bc = torch.empty(max(n, 0), dtype=torch.float64, device=rowptr.device)
    _check(load().nk_bc_exact(rp, ci, n, m, _dev(bc, torch.float64, "bc"), _stream(stream)))
    return bc


def nk_bc_sources(rowptr, colidx, sources, scale: float = 1.0, bc=None, stream=None):
    rp, ci, n, m = _graph(rowptr, colidx)
    if bc is None:
        bc = torch.empty(max(n, 0), dtype=torch.float64, device=rowptr.device)
    k = sources.numel()
    sp = _dev(sources, torch.int32, "sources") if k > 0 else ctypes.c_void_p(0)
    _check(load().nk_bc_sources(rp, ci, n, m, sp, k, float(scale), _dev(bc, torch.float64, "bc"), _stream(stream)))
    return bc


def nk_bc_sources_noalloc(rowptr, colidx, sources, scale: float = 1.0, bc=None, stream=None):
    """nk_bc_sources with the library's fixed device scratch (no allocation
    inside the call; `bc` may be passed in so the call allocates nothing)."""
    rp, ci, n, m = _graph(rowptr, colidx)
    if bc is None:
        bc = torch.empty(max(n, 0), dtype=torch.float64, device=rowptr.device)
    k = sources.numel()
    sp = _dev(sources, torch.int32, "sources") if k > 0 else ctypes.c_void_p(0)
    _check(load().nk_bc_sources_noalloc(rp, ci, n, m, sp, k, float(scale), _dev(bc, torch.float64, "bc"),
                                        _stream(stream)))
    return bc


def nk_bc_sources_linear(rowptr, colidx, sources=None, scale: float = 1.0, bc=None, stream=None):
    """Linear-scaling estimator over `sources` (None: every vertex), times
    `scale` (2 n / k estimates the exact scores)."""
    rp, ci, n, m = _graph(rowptr, colidx)
    if bc is None:
        bc = torch.empty(max(n, 0), dtype=torch.float64, device=rowptr.device)
    if sources is None:
        k, sp = n, ctypes.c_void_p(0)
    else:
        k = sources.numel()
        sp = _dev(sources, torch.int32, "sources") if k > 0 else ctypes.c_void_p(0)
    _check(load().nk_bc_sources_linear(rp, ci, n, m, sp, k, float(scale), _dev(bc, torch.float64, "bc"),
                                       _stream(stream)))
    return bc


def nk_bc_sources_bisect(rowptr, colidx, sources=None, scale: float = 1.0, bc=None, stream=None):
    """Bisection estimator over `sources` (None: every vertex), times
    `scale` (2 n / k estimates the exact scores)."""
    rp, ci, n, m = _graph(rowptr, colidx)
    if bc is None:
        bc = torch.empty(max(n, 0), dtype=torch.float64, device=rowptr.device)
    if sources is None:
        k, sp = n, ctypes.c_void_p(0)
    else:
        k = sources.numel()
        sp = _dev(sources, torch.int32, "sources") if k > 0 else ctypes.c_void_p(0)
    _check(load().nk_bc_sources_bisect(rp, ci, n, m, sp, k, float(scale), _dev(bc, torch.float64, "bc"),
                                       _stream(stream)))
    return bc


def nk_bc_weighted(rowptr, colidx, weights, sources=None, scale: float = 1.0, bc=None, stream=None):
    """Betweenness with int32 arc weights >= 1 over `sources` (None: every
    vertex) times `scale`; rowptr/colidx are out-arcs."""
    rp, ci, n, m = _graph(rowptr, colidx)
    if bc is None:
        bc = torch.empty(max(n, 0), dtype=torch.float64, device=rowptr.device)
    if sources is None:
        k, sp = n, ctypes.c_void_p(0)
    else:
        k = sources.numel()
        sp = _dev(sources, torch.int32, "sources") if k > 0 else ctypes.c_void_p(0)
    wp = _dev(weights, torch.int32, "weights") if m > 0 else ctypes.c_void_p(0)
    _check(load().nk_bc_weighted(rp, ci, wp, n, m, sp, k, float(scale), _dev(bc, torch.float64, "bc"),
                                 _stream(stream)))
    return bc


def nk_transpose(rowptr, colidx, stream=None):
    """In-arc CSR (trowptr, tcolidx) of a directed graph's out-arc CSR."""
    rp, ci, n, m = _graph(rowptr, colidx)
    trowptr = torch.empty(n + 1, dtype=torch.int32, device=rowptr.device)
    tcolidx = torch.empty(max(m, 1), dtype=torch.int32, device=rowptr.device)
    _check(load().nk_transpose(rp, ci, n, m, _dev(trowptr, torch.int32, "trowptr"),
                               _dev(tcolidx, torch.int32, "tcolidx"), _stream(stream)))
    return trowptr, tcolidx[:m]


def nk_bc_directed(rowptr, colidx, sources=None, scale: float = 1.0, trowptr=None, tcolidx=None, bc=None,
                   stream=None):
    """Directed betweenness over `sources` (None: every vertex) times
    `scale`; (trowptr, tcolidx) is the in-arc CSR or None (top-down only)."""
    rp, ci, n, m = _graph(rowptr, colidx)
    if bc is None:
        bc = torch.empty(max(n, 0), dtype=torch.float64, device=rowptr.device)
    if sources is None:
        k, sp = n, ctypes.c_void_p(0)
    else:
        k = sources.numel()
        sp = _dev(sources, torch.int32, "sources") if k > 0 else ctypes.c_void_p(0)
    trp = _dev(trowptr, torch.int32, "trowptr") if trowptr is not None else ctypes.c_void_p(0)
    tci = _dev(tcolidx, torch.int32, "tcolidx") if tcolidx is not None and tcolidx.numel() > 0 else ctypes.c_void_p(0)
    _check(load().nk_bc_directed(rp, ci, trp, tci, n, m, sp, k, float(scale), _dev(bc, torch.float64, "bc"),
                                 _stream(stream)))
    return bc


def nk_edge_bc(rowptr, colidx, sources=None, scale: float = 1.0, stream=None):
    """(ebc FP64[m] per arc, bc FP64[n]): edge and vertex betweenness over
    `sources` (None: every vertex, exact), times `scale`."""
    rp, ci, n, m = _graph(rowptr, colidx)
    ebc = torch.empty(max(m, 0), dtype=torch.float64, device=rowptr.device)
    bc = torch.empty(max(n, 0), dtype=torch.float64, device=rowptr.device)
    if sources is None:
        k, sp = n, ctypes.c_void_p(0)
    else:
        k = sources.numel()
        sp = _dev(sources, torch.int32, "sources") if k > 0 else ctypes.c_void_p(0)
    ep = _dev(ebc, torch.float64, "ebc") if m > 0 else ctypes.c_void_p(0)
    bp = _dev(bc, torch.float64, "bc") if n > 0 else ctypes.c_void_p(0)
    _check(load().nk_edge_bc(rp, ci, n, m, sp, k, float(scale), ep, bp, _stream(stream)))
    return ebc, bc


def nk_closeness(rowptr, colidx, out=None, stream=None):
    """Exact closeness (generalised to disconnected graphs), FP64[n]."""
    rp, ci, n, m = _graph(rowptr, colidx)
    if out is None:
        out = torch.empty(max(n, 0), dtype=torch.float64, device=rowptr.device)
    _check(load().nk_closeness(rp, ci, n, m, _dev(out, torch.float64, "out") if n > 0 else ctypes.c_void_p(0),
                               _stream(stream)))
    return out


def nk_closeness_sampled(rowptr, colidx, sources, out=None, stream=None):
    """Eppstein-Wang sampled closeness over `sources`, FP64[n]."""
    rp, ci, n, m = _graph(rowptr, colidx)
    if out is None:
        out = torch.empty(max(n, 0), dtype=torch.float64, device=rowptr.device)
    k = sources.numel()
    sp = _dev(sources, torch.int32, "sources") if k > 0 else ctypes.c_void_p(0)
    _check(load().nk_closeness_sampled(rp, ci, n, m, sp, k,
                                       _dev(out, torch.float64, "out") if n > 0 else ctypes.c_void_p(0),
                                       _stream(stream)))
    return out


def nk_sssp_counts(rowptr, colidx, sources, stream=None):
    """(d int32[k, n], sigma int64[k, n] holding uint64 bits)."""
    rp, ci, n, m = _graph(rowptr, colidx)
    k = sources.numel()
    d = torch.empty((k, n), dtype=torch.int32, device=rowptr.device)
    sg = torch.empty((k, n), dtype=torch.int64, device=rowptr.device)
    if k > 0 and n > 0:
        _check(load().nk_sssp_counts(rp, ci, n, m, _dev(sources, torch.int32, "sources"), k,
                                     _dev(d, torch.int32, "d"), _dev(sg, torch.int64, "sigma"), _stream(stream)))
    return d, sg


def nk_vd_bound(rowptr, colidx, stream=None) -> dict:
    rp, ci, n, m = _graph(rowptr, colidx)
    info = (ctypes.c_int32 * 8)()
    _check(load().nk_vd_bound(rp, ci, n, m, info, _stream(stream)))
    keys = ["x0", "e1", "a", "e2", "vd_ub", "vd_lb", "c0", "c2"]
    return {k: int(v) for k, v in zip(keys, info)}


def nk_rk_sample_size(eps: float, delta: float, vd: int) -> int:
    return int(load().nk_rk_sample_size(eps, delta, vd))


def nk_bc_pair_sample(rowptr, colidx, eps: float, delta: float, seed: int, stream=None):
    """(bc float64[n], counts int32[n] holding uint32, r, vd)."""
    rp, ci, n, m = _graph(rowptr, colidx)
    bc = torch.empty(max(n, 0), dtype=torch.float64, device=rowptr.device)
    cnt = torch.empty(max(n, 0), dtype=torch.int32, device=rowptr.device)
    r = ctypes.c_int64(0)
    vd = ctypes.c_int32(0)
    _check(load().nk_bc_pair_sample(rp, ci, n, m, eps, delta, seed, _dev(bc, torch.float64, "bc"),
                                    _dev(cnt, torch.int32, "counts"), ctypes.byref(r), ctypes.byref(vd),
                                    _stream(stream)))
    return bc, cnt, int(r.value), int(vd.value)


def nk_pair_counts(rowptr, colidx, r: int, seed: int, stream=None):
    rp, ci, n, m = _graph(rowptr, colidx)
    cnt = torch.empty(max(n, 0), dtype=torch.int32, device=rowptr.device)
    _check(load().nk_pair_counts(rp, ci, n, m, r, seed, _dev(cnt, torch.int32, "counts"), _stream(stream)))
    return cnt


def nk_sample_paths(rowptr, colidx, seed: int, j0: int, count: int, maxlen: int, stream=None):
    """(uv int32[count, 2], len int32[count], path int32[count, maxlen])."""
    rp, ci, n, m = _graph(rowptr, colidx)
    dev = rowptr.device
    uv = torch.empty((count, 2), dtype=torch.int32, device=dev)
    ln = torch.empty(count, dtype=torch.int32, device=dev)
    path = torch.full((count, max(maxlen, 1)), -1, dtype=torch.int32, device=dev)
    _check(load().nk_sample_paths(rp, ci, n, m, seed, j0, count, maxlen, _dev(uv, torch.int32, "uv"),
                                  _dev(ln, torch.int32, "len"), _dev(path, torch.int32, "path"), _stream(stream)))
    return uv, ln, path


def nk_bc_exact_batched(vtx_off, arc_off, rowptr_cat, colidx_cat, stream=None):
    vo = np.ascontiguousarray(vtx_off, dtype=np.int64)
    ao = np.ascontiguousarray(arc_off, dtype=np.int64)
    G = vo.shape[0] - 1
    bc = torch.empty(int(vo[-1]), dtype=torch.float64, device=rowptr_cat.device)
    i64p = ctypes.POINTER(ctypes.c_int64)
    ci = _dev(colidx_cat, torch.int32, "colidx_cat") if colidx_cat.numel() else ctypes.c_void_p(0)
    _check(load().nk_bc_exact_batched(G, vo.ctypes.data_as(i64p), ao.ctypes.data_as(i64p),
                                      _dev(rowptr_cat, torch.int32, "rowptr_cat"), ci,
                                      _dev(bc, torch.float64, "bc_cat") if bc.numel() else ctypes.c_void_p(0),
                                      _stream(stream)))
    return bc


class NkBatchPlan:
    """A batched exact run captured once into a HIP graph and replayed
    (nk_batch_plan_* in include/nk_bc.h).  Keeps the graph tensors and its
    output tensor alive; run() overwrites and returns the output."""

    def __init__(self, vtx_off, arc_off, rowptr_cat, colidx_cat):
        vo = np.ascontiguousarray(vtx_off, dtype=np.int64)
        ao = np.ascontiguousarray(arc_off, dtype=np.int64)
        i64p = ctypes.POINTER(ctypes.c_int64)
        self.bc = torch.empty(int(vo[-1]), dtype=torch.float64, device=rowptr_cat.device)
        self._keep = (rowptr_cat, colidx_cat)
        ci = _dev(colidx_cat, torch.int32, "colidx_cat") if colidx_cat.numel() else ctypes.c_void_p(0)
        out = _dev(self.bc, torch.float64, "bc_cat") if self.bc.numel() else ctypes.c_void_p(0)
        self._h = ctypes.c_void_p(0)
        _check(load().nk_batch_plan_create(vo.shape[0] - 1, vo.ctypes.data_as(i64p), ao.ctypes.data_as(i64p),
                                           _dev(rowptr_cat, torch.int32, "rowptr_cat"), ci, out,
                                           ctypes.byref(self._h)))

    def run(self, stream=None):
        _check(load().nk_batch_plan_run(self._h, _stream(stream)))
        return self.bc

    def launch(self, stream=None):
        """Enqueues a run and returns at once (see progress, finish)."""
        _check(load().nk_batch_plan_launch(self._h, _stream(stream)))

    def progress(self):
        """(sources done, sources in all, finished) of the launched run."""
        d, t, f = ctypes.c_int64(0), ctypes.c_int64(0), ctypes.c_int32(0)
        _check(load().nk_batch_plan_progress(self._h, ctypes.byref(d), ctypes.byref(t), ctypes.byref(f)))
        return int(d.value), int(t.value), bool(f.value)

    def finish(self, stream=None):
        """Waits for the launched run, checks its status; returns the scores."""
        _check(load().nk_batch_plan_finish(self._h, _stream(stream)))
        return self.bc

    def close(self):
        if self._h:
            load().nk_batch_plan_destroy(self._h)
            self._h = ctypes.c_void_p(0)

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


STAT_KEYS = ["sources", "reached", "arcs_fwd", "arcs_bwd", "dag_arcs", "levels_td", "levels_bu", "workgroups",
             "kernel_us", "block", "bitmap_lds", "arcs_reached", "levels_bw_push", "sources_per_task", "pair_deferred",
             "reserved15", "cyc_init", "cyc_topdown", "cyc_bottomup", "cyc_mark", "cyc_pull", "cyc_push",
             "cyc_reset", "cyc_other", "sub_bu_stage", "sub_bu_arcs", "sub_bu_finalize", "sub_pull_stage",
             "sub_pull_arcs", "sub_pull_finalize", "reserved30", "reserved31"]


def nk_last_stats() -> dict:
    out = (ctypes.c_int64 * 32)()
    _check(load().nk_last_stats(out))
    return {k: int(v) for k, v in zip(STAT_KEYS, out)}


def nk_set_tuning(block: int = 0, bu_ratio: float = 16.0, wg_per_cu: int = 0, flags: int = 0, bw_ratio: float = 0.1,
                  scratch_mib: int = 0, batch: int = 0, group: int = 0):
    t = NkTuning(block, bu_ratio, wg_per_cu, flags, bw_ratio, scratch_mib, batch, group)
    _check(load().nk_set_tuning(ctypes.byref(t)))


def nk_get_tuning() -> dict:
    t = NkTuning()
    _check(load().nk_get_tuning(ctypes.byref(t)))
    return _tuning_dict(t)


def _tuning_dict(t) -> dict:
    return {"block": t.block, "bu_ratio": t.bu_ratio, "wg_per_cu": t.wg_per_cu, "flags": t.flags,
            "bw_ratio": t.bw_ratio, "scratch_mib": t.scratch_mib, "batch": t.batch, "group": t.group}


def nk_set_tuning_cache(cache_path: str | None) -> None:
    """Registers an autotuner cache (None unregisters): later calls on graphs
    whose shape has an entry run under it (see include/nk_bc.h)."""
    _check(load().nk_set_tuning_cache(cache_path.encode() if cache_path else None))


def nk_autotune(rowptr, colidx, sources, cache_path: str | None = None, stream=None) -> dict:
    """Fastest tuning on a sample of sources (see include/nk_bc.h)."""
    rp, ci, n, m = _graph(rowptr, colidx)
    t = NkTuning()
    cp = cache_path.encode() if cache_path else None
    _check(load().nk_autotune(rp, ci, n, m, _dev(sources, torch.int32, "sources"), sources.numel(), cp,
                              ctypes.byref(t), _stream(stream)))
    return _tuning_dict(t)


def nk_tuning_lookup(cache_path: str, n: int, m: int, max_deg: int) -> dict:
    t = NkTuning()
    _check(load().nk_tuning_lookup(cache_path.encode(), n, m, max_deg, ctypes.byref(t)))
    return _tuning_dict(t)


class NkServer:
    """Binding of the nk_server_* family: a resident graph pool served with
    continuous batching (see include/nk_bc.h)."""

    def __init__(self, hbm_budget_bytes: int, slots: int = 4):
        self._h = ctypes.c_void_p(0)
        _check(load().nk_server_create(int(hbm_budget_bytes), int(slots), ctypes.byref(self._h)))
        self.n = []
        self._out = {}

    def add_graph(self, rowptr, colidx) -> int:
        rp, ci, n, m = _graph(rowptr, colidx)
        gid = ctypes.c_int32(0)
        _check(load().nk_server_add_graph(self._h, rp, ci, n, m, ctypes.byref(gid)))
        self.n.append(n)
        return int(gid.value)

    def submit(self, graph_id: int, sources=None, eps: float = 0.0, delta: float = 0.1, seed: int = 0) -> int:
        """Queues a request; returns its ticket.  sources: host int32 array
        (k-source request) or None (pair sampling with eps, delta, seed)."""
        known = 0 <= graph_id < len(self.n)
        out = np.zeros(self.n[graph_id] if known else 1, dtype=np.float64)  # unknown ids: the library rejects them
        t = ctypes.c_int64(0)
        if sources is not None:
            src = np.ascontiguousarray(sources, dtype=np.int32)
            k = int(src.shape[0])
            sp = src.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))
        else:
            src, k, sp = None, 0, None
        _check(load().nk_server_submit(self._h, graph_id, sp, k, float(eps), float(delta), int(seed),
                                       out.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), ctypes.byref(t)))
        self._out[int(t.value)] = out
        return int(t.value)

    def wait(self, ticket: int, timeout: float = -1.0):
        """(scores, latency in seconds) of a finished request."""
        lat = ctypes.c_double(0.0)
        code = load().nk_server_wait(self._h, ticket, float(timeout), ctypes.byref(lat))
        if code == NK_E_TIMEOUT:
            raise TimeoutError(f"ticket {ticket} not done")
        out = self._out.pop(ticket)
        _check(code)
        return out, float(lat.value)

    def poll(self, ticket: int) -> bool:
        d = ctypes.c_int32(0)
        _check(load().nk_server_poll(self._h, ticket, ctypes.byref(d)))
        return bool(d.value)

    def stats(self) -> dict:
        out = (ctypes.c_double * 8)()
        _check(load().nk_server_stats(self._h, out))
        keys = ["completed", "failed", "p50_ms", "p99_ms", "max_ms", "gteps", "max_inflight", "device_bytes"]
        return {k: float(v) for k, v in zip(keys, out)}

    def reset_stats(self):
        _check(load().nk_server_reset_stats(self._h))

    def close(self):
        if self._h:
            load().nk_server_destroy(self._h)
            self._h = ctypes.c_void_p(0)

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()
