"""CPU oracle for Brandes betweenness -- TEST INFRASTRUCTURE ONLY.

Only the test suite, the smoke check and the CPU-baseline leg of the
benchmark may import this package.  The GPU library and its Python binding
never import it, and nothing here imports them.

``brandes.c`` holds plain sequential Brandes (exact, source set, the
linear-scaling source-set estimator, edge betweenness, closeness, pair
sampling) and is loaded through ctypes; ``bruteforce.py`` holds exact
rational all-simple-paths enumeration for graphs of at most a dozen
vertices.  Status codes: 0 ok, -1 invalid argument, -2 invalid graph,
-3 sigma overflow, -4 out of memory.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "brandes.c")
# NK_SANITIZE=1 selects a build instrumented with AddressSanitizer and
# UndefinedBehaviorSanitizer (the host process must preload the ASan runtime)
_SANITIZE = os.environ.get("NK_SANITIZE") == "1"
_LIB_PATH = os.path.join(_HERE, "liboracle_san.so" if _SANITIZE else "liboracle.so")
_SAN_FLAGS = ["-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined", "-fno-sanitize-recover=all"]
_lib = None

OK, E_INVALID_ARG, E_INVALID_GRAPH, E_SIGMA_OVERFLOW, E_NO_MEMORY = 0, -1, -2, -3, -4


class OracleError(RuntimeError):
    def __init__(self, code: int, what: str):
        super().__init__(f"oracle {what} failed with status {code}")
        self.code = code


def build(force: bool = True) -> str:
    """Compile brandes.c into liboracle.so (plain C, -O2)."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp%d" % os.getpid()
        opt = _SAN_FLAGS if _SANITIZE else ["-O2"]
        subprocess.check_call(["gcc"] + opt + ["-fPIC", "-shared", "-pthread", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        build(force=False)
    lib = ctypes.CDLL(_LIB_PATH)
    c = ctypes
    i32p, u64p, f64p, i64p, u32p = (c.POINTER(c.c_int32), c.POINTER(c.c_uint64), c.POINTER(c.c_double),
                                    c.POINTER(c.c_int64), c.POINTER(c.c_uint32))
    g = [c.c_int32, c.c_int64, i32p, i32p]
    sig = {
        "or_validate": (c.c_int, g),
        "or_validate_strict": (c.c_int, g),
        "or_sssp_counts": (c.c_int, g + [c.c_int32, i32p, u64p]),
        "or_bc_sources": (c.c_int, g + [i32p, c.c_int32, c.c_double, f64p, c.c_int32]),
        "or_bc_exact": (c.c_int, g + [f64p, c.c_int32]),
        "or_bc_sources_linear": (c.c_int, g + [i32p, c.c_int32, c.c_double, f64p, c.c_int32]),
        "or_bc_sources_bisect": (c.c_int, g + [i32p, c.c_int32, c.c_double, f64p, c.c_int32]),
        "or_bc_directed": (c.c_int, g + [i32p, c.c_int32, c.c_double, f64p, c.c_int32]),
        "or_bc_weighted": (c.c_int, g + [i32p, i32p, c.c_int32, c.c_double, f64p, c.c_int32]),
        "or_sssp_weighted": (c.c_int, g + [i32p, c.c_int32, c.POINTER(c.c_int64), c.POINTER(c.c_uint64)]),
        "or_edge_bc_sources": (c.c_int, g + [i32p, c.c_int32, c.c_double, f64p, f64p, c.c_int32]),
        "or_closeness": (c.c_int, g + [f64p]),
        "or_closeness_approx": (c.c_int, g + [i32p, c.c_int32, f64p, i64p]),
        "or_work_counts": (c.c_int, g + [i32p, c.c_int32, i64p]),
        "or_mix64": (c.c_uint64, [c.c_uint64]),
        "or_draw": (c.c_uint64, [c.c_uint64] * 4),
        "or_bounded": (c.c_uint64, [c.c_uint64, c.c_uint64]),
        "or_vd_bound": (c.c_int, g + [i32p]),
        "or_rk_sample_size": (c.c_int64, [c.c_double, c.c_double, c.c_int32]),
        "or_sample_path": (c.c_int, g + [c.c_uint64, c.c_int64, i32p, i32p, i32p]),
        "or_sample_path_uv": (c.c_int, g + [c.c_uint64, c.c_int64, c.c_int32, c.c_int32, i32p, i32p]),
        "or_sample_path_given": (c.c_int, g + [c.c_int32, c.c_int32, u64p, c.c_int32, u64p, u64p, c.c_int32, i32p,
                                               i32p, i32p]),
        "or_pair_counts": (c.c_int, g + [c.c_int64, c.c_uint64, u32p, c.c_int32]),
        "or_pair_sample": (c.c_int, g + [c.c_double, c.c_double, c.c_uint64, u32p, f64p, i64p, i32p]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def _ptr(a, ctype):
    return a.ctypes.data_as(ctypes.POINTER(ctype))


def _graph_args(rowptr, colidx):
    rowptr = np.ascontiguousarray(rowptr, dtype=np.int32)
    colidx = np.ascontiguousarray(colidx, dtype=np.int32)
    if colidx.size == 0:
        colidx = np.zeros(1, dtype=np.int32)
    n = rowptr.shape[0] - 1
    m = int(rowptr[-1]) if n > 0 else 0
    return n, m, rowptr, colidx


def _check(code: int, what: str):
    if code != OK:
        raise OracleError(code, what)


def validate(rowptr, colidx, strict: bool = False, m: int | None = None) -> int:
    """Status code of the structural (or strict simple-graph) CSR checks."""
    rowptr = np.ascontiguousarray(rowptr, dtype=np.int32)
    colidx = np.ascontiguousarray(colidx, dtype=np.int32)
    n = rowptr.shape[0] - 1
    if m is None:
        m = colidx.shape[0]
    if colidx.size == 0:
        colidx = np.zeros(1, dtype=np.int32)
    fn = _load().or_validate_strict if strict else _load().or_validate
    return int(fn(n, m, _ptr(rowptr, ctypes.c_int32), _ptr(colidx, ctypes.c_int32)))


def sssp_counts(rowptr, colidx, source: int):
    """(d int32[n] with -1 unreachable, sigma uint64[n]) for one source."""
    n, m, rowptr, colidx = _graph_args(rowptr, colidx)
    d = np.empty(max(n, 1), dtype=np.int32)
    s = np.empty(max(n, 1), dtype=np.uint64)
    _check(_load().or_sssp_counts(n, m, _ptr(rowptr, ctypes.c_int32), _ptr(colidx, ctypes.c_int32),
                                  source, _ptr(d, ctypes.c_int32), _ptr(s, ctypes.c_uint64)), "sssp_counts")
    return d[:n], s[:n]


def bc_sources(rowptr, colidx, sources, scale: float = 1.0, nthreads: int = 1) -> np.ndarray:
    """Betweenness summed over `sources` (in order), times `scale`."""
    n, m, rowptr, colidx = _graph_args(rowptr, colidx)
    src = np.ascontiguousarray(sources, dtype=np.int32)
    k = int(src.shape[0])
    if k == 0:
        src = np.zeros(1, dtype=np.int32)
    bc = np.zeros(max(n, 1), dtype=np.float64)
    _check(_load().or_bc_sources(n, m, _ptr(rowptr, ctypes.c_int32), _ptr(colidx, ctypes.c_int32),
                                 _ptr(src, ctypes.c_int32), k, float(scale), _ptr(bc, ctypes.c_double),
                                 nthreads), "bc_sources")
    return bc[:n]


def bc_exact(rowptr, colidx, nthreads: int = 1) -> np.ndarray:
    n, m, rowptr, colidx = _graph_args(rowptr, colidx)
    bc = np.zeros(max(n, 1), dtype=np.float64)
    _check(_load().or_bc_exact(n, m, _ptr(rowptr, ctypes.c_int32), _ptr(colidx, ctypes.c_int32),
                               _ptr(bc, ctypes.c_double), nthreads), "bc_exact")
    return bc[:n]


def bc_sources_linear(rowptr, colidx, sources, scale: float = 1.0, nthreads: int = 1) -> np.ndarray:
    """Linear-scaling (Geisberger-Sanders-Schultes) dependencies summed over
    `sources`, times `scale` (2 n / k gives the estimate of exact scores)."""
    n, m, rowptr, colidx = _graph_args(rowptr, colidx)
    src = np.ascontiguousarray(sources, dtype=np.int32)
    k = int(src.shape[0])
    if k == 0:
        src = np.zeros(1, dtype=np.int32)
    bc = np.zeros(max(n, 1), dtype=np.float64)
    _check(_load().or_bc_sources_linear(n, m, _ptr(rowptr, ctypes.c_int32), _ptr(colidx, ctypes.c_int32),
                                        _ptr(src, ctypes.c_int32), k, float(scale), _ptr(bc, ctypes.c_double),
                                        nthreads), "bc_sources_linear")
    return bc[:n]


def bc_sources_bisect(rowptr, colidx, sources, scale: float = 1.0, nthreads: int = 1) -> np.ndarray:
    """Bisection (Geisberger-Sanders-Schultes) dependencies summed over
    `sources`, times `scale` (2 n / k gives the estimate of exact scores)."""
    n, m, rowptr, colidx = _graph_args(rowptr, colidx)
    src = np.ascontiguousarray(sources, dtype=np.int32)
    k = int(src.shape[0])
    if k == 0:
        src = np.zeros(1, dtype=np.int32)
    bc = np.zeros(max(n, 1), dtype=np.float64)
    _check(_load().or_bc_sources_bisect(n, m, _ptr(rowptr, ctypes.c_int32), _ptr(colidx, ctypes.c_int32),
                                        _ptr(src, ctypes.c_int32), k, float(scale), _ptr(bc, ctypes.c_double),
                                        nthreads), "bc_sources_bisect")
    return bc[:n]


def bc_directed(rowptr, colidx, sources=None, scale: float = 1.0, nthreads: int = 1) -> np.ndarray:
    """Directed betweenness (out-arc CSR, no symmetry needed) summed over
    `sources` (None: every vertex, the exact scores), times `scale`."""
    n, m, rowptr, colidx = _graph_args(rowptr, colidx)
    src = np.arange(n, dtype=np.int32) if sources is None else np.ascontiguousarray(sources, dtype=np.int32)
    k = int(src.shape[0])
    if k == 0:
        src = np.zeros(1, dtype=np.int32)
    bc = np.zeros(max(n, 1), dtype=np.float64)
    _check(_load().or_bc_directed(n, m, _ptr(rowptr, ctypes.c_int32), _ptr(colidx, ctypes.c_int32),
                                  _ptr(src, ctypes.c_int32), k, float(scale), _ptr(bc, ctypes.c_double), nthreads),
           "bc_directed")
    return bc[:n]


def bc_weighted(rowptr, colidx, weights, sources=None, scale: float = 1.0, nthreads: int = 1) -> np.ndarray:
    """Betweenness with int32 arc weights >= 1 (out-arc CSR) summed over
    `sources` (None: every vertex), times `scale`."""
    n, m, rowptr, colidx = _graph_args(rowptr, colidx)
    wts = np.ascontiguousarray(weights, dtype=np.int32)
    if wts.size == 0:
        wts = np.ones(1, dtype=np.int32)
    src = np.arange(n, dtype=np.int32) if sources is None else np.ascontiguousarray(sources, dtype=np.int32)
    k = int(src.shape[0])
    if k == 0:
        src = np.zeros(1, dtype=np.int32)
    bc = np.zeros(max(n, 1), dtype=np.float64)
    _check(_load().or_bc_weighted(n, m, _ptr(rowptr, ctypes.c_int32), _ptr(colidx, ctypes.c_int32),
                                  _ptr(wts, ctypes.c_int32), _ptr(src, ctypes.c_int32), k, float(scale),
                                  _ptr(bc, ctypes.c_double), nthreads), "bc_weighted")
    return bc[:n]


def sssp_weighted(rowptr, colidx, weights, source: int):
    """(d int64 with -1 unreachable, sigma uint64) from one source."""
    n, m, rowptr, colidx = _graph_args(rowptr, colidx)
    wts = np.ascontiguousarray(weights, dtype=np.int32)
    if wts.size == 0:
        wts = np.ones(1, dtype=np.int32)
    d = np.zeros(max(n, 1), dtype=np.int64)
    sigma = np.zeros(max(n, 1), dtype=np.uint64)
    _check(_load().or_sssp_weighted(n, m, _ptr(rowptr, ctypes.c_int32), _ptr(colidx, ctypes.c_int32),
                                    _ptr(wts, ctypes.c_int32), int(source), _ptr(d, ctypes.c_int64),
                                    _ptr(sigma, ctypes.c_uint64)), "sssp_weighted")
    return d[:n], sigma[:n]


def edge_bc(rowptr, colidx, sources=None, scale: float = 1.0, nthreads: int = 1):
    """(ebc, bc): edge betweenness per arc (both arcs of an edge equal) and
    vertex betweenness of the same run, over `sources` (default: all
    vertices, exact), times `scale`."""
    n, m, rowptr, colidx = _graph_args(rowptr, colidx)
    src = np.arange(n, dtype=np.int32) if sources is None else np.ascontiguousarray(sources, dtype=np.int32)
    k = int(src.shape[0])
    if k == 0:
        src = np.zeros(1, dtype=np.int32)
    ebc = np.zeros(max(m, 1), dtype=np.float64)
    bc = np.zeros(max(n, 1), dtype=np.float64)
    _check(_load().or_edge_bc_sources(n, m, _ptr(rowptr, ctypes.c_int32), _ptr(colidx, ctypes.c_int32),
                                      _ptr(src, ctypes.c_int32), k, float(scale), _ptr(ebc, ctypes.c_double),
                                      _ptr(bc, ctypes.c_double), nthreads), "edge_bc")
    return ebc[:m], bc[:n]


def closeness(rowptr, colidx) -> np.ndarray:
    """Exact closeness, generalised to disconnected graphs:
    (r-1)/(n-1) * (r-1)/farness, 0 for isolated vertices."""
    n, m, rowptr, colidx = _graph_args(rowptr, colidx)
    out = np.zeros(max(n, 1), dtype=np.float64)
    _check(_load().or_closeness(n, m, _ptr(rowptr, ctypes.c_int32), _ptr(colidx, ctypes.c_int32),
                                _ptr(out, ctypes.c_double)), "closeness")
    return out[:n]


def closeness_approx(rowptr, colidx, sources):
    """(closeness estimate, integer distance sums) of Eppstein and Wang's
    sampling over `sources`: (n-1) / (n/k * sum of d(s, v))."""
    n, m, rowptr, colidx = _graph_args(rowptr, colidx)
    src = np.ascontiguousarray(sources, dtype=np.int32)
    k = int(src.shape[0])
    if k == 0:
        src = np.zeros(1, dtype=np.int32)
    out = np.zeros(max(n, 1), dtype=np.float64)
    sums = np.zeros(max(n, 1), dtype=np.int64)
    _check(_load().or_closeness_approx(n, m, _ptr(rowptr, ctypes.c_int32), _ptr(colidx, ctypes.c_int32),
                                       _ptr(src, ctypes.c_int32), k, _ptr(out, ctypes.c_double),
                                       _ptr(sums, ctypes.c_int64)), "closeness_approx")
    return out[:n], sums[:n]


def work_counts(rowptr, colidx, sources):
    """(reached vertices, arcs of reached vertices, DAG arcs, sum of depths) over sources."""
    n, m, rowptr, colidx = _graph_args(rowptr, colidx)
    src = np.ascontiguousarray(sources, dtype=np.int32)
    out = np.zeros(4, dtype=np.int64)
    _check(_load().or_work_counts(n, m, _ptr(rowptr, ctypes.c_int32), _ptr(colidx, ctypes.c_int32),
                                  _ptr(src, ctypes.c_int32), int(src.shape[0]), _ptr(out, ctypes.c_int64)),
           "work_counts")
    return tuple(int(x) for x in out)


def mix64(z: int) -> int:
    return int(_load().or_mix64(z))


def draw(seed: int, stream: int, j: int, t: int) -> int:
    return int(_load().or_draw(seed, stream, j, t))


def bounded(x: int, n: int) -> int:
    return int(_load().or_bounded(x, n))


def vd_bound(rowptr, colidx) -> dict:
    n, m, rowptr, colidx = _graph_args(rowptr, colidx)
    info = np.zeros(8, dtype=np.int32)
    _check(_load().or_vd_bound(n, m, _ptr(rowptr, ctypes.c_int32), _ptr(colidx, ctypes.c_int32),
                               _ptr(info, ctypes.c_int32)), "vd_bound")
    keys = ["x0", "e1", "a", "e2", "vd_ub", "vd_lb", "c0", "c2"]
    return {k: int(v) for k, v in zip(keys, info)}


def rk_sample_size(eps: float, delta: float, vd: int) -> int:
    return int(_load().or_rk_sample_size(eps, delta, vd))


def sample_path(rowptr, colidx, seed: int, j: int):
    """(u, v, interior vertices from v's side) of sample j; interior is None
    if v is unreachable from u."""
    n, m, rowptr, colidx = _graph_args(rowptr, colidx)
    uv = np.zeros(2, dtype=np.int32)
    interior = np.zeros(max(n, 1), dtype=np.int32)
    ln = np.zeros(1, dtype=np.int32)
    _check(_load().or_sample_path(n, m, _ptr(rowptr, ctypes.c_int32), _ptr(colidx, ctypes.c_int32),
                                  seed, j, _ptr(uv, ctypes.c_int32), _ptr(interior, ctypes.c_int32),
                                  _ptr(ln, ctypes.c_int32)), "sample_path")
    L = int(ln[0])
    return int(uv[0]), int(uv[1]), (None if L < 0 else [int(x) for x in interior[:L]])


def sample_path_uv(rowptr, colidx, seed: int, j: int, u: int, v: int):
    """Interior vertices (from v's side) of the path that draw index j picks
    for the explicit pair (u, v); None if v is unreachable."""
    n, m, rowptr, colidx = _graph_args(rowptr, colidx)
    interior = np.zeros(max(n, 1), dtype=np.int32)
    ln = np.zeros(1, dtype=np.int32)
    _check(_load().or_sample_path_uv(n, m, _ptr(rowptr, ctypes.c_int32), _ptr(colidx, ctypes.c_int32),
                                     seed, j, u, v, _ptr(interior, ctypes.c_int32),
                                     _ptr(ln, ctypes.c_int32)), "sample_path_uv")
    L = int(ln[0])
    return None if L < 0 else [int(x) for x in interior[:L]]


def sample_path_given(rowptr, colidx, u: int, v: int, given, with_keys: bool = False):
    """(interior, ranges[, keys]): the path the sampler yields for the pair
    (u, v) when its random choices are the values `given` (in the order the
    sample requests them; missing ones are 0) instead of generator draws,
    the range N of every choice it requested and, with_keys, the generator
    index (stream, t) each choice stands for.  interior is None when v is
    unreachable from u."""
    n, m, rowptr, colidx = _graph_args(rowptr, colidx)
    giv = np.ascontiguousarray(np.asarray(given, dtype=np.uint64).reshape(-1))
    if giv.size == 0:
        giv = np.zeros(1, dtype=np.uint64)
        ng = 0
    else:
        ng = int(giv.size)
    cap = 4 * max(n, 1) + 8
    ranges = np.zeros(cap, dtype=np.uint64)
    keys = np.zeros(cap, dtype=np.uint64)
    out = np.zeros(max(n, 1), dtype=np.int32)
    used = ctypes.c_int32(0)
    ln = ctypes.c_int32(0)
    _check(_load().or_sample_path_given(n, m, _ptr(rowptr, ctypes.c_int32), _ptr(colidx, ctypes.c_int32), int(u),
                                        int(v), _ptr(giv, ctypes.c_uint64), ng, _ptr(ranges, ctypes.c_uint64),
                                        _ptr(keys, ctypes.c_uint64), cap, ctypes.byref(used),
                                        _ptr(out, ctypes.c_int32), ctypes.byref(ln)),
           "sample_path_given")
    k = min(used.value, cap)
    rng = [int(x) for x in ranges[:k]]
    interior = None if ln.value < 0 else [int(x) for x in out[:ln.value]]
    if with_keys:
        return interior, rng, [(int(x) >> 32, int(x) & 0xFFFFFFFF) for x in keys[:k]]
    return interior, rng


def pair_counts(rowptr, colidx, r: int, seed: int, nthreads: int = 1) -> np.ndarray:
    """Samples 0 .. r-1 of the pair sequence `seed`: cnt[v] = samples whose
    path has v inside (nthreads: contiguous blocks of samples, summed)."""
    n, m, rowptr, colidx = _graph_args(rowptr, colidx)
    cnt = np.zeros(max(n, 1), dtype=np.uint32)
    _check(_load().or_pair_counts(n, m, _ptr(rowptr, ctypes.c_int32), _ptr(colidx, ctypes.c_int32),
                                  r, seed, _ptr(cnt, ctypes.c_uint32), int(nthreads)), "pair_counts")
    return cnt[:n]


def pair_sample(rowptr, colidx, eps: float, delta: float, seed: int):
    """(bc estimate on the ordered-pair scale, counts, r, VD bound)."""
    n, m, rowptr, colidx = _graph_args(rowptr, colidx)
    cnt = np.zeros(max(n, 1), dtype=np.uint32)
    bc = np.zeros(max(n, 1), dtype=np.float64)
    r = np.zeros(1, dtype=np.int64)
    vd = np.zeros(1, dtype=np.int32)
    _check(_load().or_pair_sample(n, m, _ptr(rowptr, ctypes.c_int32), _ptr(colidx, ctypes.c_int32),
                                  eps, delta, seed, _ptr(cnt, ctypes.c_uint32), _ptr(bc, ctypes.c_double),
                                  _ptr(r, ctypes.c_int64), _ptr(vd, ctypes.c_int32)), "pair_sample")
    return bc[:n], cnt[:n], int(r[0]), int(vd[0])
