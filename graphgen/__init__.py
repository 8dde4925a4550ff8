"""Seeded synthetic inputs: random-graph models, closed-form families and a
CSR builder.

This module holds inputs only (no shortest-path or centrality arithmetic).
Both the CPU oracle's tests and the GPU path's tests and benchmark take their
graphs and source lists from here.

Every random draw goes through the counter-based SplitMix64 construction in
``gen.c`` (``gg_draw``), so a (model, parameters, seed) triple fixes the graph
bit for bit on any machine with the same C library.

All CSR graphs are undirected and simple: ``rowptr`` int32[n+1],
``colidx`` int32[m] with m = rowptr[n] arcs (each edge stored twice), each
adjacency list sorted ascending, no self-loops, no duplicates.
"""
from __future__ import annotations

import ctypes
import hashlib
import math
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "gen.c")
# NK_SANITIZE=1 selects a build instrumented with AddressSanitizer and
# UndefinedBehaviorSanitizer (the host process must preload the ASan runtime)
_SANITIZE = os.environ.get("NK_SANITIZE") == "1"
_LIB_PATH = os.path.join(_HERE, "libgraphgen_san.so" if _SANITIZE else "libgraphgen.so")
_SAN_FLAGS = ["-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined", "-fno-sanitize-recover=all"]
_lib = None


def build(force: bool = True) -> str:
    """Compile gen.c into libgraphgen.so next to it."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp%d" % os.getpid()
        opt = _SAN_FLAGS if _SANITIZE else ["-O2"]
        subprocess.check_call(["gcc"] + opt + ["-fPIC", "-shared", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        build(force=False)
    lib = ctypes.CDLL(_LIB_PATH)
    i32p = ctypes.POINTER(ctypes.c_int32)
    lib.gg_draw.restype = ctypes.c_uint64
    lib.gg_draw.argtypes = [ctypes.c_uint64] * 4
    lib.gg_er.restype = ctypes.c_int
    lib.gg_er.argtypes = [ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64, i32p, i32p]
    lib.gg_rmat.restype = ctypes.c_int
    lib.gg_rmat.argtypes = [ctypes.c_int32, ctypes.c_int64, ctypes.c_double, ctypes.c_double,
                            ctypes.c_double, ctypes.c_uint64, i32p, i32p]
    lib.gg_chung_lu.restype = ctypes.c_int64
    lib.gg_chung_lu.argtypes = [ctypes.c_int32, ctypes.c_double, ctypes.c_double, ctypes.c_uint64,
                                i32p, i32p, ctypes.c_int64]
    lib.gg_ba.restype = ctypes.c_int
    lib.gg_ba.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_uint64, i32p, i32p]
    lib.gg_sample_sources.restype = ctypes.c_int
    lib.gg_sample_sources.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.c_uint64, i32p]
    lib.gg_bounded_draws.restype = ctypes.c_int
    lib.gg_bounded_draws.argtypes = [ctypes.c_uint64, ctypes.c_uint64, ctypes.POINTER(ctypes.c_int64),
                                     ctypes.c_int64, ctypes.c_uint64, i32p]
    lib.gg_csr.restype = ctypes.c_int64
    lib.gg_csr.argtypes = [ctypes.c_int32, ctypes.c_int64, i32p, i32p, i32p, i32p]
    _lib = lib
    return lib


def _p(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int32))


@dataclass
class Graph:
    """Undirected simple graph in CSR form (host arrays)."""
    n: int
    rowptr: np.ndarray
    colidx: np.ndarray
    name: str = ""

    @property
    def m(self) -> int:
        """Number of stored arcs (twice the number of undirected edges)."""
        return int(self.rowptr[-1]) if self.n > 0 else 0

    @property
    def m_undirected(self) -> int:
        return self.m // 2

    def degrees(self) -> np.ndarray:
        return np.diff(self.rowptr.astype(np.int64))

    def sha256(self) -> str:
        h = hashlib.sha256()
        h.update(np.int64(self.n).tobytes())
        h.update(np.ascontiguousarray(self.rowptr, dtype=np.int32).tobytes())
        h.update(np.ascontiguousarray(self.colidx, dtype=np.int32).tobytes())
        return h.hexdigest()

    def edges(self):
        """Undirected edge list (u < v) as two int64 arrays."""
        src = np.repeat(np.arange(self.n, dtype=np.int64), self.degrees())
        dst = self.colidx.astype(np.int64)
        keep = src < dst
        return src[keep], dst[keep]


def draw(seed: int, stream: int, j: int, t: int) -> int:
    """The counter-based 64-bit draw used by every generator."""
    return int(_load().gg_draw(seed, stream, j, t))


def from_edges(n: int, u, v, name: str = "") -> Graph:
    """Symmetric, sorted, deduplicated CSR from an edge list (self-loops dropped)."""
    u = np.ascontiguousarray(np.asarray(u, dtype=np.int32))
    v = np.ascontiguousarray(np.asarray(v, dtype=np.int32))
    if u.shape != v.shape:
        raise ValueError("edge arrays differ in length")
    ne = int(u.shape[0])
    rowptr = np.zeros(n + 1, dtype=np.int32)
    colidx = np.zeros(max(2 * ne, 1), dtype=np.int32)
    m = _load().gg_csr(n, ne, _p(u), _p(v), _p(rowptr), _p(colidx))
    if m < 0:
        raise ValueError("edge list has a vertex id outside [0, n) or too many arcs")
    return Graph(n, rowptr, colidx[:m].copy(), name)


def directed_from_arcs(n: int, u, v, name: str = "") -> Graph:
    """Directed CSR of out-arcs from an arc list u[i] -> v[i]: rows sorted,
    duplicates and self-loops dropped, no symmetrisation."""
    u = np.asarray(u, dtype=np.int64)
    v = np.asarray(v, dtype=np.int64)
    if u.shape != v.shape:
        raise ValueError("arc arrays differ in length")
    if u.size and (u.min() < 0 or v.min() < 0 or u.max() >= n or v.max() >= n):
        raise ValueError("arc list has a vertex id outside [0, n)")
    keep = u != v
    key = np.unique(u[keep] * n + v[keep])
    rowptr = np.zeros(n + 1, dtype=np.int32)
    if n > 0:
        np.cumsum(np.bincount(key // n, minlength=n), out=rowptr[1:])
    return Graph(n, rowptr, (key % n).astype(np.int32), name)


def transpose(g: Graph) -> Graph:
    """In-arc CSR of a directed graph (rows sorted)."""
    src = np.repeat(np.arange(g.n, dtype=np.int64), g.degrees())
    return directed_from_arcs(g.n, g.colidx, src, g.name + "_T")


def directed_rmat(scale: int, edge_factor: int, seed: int, a=0.57, b=0.19, c=0.19) -> Graph:
    """R-MAT arcs taken as directed (first draw -> second draw), not
    symmetrised: skewed out- and in-degrees, many vertices reachable from few."""
    n = 1 << scale
    ne = edge_factor * n
    u = np.zeros(ne, dtype=np.int32)
    v = np.zeros(ne, dtype=np.int32)
    if _load().gg_rmat(scale, ne, a, b, c, seed, _p(u), _p(v)) != 0:
        raise ValueError("bad R-MAT parameters")
    return directed_from_arcs(n, u, v, f"drmat_s{scale}_ef{edge_factor}_s{seed}")


def directed_random(n: int, m: int, seed: int) -> Graph:
    """m arcs with independent uniform endpoints (counter draws on stream
    90), then deduplicated: a directed G(n, p)-like graph."""
    u = np.array([(draw(seed, 90, i, 0) * n) >> 64 for i in range(m)], dtype=np.int64)
    v = np.array([(draw(seed, 90, i, 1) * n) >> 64 for i in range(m)], dtype=np.int64)
    return directed_from_arcs(n, u, v, f"dgnm_n{n}_m{m}_s{seed}")


def edge_weights(g: Graph, wmax: int, seed: int, symmetric: bool = True) -> np.ndarray:
    """int32 weight per arc, uniform in [1, wmax] from counter draws (stream
    91) keyed by the edge {u, v} (both arcs equal: an undirected weighted
    graph) or, with symmetric=False, by the arc index."""
    src = np.repeat(np.arange(g.n, dtype=np.int64), g.degrees())
    dst = g.colidx.astype(np.int64)
    key = np.minimum(src, dst) * g.n + np.maximum(src, dst) if symmetric else np.arange(g.m, dtype=np.int64)
    if g.m == 0:
        return np.zeros(0, dtype=np.int32)
    uniq, inv = np.unique(key, return_inverse=True)
    uniq = np.ascontiguousarray(uniq, dtype=np.int64)
    w = np.zeros(uniq.shape[0], dtype=np.int32)
    if _load().gg_bounded_draws(seed, 91, uniq.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)), uniq.shape[0],
                                wmax, _p(w)) != 0:
        raise ValueError("bad weight range")
    return (w[inv] + 1).astype(np.int32)


# ---------------------------------------------------------------- models --

def erdos_renyi(n: int, m: int, seed: int) -> Graph:
    """G(n, m): m distinct edges drawn uniformly, no self-loops."""
    u = np.zeros(max(m, 1), dtype=np.int32)
    v = np.zeros(max(m, 1), dtype=np.int32)
    if _load().gg_er(n, m, seed, _p(u), _p(v)) != 0:
        raise ValueError("bad G(n,m) parameters")
    return from_edges(n, u[:m], v[:m], f"er_n{n}_m{m}_s{seed}")


def rmat(scale: int, edge_factor: int, seed: int, a=0.57, b=0.19, c=0.19) -> Graph:
    """R-MAT with 2**scale vertices and edge_factor * 2**scale generated edges."""
    n = 1 << scale
    ne = edge_factor * n
    u = np.zeros(ne, dtype=np.int32)
    v = np.zeros(ne, dtype=np.int32)
    if _load().gg_rmat(scale, ne, a, b, c, seed, _p(u), _p(v)) != 0:
        raise ValueError("bad R-MAT parameters")
    return from_edges(n, u, v, f"rmat_s{scale}_ef{edge_factor}_s{seed}")


def chung_lu(n: int, gamma: float, mean_deg: float, seed: int) -> Graph:
    """Chung-Lu power-law graph with exponent gamma and the given mean expected degree."""
    cap = int(n * mean_deg * 0.6) + 1024
    for _ in range(3):
        u = np.zeros(cap, dtype=np.int32)
        v = np.zeros(cap, dtype=np.int32)
        got = _load().gg_chung_lu(n, gamma, mean_deg, seed, _p(u), _p(v), cap)
        if got == -1 and n < 1:
            raise ValueError("bad Chung-Lu parameters")
        if got >= 0:
            return from_edges(n, u[:got], v[:got], f"chunglu_n{n}_g{gamma}_d{mean_deg}_s{seed}")
        cap = -got + 16
    raise RuntimeError("Chung-Lu buffer sizing failed")


def barabasi_albert(n: int, m0: int, seed: int) -> Graph:
    """Preferential attachment with m0 edges per new vertex, from K_{m0+1}."""
    ne = (m0 + 1) * m0 // 2 + (n - m0 - 1) * m0
    u = np.zeros(ne, dtype=np.int32)
    v = np.zeros(ne, dtype=np.int32)
    if _load().gg_ba(n, m0, seed, _p(u), _p(v)) != 0:
        raise ValueError("bad BA parameters")
    return from_edges(n, u, v, f"ba_n{n}_m{m0}_s{seed}")


def sample_sources(n: int, k: int, seed: int) -> np.ndarray:
    """k distinct vertices of [0, n), uniformly, by partial Fisher-Yates."""
    out = np.zeros(max(k, 1), dtype=np.int32)
    if _load().gg_sample_sources(n, k, seed, _p(out)) != 0:
        raise ValueError("k must lie in [0, n]")
    return out[:k].copy()


# ------------------------------------------------------ closed-form families --

def path(n: int) -> Graph:
    i = np.arange(max(n - 1, 0))
    return from_edges(n, i, i + 1, f"path{n}")


def star(n: int) -> Graph:
    """Centre 0 and n-1 leaves."""
    i = np.arange(1, n)
    return from_edges(n, np.zeros_like(i), i, f"star{n}")


def cycle(n: int) -> Graph:
    i = np.arange(n)
    return from_edges(n, i, (i + 1) % n, f"cycle{n}")


def complete(n: int) -> Graph:
    u, v = np.triu_indices(n, 1)
    return from_edges(n, u, v, f"K{n}")


def complete_bipartite(a: int, b: int) -> Graph:
    """Side A = [0, a), side B = [a, a+b)."""
    u, v = np.meshgrid(np.arange(a), np.arange(a, a + b), indexing="ij")
    return from_edges(a + b, u.ravel(), v.ravel(), f"K{a},{b}")


def grid(rows: int, cols: int) -> Graph:
    """rows x cols lattice; vertex (i, j) has id i*cols + j."""
    idx = np.arange(rows * cols).reshape(rows, cols)
    u = np.concatenate([idx[:, :-1].ravel(), idx[:-1, :].ravel()])
    v = np.concatenate([idx[:, 1:].ravel(), idx[1:, :].ravel()])
    return from_edges(rows * cols, u, v, f"grid{rows}x{cols}")


def hypercube(d: int) -> Graph:
    n = 1 << d
    us, vs = [], []
    for bit in range(d):
        i = np.arange(n)
        keep = (i >> bit) & 1 == 0
        us.append(i[keep])
        vs.append(i[keep] | (1 << bit))
    if d == 0:
        return from_edges(1, [], [], "Q0")
    return from_edges(n, np.concatenate(us), np.concatenate(vs), f"Q{d}")


def diamond_chain(k: int) -> Graph:
    """k 4-cycles glued in series: joints 0, 3, 6, ..., 3k; the two middle
    vertices of diamond i are 3i+1 and 3i+2.  End-to-end path count is 2**k."""
    n = 3 * k + 1
    us, vs = [], []
    for i in range(k):
        a, x, y, b = 3 * i, 3 * i + 1, 3 * i + 2, 3 * i + 3
        us += [a, a, x, y]
        vs += [x, y, b, b]
    return from_edges(n, us, vs, f"diamonds{k}")


def random_tree(n: int, seed: int) -> Graph:
    """Random recursive tree: vertex i > 0 attaches to a uniform earlier vertex."""
    lib = _load()
    parent = [0] * n
    for i in range(1, n):
        parent[i] = int((lib.gg_draw(seed, 70, i, 0) * i) >> 64)
    i = np.arange(1, n)
    return from_edges(n, np.array(parent[1:], dtype=np.int32), i, f"tree{n}_s{seed}")


def disjoint_union(graphs) -> Graph:
    us, vs, off = [], [], 0
    for g in graphs:
        a, b = g.edges()
        us.append(a + off)
        vs.append(b + off)
        off += g.n
    if not us:
        return from_edges(0, [], [], "empty")
    return from_edges(off, np.concatenate(us), np.concatenate(vs), "union")


# ------------------------------------------------------------- workloads --

def workload_er2000(seed: int = 1) -> Graph:
    """Erdos-Renyi G(2000, 10000), the exact all-sources workload."""
    return erdos_renyi(2000, 10000, seed)


def workload_rmat20(seed: int = 2):
    """R-MAT scale 20, 16 * 2**20 generated edges, (0.57, 0.19, 0.19, 0.05),
    and 4096 distinct uniform sources; scores are scaled by n / 4096."""
    g = rmat(20, 16, seed)
    src = sample_sources(g.n, 4096, seed)
    return g, src


def workload_chung_lu4m(seed: int = 3) -> Graph:
    """Chung-Lu, n = 4e6, exponent 2.5, mean expected degree 20."""
    return chung_lu(4_000_000, 2.5, 20.0, seed)


def batched_sizes(count: int, lo: int, hi: int, seed: int):
    """Vertex counts log-uniform in [lo, hi] for a batch of graphs."""
    out = []
    for g in range(count):
        x = (draw(seed, 60, g, 0) >> 11) * (1.0 / 9007199254740992.0)
        out.append(int(round(math.exp(math.log(lo) + x * (math.log(hi) - math.log(lo))))))
    return out


def workload_batched(count: int = 512, lo: int = 1000, hi: int = 200_000, seed: int = 4):
    """Half Erdos-Renyi (m = 4n, even index) and half Barabasi-Albert (m0 = 4,
    odd index) graphs with log-uniform sizes."""
    graphs = []
    for g, n in enumerate(batched_sizes(count, lo, hi, seed)):
        gs = draw(seed, 61, g, 0)
        if g % 2 == 0:
            graphs.append(erdos_renyi(n, 4 * n, gs))
        else:
            graphs.append(barabasi_albert(n, 4, gs))
    return graphs


def serving_pool(count: int = 64, seed: int = 5, rmat_scales=(14, 20), ba_range=(10_000, 1_000_000)):
    """Half R-MAT graphs with scale 14 + (i mod 7) (clipped to rmat_scales) and
    edge factor 16; half Barabasi-Albert with n log-uniform in ba_range."""
    pool = []
    half = count // 2
    lo_s, hi_s = rmat_scales
    span = hi_s - lo_s + 1
    sizes = batched_sizes(count - half, ba_range[0], ba_range[1], draw(seed, 62, 0, 0))
    for i in range(half):
        pool.append(rmat(lo_s + (i % span), 16, draw(seed, 63, i, 0)))
    for i, n in enumerate(sizes):
        pool.append(barabasi_albert(n, 4, draw(seed, 64, i, 0)))
    return pool


# --------------------------------------------------------- request streams --

REQUEST_KINDS = (("k", 64), ("k", 256), ("k", 1024), ("eps", 0.05), ("eps", 0.02))


def request_stream(count: int, qps: float, pool_sizes, seed: int = 5, kinds=REQUEST_KINDS, delta: float = 0.1):
    """A Poisson request stream over a graph pool: arrival times with
    exponential gaps of mean 1/qps, graph uniform over the pool, kind uniform
    over `kinds` (k sampled sources, or pair sampling at a given epsilon), and
    a per-request seed.  Sources of k-requests are drawn here (distinct,
    uniform).  Request i uses draws (seed, 80, i, 0..3)."""
    out = []
    t = 0.0
    for i in range(count):
        u = ((draw(seed, 80, i, 0) >> 11) + 0.5) * (1.0 / 9007199254740992.0)
        t += -math.log(u) / qps
        g = int((draw(seed, 80, i, 1) * len(pool_sizes)) >> 64)
        kind, val = kinds[int((draw(seed, 80, i, 2) * len(kinds)) >> 64)]
        rseed = draw(seed, 80, i, 3)
        req = {"id": i, "t": t, "graph": g, "seed": rseed}
        n = pool_sizes[g]
        if kind == "k":
            req["sources"] = sample_sources(n, min(int(val), n), rseed)
        else:
            req["eps"] = float(val)
            req["delta"] = delta
        out.append(req)
    return out
