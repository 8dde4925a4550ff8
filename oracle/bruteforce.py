"""Exact betweenness by enumerating every simple path -- TEST INFRASTRUCTURE ONLY.

For graphs of at most a dozen vertices.  For each ordered pair (s, t),
s != t, a depth-first search lists all simple s-t paths; the shortest ones
give d(s, t) and sigma(s, t), and each interior vertex v of a shortest path
gets 1 / sigma(s, t).  This is the definition of betweenness the paper
relies on (shortest paths through a node, section "Heuristics and
Approximation Algorithms"), evaluated in exact rationals with no shortcut
that Brandes' algorithm takes.
"""
from __future__ import annotations

from fractions import Fraction


def _adjacency(rowptr, colidx):
    n = len(rowptr) - 1
    return [[int(colidx[e]) for e in range(int(rowptr[v]), int(rowptr[v + 1]))] for v in range(n)]


def all_pairs_paths(rowptr, colidx):
    """dict (s, t) -> list of shortest simple s-t paths (vertex tuples)."""
    adj = _adjacency(rowptr, colidx)
    n = len(adj)
    out = {}
    for s in range(n):
        paths_to = {t: [] for t in range(n)}
        stack = [(s, (s,), {s})]
        while stack:
            v, p, seen = stack.pop()
            if v != s:
                paths_to[v].append(p)
            for w in adj[v]:
                if w not in seen:
                    stack.append((w, p + (w,), seen | {w}))
        for t in range(n):
            if t == s or not paths_to[t]:
                continue
            best = min(len(p) for p in paths_to[t])
            out[(s, t)] = [p for p in paths_to[t] if len(p) == best]
    return out


def brute_force(rowptr, colidx):
    """(d, sigma, bc): d[s][t] (-1 unreachable, 0 on the diagonal),
    sigma[s][t] (1 on the diagonal), bc[v] as exact Fractions over ordered pairs."""
    n = len(rowptr) - 1
    paths = all_pairs_paths(rowptr, colidx)
    d = [[-1] * n for _ in range(n)]
    sigma = [[0] * n for _ in range(n)]
    bc = [Fraction(0)] * n
    for s in range(n):
        d[s][s] = 0
        sigma[s][s] = 1
    for (s, t), ps in paths.items():
        d[s][t] = len(ps[0]) - 1
        sigma[s][t] = len(ps)
        through = [0] * n
        for p in ps:
            for v in p[1:-1]:
                through[v] += 1
        for v in range(n):
            if through[v]:
                bc[v] += Fraction(through[v], len(ps))
    return d, sigma, bc


def linear_dependencies(rowptr, colidx, sources):
    """Sum over s in `sources` and every t != s of sigma_st(v) / sigma_st *
    d(s, v) / d(s, t), as exact Fractions: the linear-scaling estimator of
    Geisberger, Sanders and Schultes written out from its definition (each
    shortest s-t path through v weighted by v's relative distance from s)."""
    n = len(rowptr) - 1
    paths = all_pairs_paths(rowptr, colidx)
    out = [Fraction(0)] * n
    for s in sources:
        for t in range(n):
            ps = paths.get((s, t))
            if not ps:
                continue
            dst = len(ps[0]) - 1
            for p in ps:
                for pos, v in enumerate(p[1:-1], start=1):
                    out[v] += Fraction(pos, dst) / len(ps)
    return out


def bisection_dependencies(rowptr, colidx, sources):
    """Sum over s in `sources` and every t != s of sigma_st(v) / sigma_st
    weighted 1 when v is on the far half of the path (2 d(s, v) > d(s, t)),
    1/2 in its exact middle and 0 on the near half, as exact Fractions: the
    bisection estimator of Geisberger, Sanders and Schultes written out from
    its definition, path by path."""
    n = len(rowptr) - 1
    paths = all_pairs_paths(rowptr, colidx)
    out = [Fraction(0)] * n
    for s in sources:
        for t in range(n):
            ps = paths.get((s, t))
            if not ps:
                continue
            dst = len(ps[0]) - 1
            for p in ps:
                for pos, v in enumerate(p[1:-1], start=1):
                    if 2 * pos > dst:
                        out[v] += Fraction(1, len(ps))
                    elif 2 * pos == dst:
                        out[v] += Fraction(1, 2 * len(ps))
    return out


def edge_betweenness(rowptr, colidx):
    """dict {(u, v): Fraction} with u < v: over ordered pairs (s, t), the
    share of shortest s-t paths that use the edge {u, v}."""
    paths = all_pairs_paths(rowptr, colidx)
    out = {}
    n = len(rowptr) - 1
    for u in range(n):
        for e in range(int(rowptr[u]), int(rowptr[u + 1])):
            v = int(colidx[e])
            if u < v:
                out[(u, v)] = Fraction(0)
    for (s, t), ps in paths.items():
        for p in ps:
            for a, b in zip(p[:-1], p[1:]):
                out[(min(a, b), max(a, b))] += Fraction(1, len(ps))
    return out


def brute_force_weighted(rowptr, colidx, weights):
    """(d, sigma, bc) with arc weights: every simple s-t path is listed, the
    minimum weight sum is d(s, t), the paths reaching it are the shortest
    ones; bc[v] over ordered pairs as exact Fractions."""
    n = len(rowptr) - 1
    adj = [[(int(colidx[e]), int(weights[e])) for e in range(int(rowptr[v]), int(rowptr[v + 1]))] for v in range(n)]
    d = [[-1] * n for _ in range(n)]
    sigma = [[0] * n for _ in range(n)]
    bc = [Fraction(0)] * n
    for s in range(n):
        d[s][s] = 0
        sigma[s][s] = 1
        found = {t: [] for t in range(n)}
        stack = [(s, (s,), 0, {s})]
        while stack:
            v, p, wsum, seen = stack.pop()
            if v != s:
                found[v].append((wsum, p))
            for x, w in adj[v]:
                if x not in seen:
                    stack.append((x, p + (x,), wsum + w, seen | {x}))
        for t in range(n):
            if t == s or not found[t]:
                continue
            best = min(ws for ws, _ in found[t])
            ps = [p for ws, p in found[t] if ws == best]
            d[s][t] = best
            sigma[s][t] = len(ps)
            for p in ps:
                for v in p[1:-1]:
                    bc[v] += Fraction(1, len(ps))
    return d, sigma, bc
