/*
 * CPU ORACLE -- TEST INFRASTRUCTURE ONLY.
 *
 * Plain, sequential Brandes betweenness for undirected, unweighted graphs in
 * CSR form, written to be checked by eye against the method the paper uses
 * (Brandes 2001, cited in the section "Heuristics and Approximation
 * Algorithms" and in Table 1, "betweenness", O(nm) time).  Only the test
 * suite, the smoke check and the CPU-baseline leg of the benchmark may load
 * it; the GPU library neither links nor calls it.
 *
 * Forms:
 *   - exact: sum of dependencies over all sources (Table 1, "betweenness");
 *   - source set: sum over a given source list times a scale factor
 *     (Table 1, "ap. betweenness", sampling shortest-path trees);
 *   - the linear-scaling and bisection source-set estimators of
 *     Geisberger, Sanders and Schultes (the reference cited for that
 *     sampling);
 *   - directed graphs (out-arc CSR) for the exact and source-set forms;
 *   - positive integer arc weights (Dijkstra instead of breadth-first
 *     search) for the exact and source-set forms;
 *   - edge betweenness (section "Edge Centrality, Sparsification and Link
 *     Prediction");
 *   - closeness, exact and sampled (Table 1, "closeness", "ap. closeness");
 *   - pair sampling (Riondato and Kornaropoulos, cited for the epsilon
 *     guarantee in "Heuristics and Approximation Algorithms").
 *
 * Conventions (the paper is silent on these; each is a stated reading):
 *   - scores sum over ordered (s, t) pairs, endpoints excluded;
 *   - sigma is uint64 and any addition that wraps is reported as
 *     OR_E_SIGMA_OVERFLOW (no saturation);
 *   - unreachable vertices have d = -1, sigma = 0 and add nothing;
 *   - scores are FP64.
 *
 * The multi-threaded timing mode splits the source list into contiguous
 * blocks, one per thread, each with private arrays, and adds the per-thread
 * score arrays in thread order at the end: the parallel pattern the paper
 * describes for its own implementation (per-thread dependency arrays summed
 * at the end).  Each source is still plain sequential Brandes.
 */
#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define OR_OK 0
#define OR_E_INVALID_ARG (-1)
#define OR_E_INVALID_GRAPH (-2)
#define OR_E_SIGMA_OVERFLOW (-3)
#define OR_E_NO_MEMORY (-4)

typedef struct {
    int32_t n;
    const int32_t *rowptr;
    const int32_t *colidx;
} graph_t;

/* Structural checks: rowptr[0] = 0, rowptr non-decreasing, rowptr[n] = m,
 * every column index in [0, n). */
int or_validate(int32_t n, int64_t m, const int32_t *rowptr, const int32_t *colidx) {
    if (n < 0 || m < 0) return OR_E_INVALID_ARG;
    if (n == 0) return OR_OK;
    if (!rowptr || (m > 0 && !colidx)) return OR_E_INVALID_ARG;
    if (rowptr[0] != 0) return OR_E_INVALID_GRAPH;
    for (int32_t i = 0; i < n; ++i)
        if (rowptr[i + 1] < rowptr[i]) return OR_E_INVALID_GRAPH;
    if ((int64_t)rowptr[n] != m) return OR_E_INVALID_GRAPH;
    for (int64_t e = 0; e < m; ++e)
        if (colidx[e] < 0 || colidx[e] >= n) return OR_E_INVALID_GRAPH;
    return OR_OK;
}

/* Simple-graph checks on top of or_validate: adjacency strictly ascending
 * (no duplicates), no self-loops, and every arc u->v has its reverse v->u. */
int or_validate_strict(int32_t n, int64_t m, const int32_t *rowptr, const int32_t *colidx) {
    int st = or_validate(n, m, rowptr, colidx);
    if (st != OR_OK) return st;
    for (int32_t u = 0; u < n; ++u) {
        for (int32_t e = rowptr[u]; e < rowptr[u + 1]; ++e) {
            int32_t v = colidx[e];
            if (v == u) return OR_E_INVALID_GRAPH;
            if (e > rowptr[u] && colidx[e - 1] >= v) return OR_E_INVALID_GRAPH;
            int found = 0;
            for (int32_t f = rowptr[v]; f < rowptr[v + 1]; ++f)
                if (colidx[f] == u) { found = 1; break; }
            if (!found) return OR_E_INVALID_GRAPH;
        }
    }
    return OR_OK;
}

/*
 * Forward phase of Brandes' algorithm from source s: breadth-first search
 * that records the distance d and the number of shortest paths sigma of
 * every vertex, and the visit order S (non-decreasing distance).
 * Returns OR_OK or OR_E_SIGMA_OVERFLOW.  d must be -1 and sigma 0 on entry.
 */
static int forward(const graph_t *g, int32_t s, int32_t *d, uint64_t *sigma,
                   int32_t *S, int32_t *nS, int32_t *queue) {
    int32_t head = 0, tail = 0, ns = 0;
    int status = OR_OK;
    d[s] = 0;
    sigma[s] = 1;
    queue[tail++] = s;
    while (head < tail) {
        int32_t v = queue[head++];
        S[ns++] = v;
        for (int32_t e = g->rowptr[v]; e < g->rowptr[v + 1]; ++e) {
            int32_t w = g->colidx[e];
            if (d[w] < 0) {
                d[w] = d[v] + 1;
                queue[tail++] = w;
            }
            if (d[w] == d[v] + 1) {
                uint64_t sum;
                if (__builtin_add_overflow(sigma[w], sigma[v], &sum)) status = OR_E_SIGMA_OVERFLOW;
                sigma[w] = sum;
            }
        }
    }
    *nS = ns;
    return status;
}

typedef struct {
    int32_t *d, *S, *queue;
    uint64_t *sigma;
    double *delta;
} work_t;

static int work_alloc(work_t *w, int32_t n) {
    size_t nn = (size_t)(n > 0 ? n : 1);
    w->d = (int32_t *)malloc(nn * sizeof(int32_t));
    w->S = (int32_t *)malloc(nn * sizeof(int32_t));
    w->queue = (int32_t *)malloc(nn * sizeof(int32_t));
    w->sigma = (uint64_t *)malloc(nn * sizeof(uint64_t));
    w->delta = (double *)malloc(nn * sizeof(double));
    if (!w->d || !w->S || !w->queue || !w->sigma || !w->delta) return OR_E_NO_MEMORY;
    for (int32_t i = 0; i < n; ++i) { w->d[i] = -1; w->sigma[i] = 0; w->delta[i] = 0.0; }
    return OR_OK;
}

static void work_free(work_t *w) {
    free(w->d); free(w->S); free(w->queue); free(w->sigma); free(w->delta);
}

/* Restore d, sigma, delta of the vertices reached from the last source. */
static void work_reset(work_t *w, int32_t nS) {
    for (int32_t i = 0; i < nS; ++i) {
        int32_t v = w->S[i];
        w->d[v] = -1; w->sigma[v] = 0; w->delta[v] = 0.0;
    }
}

/*
 * One source of Brandes' algorithm: forward phase, then the dependency
 * accumulation in reverse visit order,
 *     delta[v] += sigma[v] / sigma[w] * (1 + delta[w])
 * for every predecessor v of w (d[v] = d[w] - 1), and bc[w] += delta[w]
 * for w != s.
 */
static int one_source(const graph_t *g, int32_t s, work_t *w, double *bc) {
    int32_t nS = 0;
    int status = forward(g, s, w->d, w->sigma, w->S, &nS, w->queue);
    if (status == OR_OK) {
        for (int32_t i = nS - 1; i >= 0; --i) {
            int32_t x = w->S[i];
            for (int32_t e = g->rowptr[x]; e < g->rowptr[x + 1]; ++e) {
                int32_t v = g->colidx[e];
                if (w->d[v] == w->d[x] - 1)
                    w->delta[v] += (double)w->sigma[v] / (double)w->sigma[x] * (1.0 + w->delta[x]);
            }
            if (x != s) bc[x] += w->delta[x];
        }
    }
    work_reset(w, nS);
    return status;
}

/*
 * One source of the linear-scaling estimator of Geisberger, Sanders and
 * Schultes (the "better approximation" the paper cites for betweenness from
 * sampled shortest-path trees, section "Heuristics and Approximation
 * Algorithms"): the pair (s, t) adds sigma_st(v) / sigma_st times the
 * weight d(s, v) / d(s, t) to v.  Because the weight of t splits along the
 * shortest-path DAG as d(s,v)/d(s,w) * d(s,w)/d(s,t), the accumulation in
 * reverse visit order becomes
 *     delta[v] += sigma[v] / sigma[w] * d[v] / d[w] * (1 + delta[w])
 * for every predecessor v of w, and bc[w] += delta[w] for w != s.
 */
static int one_source_linear(const graph_t *g, int32_t s, work_t *w, double *bc) {
    int32_t nS = 0;
    int status = forward(g, s, w->d, w->sigma, w->S, &nS, w->queue);
    if (status == OR_OK) {
        for (int32_t i = nS - 1; i >= 0; --i) {
            int32_t x = w->S[i];
            for (int32_t e = g->rowptr[x]; e < g->rowptr[x + 1]; ++e) {
                int32_t v = g->colidx[e];
                if (w->d[v] == w->d[x] - 1)
                    w->delta[v] += (double)w->sigma[v] / (double)w->sigma[x] * ((double)w->d[v] / (double)w->d[x]) *
                                   (1.0 + w->delta[x]);
            }
            if (x != s) bc[x] += w->delta[x];
        }
    }
    work_reset(w, nS);
    return status;
}

/*
 * One source of the bisection estimator of the same Geisberger, Sanders and
 * Schultes paper: the pair (s, t) adds sigma_st(v) / sigma_st to v when v
 * lies on the far half of its shortest paths (2 d(s,v) > d(s,t)), half of
 * that when v is exactly in the middle (2 d(s,v) = d(s,t)), and nothing on
 * the near half.  Let D_T(v) be Brandes' dependency of v counting only the
 * targets at depth <= T.  Then v at depth l receives
 *     (D_{2l-1}(v) + D_{2l}(v)) / 2,
 * where D_T = D_L for T >= L, the depth of the deepest vertex.  Each D_T is
 * the plain accumulation in reverse visit order over the vertices at depth
 * <= T; every T = 1..L is computed over the whole tree and added to the
 * vertices whose depths select it.
 */
static int one_source_bisect(const graph_t *g, int32_t s, work_t *w, double *bc) {
    int32_t nS = 0;
    int status = forward(g, s, w->d, w->sigma, w->S, &nS, w->queue);
    if (status == OR_OK && nS > 1) {
        const int32_t L = w->d[w->S[nS - 1]];
        for (int32_t T = 1; T <= L; ++T) {
            for (int32_t i = 0; i < nS; ++i) w->delta[w->S[i]] = 0.0;
            for (int32_t i = nS - 1; i >= 0; --i) {
                int32_t x = w->S[i];
                if (w->d[x] > T) continue;
                for (int32_t e = g->rowptr[x]; e < g->rowptr[x + 1]; ++e) {
                    int32_t v = g->colidx[e];
                    if (w->d[v] == w->d[x] - 1)
                        w->delta[v] += (double)w->sigma[v] / (double)w->sigma[x] * (1.0 + w->delta[x]);
                }
            }
            for (int32_t i = 0; i < nS; ++i) {
                int32_t x = w->S[i];
                if (x == s) continue;
                const int32_t l = w->d[x];
                const int32_t t1 = 2 * l - 1 < L ? 2 * l - 1 : L, t2 = 2 * l < L ? 2 * l : L;
                double wt = 0.0;
                if (T == t1) wt += 0.5;
                if (T == t2) wt += 0.5;
                if (wt != 0.0) bc[x] += wt * w->delta[x];
            }
        }
    }
    work_reset(w, nS);
    return status;
}

/*
 * One source of Brandes' algorithm on a directed graph (the paper's graph
 * model allows directed edges, section "Graph data structure"; the
 * adjacency arrays hold out-arcs).  The forward phase follows out-arcs as
 * it is.  Predecessors of x are its in-neighbours, which the out-arc
 * arrays do not list, so the accumulation is written in the successor
 * form: in reverse visit order,
 *     delta[v] = sum over out-arcs v -> w with d[w] = d[v] + 1 of
 *                sigma[v] / sigma[w] * (1 + delta[w]),
 * every such w coming later in the visit order and so already final; then
 * bc[v] += delta[v] for v != s.
 */
static int one_source_directed(const graph_t *g, int32_t s, work_t *w, double *bc) {
    int32_t nS = 0;
    int status = forward(g, s, w->d, w->sigma, w->S, &nS, w->queue);
    if (status == OR_OK) {
        for (int32_t i = nS - 1; i >= 0; --i) {
            int32_t v = w->S[i];
            double acc = 0.0;
            for (int32_t e = g->rowptr[v]; e < g->rowptr[v + 1]; ++e) {
                int32_t x = g->colidx[e];
                if (w->d[x] == w->d[v] + 1)
                    acc += (double)w->sigma[v] / (double)w->sigma[x] * (1.0 + w->delta[x]);
            }
            w->delta[v] = acc;
            if (v != s) bc[v] += acc;
        }
    }
    work_reset(w, nS);
    return status;
}

/*
 * One source of Brandes' algorithm with edge dependencies (edge
 * betweenness, named in the section "Edge Centrality, Sparsification and
 * Link Prediction"): the shortest-path DAG arc v -> w carries
 *     c = sigma[v] / sigma[w] * (1 + delta[w]),
 * the share of shortest paths from s to w and beyond that use the edge
 * {v, w}.  c is added to delta[v] (as in one_source) and to the score slot
 * of the arc w -> v, which is the arc the accumulation scans; the two arcs
 * of an edge are summed after all sources.
 */
static int one_source_edge(const graph_t *g, int32_t s, work_t *w, double *bc, double *ebc) {
    int32_t nS = 0;
    int status = forward(g, s, w->d, w->sigma, w->S, &nS, w->queue);
    if (status == OR_OK) {
        for (int32_t i = nS - 1; i >= 0; --i) {
            int32_t x = w->S[i];
            for (int32_t e = g->rowptr[x]; e < g->rowptr[x + 1]; ++e) {
                int32_t v = g->colidx[e];
                if (w->d[v] == w->d[x] - 1) {
                    double c = (double)w->sigma[v] / (double)w->sigma[x] * (1.0 + w->delta[x]);
                    w->delta[v] += c;
                    ebc[e] += c;
                }
            }
            if (x != s && bc) bc[x] += w->delta[x];
        }
    }
    work_reset(w, nS);
    return status;
}

/* d (-1 = unreachable) and sigma of every vertex for one source. */
int or_sssp_counts(int32_t n, int64_t m, const int32_t *rowptr, const int32_t *colidx,
                   int32_t s, int32_t *d, uint64_t *sigma) {
    int st = or_validate(n, m, rowptr, colidx);
    if (st != OR_OK) return st;
    if (s < 0 || s >= n || !d || !sigma) return OR_E_INVALID_ARG;
    graph_t g = {n, rowptr, colidx};
    int32_t *S = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    int32_t *q = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    if (!S || !q) { free(S); free(q); return OR_E_NO_MEMORY; }
    for (int32_t i = 0; i < n; ++i) { d[i] = -1; sigma[i] = 0; }
    int32_t nS;
    st = forward(&g, s, d, sigma, S, &nS, q);
    free(S); free(q);
    return st;
}

/*
 * Weighted graphs (positive integer arc weights; the paper's graph model
 * carries edge weights).  Forward phase: Dijkstra's algorithm with a binary
 * heap of (distance, vertex) entries, stale entries skipped when popped.
 * A vertex is settled when popped with its final distance; its path count
 * is final then, since every predecessor has a smaller distance.  For each
 * out-arc v -> x of weight w: a shorter d(v) + w replaces d(x) and
 * sigma(x) = sigma(v); an equal one adds sigma(v).  S is the settle order.
 * Accumulation in reverse settle order, successor form (as for directed
 * graphs): delta(v) = sum over out-arcs v -> x with d(v) + w = d(x) of
 * sigma(v) / sigma(x) * (1 + delta(x)).
 */
typedef struct {
    int64_t d;
    int32_t v;
} heap_item_t;

static void heap_push(heap_item_t *h, int64_t *size, int64_t d, int32_t v) {
    int64_t i = (*size)++;
    h[i].d = d;
    h[i].v = v;
    while (i > 0) {
        int64_t p = (i - 1) / 2;
        if (h[p].d <= h[i].d) break;
        heap_item_t t = h[p]; h[p] = h[i]; h[i] = t;
        i = p;
    }
}

static heap_item_t heap_pop(heap_item_t *h, int64_t *size) {
    heap_item_t top = h[0];
    h[0] = h[--(*size)];
    int64_t i = 0;
    for (;;) {
        int64_t l = 2 * i + 1, r = l + 1, b = i;
        if (l < *size && h[l].d < h[b].d) b = l;
        if (r < *size && h[r].d < h[b].d) b = r;
        if (b == i) break;
        heap_item_t t = h[b]; h[b] = h[i]; h[i] = t;
        i = b;
    }
    return top;
}

/* d (-1 unreached), sigma and settle order S from s; heap holds m + 1 items. */
static int forward_weighted(const graph_t *g, const int32_t *wt, int32_t s, int64_t *d, uint64_t *sigma,
                            uint8_t *done, int32_t *S, int32_t *nS, heap_item_t *heap) {
    int status = OR_OK;
    int64_t size = 0;
    int32_t ns = 0;
    d[s] = 0;
    sigma[s] = 1;
    heap_push(heap, &size, 0, s);
    while (size > 0) {
        heap_item_t it = heap_pop(heap, &size);
        int32_t v = it.v;
        if (done[v] || it.d != d[v]) continue;
        done[v] = 1;
        S[ns++] = v;
        for (int32_t e = g->rowptr[v]; e < g->rowptr[v + 1]; ++e) {
            int32_t x = g->colidx[e];
            int64_t nd = d[v] + (int64_t)wt[e];
            if (d[x] < 0 || nd < d[x]) {
                d[x] = nd;
                sigma[x] = sigma[v];
                heap_push(heap, &size, nd, x);
            } else if (nd == d[x]) {
                uint64_t sum;
                if (__builtin_add_overflow(sigma[x], sigma[v], &sum)) status = OR_E_SIGMA_OVERFLOW;
                sigma[x] = sum;
            }
        }
    }
    *nS = ns;
    return status;
}

typedef struct {
    int64_t *d;
    uint64_t *sigma;
    double *delta;
    uint8_t *done;
    int32_t *S;
    heap_item_t *heap;
} wwork_t;

static int wwork_alloc(wwork_t *w, int32_t n, int64_t m) {
    size_t nn = (size_t)(n > 0 ? n : 1);
    w->d = (int64_t *)malloc(nn * sizeof(int64_t));
    w->sigma = (uint64_t *)malloc(nn * sizeof(uint64_t));
    w->delta = (double *)malloc(nn * sizeof(double));
    w->done = (uint8_t *)malloc(nn);
    w->S = (int32_t *)malloc(nn * sizeof(int32_t));
    w->heap = (heap_item_t *)malloc((size_t)(m + 1) * sizeof(heap_item_t));
    if (!w->d || !w->sigma || !w->delta || !w->done || !w->S || !w->heap) return OR_E_NO_MEMORY;
    for (int32_t i = 0; i < n; ++i) { w->d[i] = -1; w->sigma[i] = 0; w->delta[i] = 0.0; w->done[i] = 0; }
    return OR_OK;
}

static void wwork_free(wwork_t *w) {
    free(w->d); free(w->sigma); free(w->delta); free(w->done); free(w->S); free(w->heap);
}

static int one_source_weighted(const graph_t *g, const int32_t *wt, int32_t s, wwork_t *w, double *bc) {
    int32_t nS = 0;
    int status = forward_weighted(g, wt, s, w->d, w->sigma, w->done, w->S, &nS, w->heap);
    if (status == OR_OK) {
        for (int32_t i = nS - 1; i >= 0; --i) {
            int32_t v = w->S[i];
            double acc = 0.0;
            for (int32_t e = g->rowptr[v]; e < g->rowptr[v + 1]; ++e) {
                int32_t x = g->colidx[e];
                if (w->d[x] == w->d[v] + (int64_t)wt[e])
                    acc += (double)w->sigma[v] / (double)w->sigma[x] * (1.0 + w->delta[x]);
            }
            w->delta[v] = acc;
            if (v != s) bc[v] += acc;
        }
    }
    for (int32_t i = 0; i < nS; ++i) {
        int32_t v = w->S[i];
        w->d[v] = -1; w->sigma[v] = 0; w->delta[v] = 0.0; w->done[v] = 0;
    }
    return status;
}

static int weights_ok(int64_t m, const int32_t *wt) {
    for (int64_t e = 0; e < m; ++e)
        if (wt[e] < 1) return 0;
    return 1;
}

/* Weighted d (-1 unreachable) and sigma of every vertex for one source. */
int or_sssp_weighted(int32_t n, int64_t m, const int32_t *rowptr, const int32_t *colidx, const int32_t *wt,
                     int32_t s, int64_t *d, uint64_t *sigma) {
    int st = or_validate(n, m, rowptr, colidx);
    if (st != OR_OK) return st;
    if (m > 0 && (!wt || !weights_ok(m, wt))) return OR_E_INVALID_GRAPH;
    if (s < 0 || s >= n || !d || !sigma) return OR_E_INVALID_ARG;
    graph_t g = {n, rowptr, colidx};
    wwork_t w;
    if ((st = wwork_alloc(&w, n, m)) != OR_OK) { wwork_free(&w); return st; }
    int32_t nS;
    st = forward_weighted(&g, wt, s, w.d, w.sigma, w.done, w.S, &nS, w.heap);
    for (int32_t i = 0; i < n; ++i) { d[i] = w.d[i]; sigma[i] = w.sigma[i]; }
    wwork_free(&w);
    return st;
}

typedef struct {
    const graph_t *g;
    const int32_t *wt;
    const int32_t *src;
    int32_t lo, hi;
    int64_t m;
    double *bc;
    int status;
} wjob_t;

static void *run_wjob(void *arg) {
    wjob_t *j = (wjob_t *)arg;
    wwork_t w;
    j->status = wwork_alloc(&w, j->g->n, j->m);
    if (j->status == OR_OK)
        for (int32_t i = j->lo; i < j->hi; ++i) {
            int st = one_source_weighted(j->g, j->wt, j->src[i], &w, j->bc);
            if (st != OR_OK) { j->status = st; break; }
        }
    wwork_free(&w);
    return NULL;
}

int or_bc_weighted(int32_t n, int64_t m, const int32_t *rowptr, const int32_t *colidx, const int32_t *wt,
                   const int32_t *src, int32_t k, double scale, double *bc, int32_t nthreads);

enum { KIND_PLAIN = 0, KIND_LINEAR = 1, KIND_EDGE = 2, KIND_BISECT = 3, KIND_DIRECTED = 4 };

typedef struct {
    const graph_t *g;
    const int32_t *src;
    int32_t lo, hi;
    int kind;
    double *bc;
    double *ebc;   /* per-arc accumulators (KIND_EDGE) */
    int status;
} job_t;

static void *run_job(void *arg) {
    job_t *j = (job_t *)arg;
    work_t w;
    j->status = work_alloc(&w, j->g->n);
    if (j->status == OR_OK) {
        for (int32_t i = j->lo; i < j->hi; ++i) {
            int st;
            if (j->kind == KIND_LINEAR)
                st = one_source_linear(j->g, j->src[i], &w, j->bc);
            else if (j->kind == KIND_DIRECTED)
                st = one_source_directed(j->g, j->src[i], &w, j->bc);
            else if (j->kind == KIND_BISECT)
                st = one_source_bisect(j->g, j->src[i], &w, j->bc);
            else if (j->kind == KIND_EDGE)
                st = one_source_edge(j->g, j->src[i], &w, j->bc, j->ebc);
            else
                st = one_source(j->g, j->src[i], &w, j->bc);
            if (st != OR_OK) { j->status = st; break; }
        }
    }
    work_free(&w);
    return NULL;
}

/*
 * Runs one_source (or a variant) over the sources src[0..k) in the given
 * order (duplicates count twice).  nthreads <= 1 runs sequentially;
 * otherwise sources are split into contiguous blocks with private score
 * arrays per thread, summed in thread order.  bc (n) and ebc (m, KIND_EDGE
 * only) are overwritten with the unscaled sums.
 */
static int run_sources(const graph_t *g, int64_t m, const int32_t *src, int32_t k, int kind, double *bc,
                       double *ebc, int32_t nthreads) {
    const int32_t n = g->n;
    for (int32_t i = 0; i < n; ++i) bc[i] = 0.0;
    if (ebc)
        for (int64_t e = 0; e < m; ++e) ebc[e] = 0.0;
    if (n == 0 || k == 0) return OR_OK;
    int st;
    if (nthreads <= 1) {
        job_t j = {g, src, 0, k, kind, bc, ebc, OR_OK};
        run_job(&j);
        st = j.status;
    } else {
        if (nthreads > k) nthreads = k;
        job_t *jobs = (job_t *)calloc((size_t)nthreads, sizeof(job_t));
        pthread_t *th = (pthread_t *)calloc((size_t)nthreads, sizeof(pthread_t));
        if (!jobs || !th) { free(jobs); free(th); return OR_E_NO_MEMORY; }
        for (int32_t t = 0; t < nthreads; ++t) {
            jobs[t].g = g;
            jobs[t].src = src;
            jobs[t].lo = (int32_t)((int64_t)k * t / nthreads);
            jobs[t].hi = (int32_t)((int64_t)k * (t + 1) / nthreads);
            jobs[t].kind = kind;
            jobs[t].bc = (double *)calloc((size_t)n, sizeof(double));
            jobs[t].ebc = ebc ? (double *)calloc((size_t)(m > 0 ? m : 1), sizeof(double)) : NULL;
            jobs[t].status = (jobs[t].bc && (!ebc || jobs[t].ebc)) ? OR_OK : OR_E_NO_MEMORY;
        }
        char *started = (char *)calloc((size_t)nthreads, 1);
        for (int32_t t = 0; t < nthreads; ++t)
            if (started && jobs[t].status == OR_OK) started[t] = pthread_create(&th[t], NULL, run_job, &jobs[t]) == 0;
        for (int32_t t = 0; t < nthreads; ++t)
            if (started && started[t]) pthread_join(th[t], NULL);
            else if (jobs[t].status == OR_OK) jobs[t].status = OR_E_NO_MEMORY;
        free(started);
        st = OR_OK;
        for (int32_t t = 0; t < nthreads; ++t) {
            if (jobs[t].status != OR_OK && st == OR_OK) st = jobs[t].status;
            if (jobs[t].bc) {
                for (int32_t i = 0; i < n; ++i) bc[i] += jobs[t].bc[i];
                free(jobs[t].bc);
            }
            if (jobs[t].ebc) {
                for (int64_t e = 0; e < m; ++e) ebc[e] += jobs[t].ebc[e];
                free(jobs[t].ebc);
            }
        }
        free(jobs);
        free(th);
    }
    return st;
}

static int check_sources(int32_t n, const int32_t *src, int32_t k) {
    if (k < 0 || (k > 0 && !src)) return OR_E_INVALID_ARG;
    for (int32_t i = 0; i < k; ++i)
        if (src[i] < 0 || src[i] >= n) return OR_E_INVALID_ARG;
    return OR_OK;
}

/*
 * Betweenness summed over the sources src[0..k) in the given order
 * (duplicates count twice), then multiplied by `scale`.
 */
int or_bc_sources(int32_t n, int64_t m, const int32_t *rowptr, const int32_t *colidx,
                  const int32_t *src, int32_t k, double scale, double *bc, int32_t nthreads) {
    int st = or_validate(n, m, rowptr, colidx);
    if (st != OR_OK) return st;
    if ((st = check_sources(n, src, k)) != OR_OK) return st;
    if (n > 0 && !bc) return OR_E_INVALID_ARG;
    graph_t g = {n, rowptr, colidx};
    st = run_sources(&g, m, src, k, KIND_PLAIN, bc, NULL, nthreads);
    if (st == OR_OK && scale != 1.0)
        for (int32_t i = 0; i < n; ++i) bc[i] *= scale;
    return st;
}

/*
 * Linear-scaling estimator over the sources src[0..k): the sum of
 * one_source_linear dependencies times `scale`.  Summed over every vertex
 * as a source it is half of exact betweenness, so the unbiased estimate
 * from k sampled sources uses scale = 2 n / k.
 */
int or_bc_sources_linear(int32_t n, int64_t m, const int32_t *rowptr, const int32_t *colidx,
                         const int32_t *src, int32_t k, double scale, double *bc, int32_t nthreads) {
    int st = or_validate(n, m, rowptr, colidx);
    if (st != OR_OK) return st;
    if ((st = check_sources(n, src, k)) != OR_OK) return st;
    if (n > 0 && !bc) return OR_E_INVALID_ARG;
    graph_t g = {n, rowptr, colidx};
    st = run_sources(&g, m, src, k, KIND_LINEAR, bc, NULL, nthreads);
    if (st == OR_OK && scale != 1.0)
        for (int32_t i = 0; i < n; ++i) bc[i] *= scale;
    return st;
}

/*
 * Bisection estimator over the sources src[0..k): the sum of
 * one_source_bisect dependencies times `scale`.  Summed over every vertex
 * as a source it is half of exact betweenness, so the unbiased estimate
 * from k sampled sources uses scale = 2 n / k.
 */
int or_bc_sources_bisect(int32_t n, int64_t m, const int32_t *rowptr, const int32_t *colidx,
                         const int32_t *src, int32_t k, double scale, double *bc, int32_t nthreads) {
    int st = or_validate(n, m, rowptr, colidx);
    if (st != OR_OK) return st;
    if ((st = check_sources(n, src, k)) != OR_OK) return st;
    if (n > 0 && !bc) return OR_E_INVALID_ARG;
    graph_t g = {n, rowptr, colidx};
    st = run_sources(&g, m, src, k, KIND_BISECT, bc, NULL, nthreads);
    if (st == OR_OK && scale != 1.0)
        for (int32_t i = 0; i < n; ++i) bc[i] *= scale;
    return st;
}

/*
 * Directed betweenness over the sources src[0..k) (every vertex for exact
 * scores): the sum of one_source_directed dependencies times `scale`.
 * rowptr/colidx are out-arcs; no symmetry is required.
 */
int or_bc_directed(int32_t n, int64_t m, const int32_t *rowptr, const int32_t *colidx,
                   const int32_t *src, int32_t k, double scale, double *bc, int32_t nthreads) {
    int st = or_validate(n, m, rowptr, colidx);
    if (st != OR_OK) return st;
    if ((st = check_sources(n, src, k)) != OR_OK) return st;
    if (n > 0 && !bc) return OR_E_INVALID_ARG;
    graph_t g = {n, rowptr, colidx};
    st = run_sources(&g, m, src, k, KIND_DIRECTED, bc, NULL, nthreads);
    if (st == OR_OK && scale != 1.0)
        for (int32_t i = 0; i < n; ++i) bc[i] *= scale;
    return st;
}

/*
 * Weighted betweenness over the sources src[0..k) (every vertex for exact
 * scores) times `scale`: one_source_weighted per source; with nthreads > 1,
 * contiguous source blocks with private score arrays summed in thread
 * order, as run_sources does.
 */
int or_bc_weighted(int32_t n, int64_t m, const int32_t *rowptr, const int32_t *colidx, const int32_t *wt,
                   const int32_t *src, int32_t k, double scale, double *bc, int32_t nthreads) {
    int st = or_validate(n, m, rowptr, colidx);
    if (st != OR_OK) return st;
    if (m > 0 && (!wt || !weights_ok(m, wt))) return OR_E_INVALID_GRAPH;
    if ((st = check_sources(n, src, k)) != OR_OK) return st;
    if (n > 0 && !bc) return OR_E_INVALID_ARG;
    for (int32_t i = 0; i < n; ++i) bc[i] = 0.0;
    if (n == 0 || k == 0) return OR_OK;
    graph_t g = {n, rowptr, colidx};
    if (nthreads < 1) nthreads = 1;
    if (nthreads > k) nthreads = k;
    wjob_t *jobs = (wjob_t *)calloc((size_t)nthreads, sizeof(wjob_t));
    double *part = (double *)calloc((size_t)nthreads * (size_t)n, sizeof(double));
    pthread_t *th = (pthread_t *)calloc((size_t)nthreads, sizeof(pthread_t));
    if (!jobs || !part || !th) { free(jobs); free(part); free(th); return OR_E_NO_MEMORY; }
    for (int32_t t = 0; t < nthreads; ++t) {
        jobs[t].g = &g;
        jobs[t].wt = wt;
        jobs[t].src = src;
        jobs[t].lo = (int32_t)((int64_t)k * t / nthreads);
        jobs[t].hi = (int32_t)((int64_t)k * (t + 1) / nthreads);
        jobs[t].m = m;
        jobs[t].bc = part + (size_t)t * (size_t)n;
        if (nthreads == 1) run_wjob(&jobs[t]);
        else pthread_create(&th[t], NULL, run_wjob, &jobs[t]);
    }
    st = OR_OK;
    for (int32_t t = 0; t < nthreads; ++t) {
        if (nthreads > 1) pthread_join(th[t], NULL);
        if (jobs[t].status != OR_OK) st = jobs[t].status;
    }
    for (int32_t t = 0; t < nthreads; ++t)
        for (int32_t i = 0; i < n; ++i) bc[i] += part[(size_t)t * (size_t)n + i];
    free(jobs); free(part); free(th);
    if (st == OR_OK && scale != 1.0)
        for (int32_t i = 0; i < n; ++i) bc[i] *= scale;
    return st;
}

/*
 * Edge betweenness over the sources src[0..k): ebc[e] for the arc e = u->v
 * is the score of the undirected edge {u, v} -- the sum over the sources
 * and every target t of the share of shortest s-t paths using the edge --
 * times `scale`; both arcs of an edge hold the same value.  bc (optional)
 * receives the vertex scores of the same run, times `scale`.  Needs the
 * reverse of every arc (OR_E_INVALID_GRAPH otherwise).
 */
int or_edge_bc_sources(int32_t n, int64_t m, const int32_t *rowptr, const int32_t *colidx,
                       const int32_t *src, int32_t k, double scale, double *ebc, double *bc, int32_t nthreads) {
    int st = or_validate(n, m, rowptr, colidx);
    if (st != OR_OK) return st;
    if ((st = check_sources(n, src, k)) != OR_OK) return st;
    if (m > 0 && !ebc) return OR_E_INVALID_ARG;
    double *vb = bc ? bc : (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    if (!vb) return OR_E_NO_MEMORY;
    graph_t g = {n, rowptr, colidx};
    st = run_sources(&g, m, src, k, KIND_EDGE, vb, ebc, nthreads);
    if (!bc) free(vb);
    if (st != OR_OK) return st;
    /* an edge's score is the sum over its two arcs */
    for (int32_t u = 0; u < n; ++u) {
        for (int32_t e = rowptr[u]; e < rowptr[u + 1]; ++e) {
            int32_t v = colidx[e];
            if (v <= u) continue;
            int32_t r = -1;
            for (int32_t f = rowptr[v]; f < rowptr[v + 1]; ++f)
                if (colidx[f] == u) { r = f; break; }
            if (r < 0) return OR_E_INVALID_GRAPH;
            double tot = (ebc[e] + ebc[r]) * scale;
            ebc[e] = tot;
            ebc[r] = tot;
        }
    }
    if (bc && scale != 1.0)
        for (int32_t i = 0; i < n; ++i) bc[i] *= scale;
    return OR_OK;
}

/* Exact betweenness: every vertex is a source, in order 0..n-1. */
int or_bc_exact(int32_t n, int64_t m, const int32_t *rowptr, const int32_t *colidx,
                double *bc, int32_t nthreads) {
    if (n < 0) return OR_E_INVALID_ARG;
    int32_t *src = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    if (!src) return OR_E_NO_MEMORY;
    for (int32_t i = 0; i < n; ++i) src[i] = i;
    int st = or_bc_sources(n, m, rowptr, colidx, src, n, 1.0, bc, nthreads);
    free(src);
    return st;
}

/*
 * Work done by Brandes for a source list, summed over the sources:
 *   out[0] = reached vertices (source included),
 *   out[1] = arcs leaving reached vertices (sum of their degrees),
 *   out[2] = shortest-path DAG arcs (v -> w with d[w] = d[v] + 1),
 *   out[3] = sum over sources of the deepest level.
 */
int or_work_counts(int32_t n, int64_t m, const int32_t *rowptr, const int32_t *colidx,
                   const int32_t *src, int32_t k, int64_t *out) {
    int st = or_validate(n, m, rowptr, colidx);
    if (st != OR_OK) return st;
    graph_t g = {n, rowptr, colidx};
    work_t w;
    if (work_alloc(&w, n) != OR_OK) { work_free(&w); return OR_E_NO_MEMORY; }
    out[0] = out[1] = out[2] = out[3] = 0;
    for (int32_t i = 0; i < k; ++i) {
        int32_t nS;
        int s2 = forward(&g, src[i], w.d, w.sigma, w.S, &nS, w.queue);
        (void)s2;
        out[0] += nS;
        int32_t deepest = 0;
        for (int32_t q = 0; q < nS; ++q) {
            int32_t v = w.S[q];
            out[1] += rowptr[v + 1] - rowptr[v];
            if (w.d[v] > deepest) deepest = w.d[v];
            for (int32_t e = rowptr[v]; e < rowptr[v + 1]; ++e)
                if (w.d[colidx[e]] == w.d[v] + 1) out[2]++;
        }
        out[3] += deepest;
        work_reset(&w, nS);
    }
    work_free(&w);
    return OR_OK;
}

/* ------------------------------------------------------------------------
 * Closeness (Table 1, "closeness": a shortest-path search from each node;
 * "ap. closeness": Eppstein and Wang's sampling, cited there).
 *
 * Plain BFS distances from s; returns the number of vertices reached
 * (s included) and their distance sum. */
static int32_t bfs_farness(const graph_t *g, int32_t s, int32_t *d, int32_t *queue, int64_t *far) {
    int32_t head = 0, tail = 0;
    int64_t sum = 0;
    d[s] = 0;
    queue[tail++] = s;
    while (head < tail) {
        int32_t v = queue[head++];
        sum += d[v];
        for (int32_t e = g->rowptr[v]; e < g->rowptr[v + 1]; ++e) {
            int32_t w = g->colidx[e];
            if (d[w] < 0) { d[w] = d[v] + 1; queue[tail++] = w; }
        }
    }
    for (int32_t i = 0; i < tail; ++i) d[queue[i]] = -1;
    *far = sum;
    return tail;
}

/*
 * Exact closeness of every vertex, generalised to disconnected graphs:
 * with r the number of vertices reachable from v (v included) and F the sum
 * of their distances from v,
 *     C(v) = (r - 1) / (n - 1) * (r - 1) / F,   and C(v) = 0 when r = 1,
 * which is (n - 1) / F on a connected graph.
 */
int or_closeness(int32_t n, int64_t m, const int32_t *rowptr, const int32_t *colidx, double *out) {
    int st = or_validate(n, m, rowptr, colidx);
    if (st != OR_OK) return st;
    if (n == 0) return OR_OK;
    graph_t g = {n, rowptr, colidx};
    int32_t *d = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    int32_t *q = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    if (!d || !q) { free(d); free(q); return OR_E_NO_MEMORY; }
    for (int32_t i = 0; i < n; ++i) d[i] = -1;
    for (int32_t v = 0; v < n; ++v) {
        int64_t far;
        int32_t r = bfs_farness(&g, v, d, q, &far);
        out[v] = (r <= 1 || n <= 1) ? 0.0 : ((double)(r - 1) / (double)(n - 1)) * ((double)(r - 1) / (double)far);
    }
    free(d); free(q);
    return OR_OK;
}

/*
 * Eppstein-Wang sampled closeness: with the sources S (k of them),
 *     F(v) = n / k * sum over s in S of d(s, v)   (unreachable pairs add 0),
 *     C(v) = (n - 1) / F(v),  0 when no source reaches v (F = 0).
 * The distance sums are kept as exact integers; sums[v] (optional, k-sum of
 * distances) is returned for inspection.
 */
int or_closeness_approx(int32_t n, int64_t m, const int32_t *rowptr, const int32_t *colidx,
                        const int32_t *src, int32_t k, double *out, int64_t *sums) {
    int st = or_validate(n, m, rowptr, colidx);
    if (st != OR_OK) return st;
    if ((st = check_sources(n, src, k)) != OR_OK) return st;
    if (n == 0) return OR_OK;
    int32_t *d = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    int32_t *q = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    int64_t *acc = (int64_t *)calloc((size_t)n, sizeof(int64_t));
    if (!d || !q || !acc) { free(d); free(q); free(acc); return OR_E_NO_MEMORY; }
    for (int32_t i = 0; i < n; ++i) d[i] = -1;
    for (int32_t i = 0; i < k; ++i) {
        int32_t s = src[i], head = 0, tail = 0;
        d[s] = 0;
        q[tail++] = s;
        while (head < tail) {
            int32_t v = q[head++];
            acc[v] += d[v];
            for (int32_t e = rowptr[v]; e < rowptr[v + 1]; ++e) {
                int32_t w = colidx[e];
                if (d[w] < 0) { d[w] = d[v] + 1; q[tail++] = w; }
            }
        }
        for (int32_t t = 0; t < tail; ++t) d[q[t]] = -1;
    }
    for (int32_t v = 0; v < n; ++v) {
        double F = k > 0 ? (double)n / (double)k * (double)acc[v] : 0.0;
        out[v] = F > 0.0 ? (double)(n - 1) / F : 0.0;
        if (sums) sums[v] = acc[v];
    }
    free(d); free(q); free(acc);
    return OR_OK;
}

/* ------------------------------------------------------------------------
 * Pair sampling (Riondato and Kornaropoulos).
 *
 * Random numbers: the counter-based SplitMix64 construction
 * (Steele, Lea, Flood 2014).  mix64 is the SplitMix64 output function; the
 * k-th output of a stream seeded with x is mix64(x + k*GAMMA); a draw
 * indexed by (seed, stream, j, t) is output t+1 of the stream seeded with
 * output j+1 of the stream seeded with output stream+1 of the stream seeded
 * with `seed`.  bounded(x, N) = floor(x * N / 2^64).
 * ---------------------------------------------------------------------- */
#define GOLDEN 0x9E3779B97F4A7C15ULL

uint64_t or_mix64(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

uint64_t or_draw(uint64_t seed, uint64_t stream, uint64_t j, uint64_t t) {
    uint64_t a = or_mix64(seed + (stream + 1) * GOLDEN);
    uint64_t b = or_mix64(a + (j + 1) * GOLDEN);
    return or_mix64(b + (t + 1) * GOLDEN);
}

uint64_t or_bounded(uint64_t x, uint64_t N) {
    return (uint64_t)(((unsigned __int128)x * N) >> 64);
}

/* Plain BFS distances from s (d = -1 unreachable); returns eccentricity of
 * s within its component and the lowest-id vertex at that distance. */
static int32_t bfs_ecc(const graph_t *g, int32_t s, int32_t *d, int32_t *queue,
                       int32_t *far_vertex, int32_t *reached) {
    for (int32_t i = 0; i < g->n; ++i) d[i] = -1;
    int32_t head = 0, tail = 0;
    d[s] = 0;
    queue[tail++] = s;
    while (head < tail) {
        int32_t v = queue[head++];
        for (int32_t e = g->rowptr[v]; e < g->rowptr[v + 1]; ++e) {
            int32_t w = g->colidx[e];
            if (d[w] < 0) { d[w] = d[v] + 1; queue[tail++] = w; }
        }
    }
    int32_t ecc = 0, far = s;
    for (int32_t i = 0; i < tail; ++i) {
        int32_t v = queue[i];
        if (d[v] > ecc || (d[v] == ecc && v < far)) { ecc = d[v]; far = v; }
    }
    *far_vertex = far;
    *reached = tail;
    return ecc;
}

/*
 * Upper bound on the vertex diameter (number of vertices on a longest
 * shortest path), for the sample size of pair sampling.
 *   x0 = vertex of maximum degree, lowest id on ties;
 *   e1 = eccentricity of x0, a = lowest-id vertex at distance e1;
 *   e2 = eccentricity of a (double sweep; e2 + 1 is a lower bound);
 *   c0 = size of the component of x0; c2 = largest other component.
 * Within x0's component every shortest path has at most 2*e1 + 1 vertices
 * and at most c0; in any other component at most its size.  Hence
 *   VD_ub = max(min(2*e1 + 1, c0), c2).
 * info = {x0, e1, a, e2, vd_ub, vd_lb = e2 + 1, c0, c2}.
 */
int or_vd_bound(int32_t n, int64_t m, const int32_t *rowptr, const int32_t *colidx, int32_t *info) {
    int st = or_validate(n, m, rowptr, colidx);
    if (st != OR_OK) return st;
    if (n == 0) { for (int i = 0; i < 8; ++i) info[i] = 0; return OR_OK; }
    graph_t g = {n, rowptr, colidx};
    int32_t *d = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    int32_t *q = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
    if (!d || !q) { free(d); free(q); return OR_E_NO_MEMORY; }
    int32_t x0 = 0;
    for (int32_t v = 1; v < n; ++v)
        if (rowptr[v + 1] - rowptr[v] > rowptr[x0 + 1] - rowptr[x0]) x0 = v;
    int32_t a, c0, c_a;
    int32_t e1 = bfs_ecc(&g, x0, d, q, &a, &c0);
    int32_t far2;
    int32_t e2 = bfs_ecc(&g, a, d, q, &far2, &c_a);
    /* component sizes: label every component by BFS from its lowest vertex */
    int32_t c2 = 0;
    for (int32_t i = 0; i < n; ++i) d[i] = -1;
    int32_t comp = 0;
    for (int32_t s = 0; s < n; ++s) {
        if (d[s] >= 0) continue;
        int32_t head = 0, tail = 0;
        d[s] = comp;
        q[tail++] = s;
        int contains_x0 = (s == x0);
        while (head < tail) {
            int32_t v = q[head++];
            for (int32_t e = rowptr[v]; e < rowptr[v + 1]; ++e) {
                int32_t w = colidx[e];
                if (d[w] < 0) { d[w] = comp; q[tail++] = w; if (w == x0) contains_x0 = 1; }
            }
        }
        if (!contains_x0 && tail > c2) c2 = tail;
        ++comp;
    }
    int32_t ub = 2 * e1 + 1;
    if (ub > c0) ub = c0;
    if (c2 > ub) ub = c2;
    info[0] = x0; info[1] = e1; info[2] = a; info[3] = e2;
    info[4] = ub; info[5] = e2 + 1; info[6] = c0; info[7] = c2;
    free(d); free(q);
    return OR_OK;
}

/*
 * Riondato-Kornaropoulos sample size with constant c = 0.5:
 *   r = ceil( c / eps^2 * ( floor(log2(VD - 2)) + 1 + ln(1/delta) ) ),
 * with VD - 2 taken as at least 1.  floor(log2) is computed on integers.
 */
int64_t or_rk_sample_size(double eps, double delta, int32_t vd) {
    if (!(eps > 0.0 && eps < 1.0) || !(delta > 0.0 && delta < 1.0)) return -1;
    int64_t x = (int64_t)vd - 2;
    if (x < 1) x = 1;
    int32_t fl = 0;
    while ((x >> (fl + 1)) > 0) ++fl;
    double k = (double)(fl + 1) + (-log(delta));
    double rr = 0.5 / (eps * eps) * k;
    return (int64_t)ceil(rr);
}

/* Pair j: u uniform in [0, n), v uniform in [0, n) minus {u}. */
static void pair_of(uint64_t seed, int64_t j, int32_t n, int32_t *u, int32_t *v) {
    int32_t a = (int32_t)or_bounded(or_draw(seed, 1, (uint64_t)j, 0), (uint64_t)n);
    int32_t b = (int32_t)or_bounded(or_draw(seed, 2, (uint64_t)j, 0), (uint64_t)(n - 1));
    if (b >= a) b += 1;
    *u = a;
    *v = b;
}

/*
 * One side of the bidirectional search: distances d (-1 = not reached),
 * path counts sigma from the side's root, its visit order S with level
 * bounds lvl[0..depth+1].
 */
typedef struct {
    int32_t *d;
    uint64_t *sigma;
    int32_t *S;
    int32_t *lvl;     /* level l occupies S[lvl[l] .. lvl[l+1]) */
    int32_t depth;    /* deepest complete level */
    int64_t cost;     /* arcs leaving the deepest level */
} side_t;

/* Expands side x by one level: every arc y -> z out of level depth with z
 * not yet reached by x adds sigma[y] to sigma[z]; the new level lists the
 * new vertices in visit order.  Returns the number of new vertices, or -1
 * on a path-count overflow. */
static int32_t expand_level(const graph_t *g, side_t *x) {
    int32_t lo = x->lvl[x->depth], hi = x->lvl[x->depth + 1], tail = hi;
    int overflow = 0;
    for (int32_t i = lo; i < hi; ++i) {
        int32_t y = x->S[i];
        for (int32_t e = g->rowptr[y]; e < g->rowptr[y + 1]; ++e) {
            int32_t z = g->colidx[e];
            if (x->d[z] < 0) {
                x->d[z] = x->depth + 1;
                x->S[tail++] = z;
            }
            if (x->d[z] == x->depth + 1) {
                uint64_t sum;
                if (__builtin_add_overflow(x->sigma[z], x->sigma[y], &sum)) overflow = 1;
                x->sigma[z] = sum;
            }
        }
    }
    x->depth += 1;
    x->lvl[x->depth + 1] = tail;
    int64_t cost = 0;
    for (int32_t i = hi; i < tail; ++i) cost += g->rowptr[x->S[i] + 1] - g->rowptr[x->S[i]];
    x->cost = cost;
    return overflow ? -1 : tail - hi;
}

static void side_start(const graph_t *g, side_t *x, int32_t root) {
    x->d[root] = 0;
    x->sigma[root] = 1;
    x->S[0] = root;
    x->lvl[0] = 0;
    x->lvl[1] = 1;
    x->depth = 0;
    x->cost = g->rowptr[root + 1] - g->rowptr[root];
}

static void side_reset(side_t *x) {
    for (int32_t i = 0; i < x->lvl[x->depth + 1]; ++i) {
        x->d[x->S[i]] = -1;
        x->sigma[x->S[i]] = 0;
    }
}

/*
 * Where a sample's random choices come from.  Normally each choice is
 * bounded(draw(seed, stream, j, t), N): uniform on [0, N) up to the
 * multiply-shift bias.  For inspection the caller may instead give the
 * chosen values themselves, consumed in the order the sample asks for them
 * (meeting vertex, then the walk towards v, then the walk towards u); the
 * range N of every request is recorded, so that a test can enumerate every
 * outcome of a sample and weigh it exactly.
 */
typedef struct {
    uint64_t seed;
    int64_t j;
    const uint64_t *given;   /* NULL: the counter generator */
    int32_t ngiven;          /* values in `given`; later requests take 0 */
    int32_t used;            /* requests made so far */
    uint64_t *ranges;        /* inspection: N of each request (cap entries) */
    uint64_t *keys;          /* inspection: stream << 32 | t of each request */
    int32_t cap;
    int bad;                 /* a given value was outside its range */
} chooser_t;

static uint64_t choose(chooser_t *c, uint64_t stream, uint64_t t, uint64_t N) {
    if (!c->given) return or_bounded(or_draw(c->seed, stream, (uint64_t)c->j, t), N);
    int32_t i = c->used++;
    if (c->ranges && i < c->cap) c->ranges[i] = N;
    if (c->keys && i < c->cap) c->keys[i] = stream << 32 | t;
    uint64_t x = i < c->ngiven ? c->given[i] : 0;
    if (x >= N) { c->bad = 1; x = 0; }
    return x;
}

/* Walks from `from` to the side's root: at w (step t) chooses
 * r in [0, sigma[w]) (choice stream `stream`, index t) and takes the first
 * neighbour p one level closer to the root, in adjacency order, whose
 * running sigma sum exceeds r (so p has probability sigma[p] / sigma[w]).
 * Writes the vertices strictly between `from` and the root to out in walk
 * order and returns their number. */
static int32_t walk_to_root(const graph_t *g, const side_t *x, int32_t from, chooser_t *ch, uint64_t stream,
                            int32_t *out) {
    int32_t w = from, len = 0;
    uint64_t t = 0;
    while (x->d[w] > 0) {
        uint64_t r = choose(ch, stream, t, x->sigma[w]);
        uint64_t acc = 0;
        int32_t pick = -1;
        for (int32_t e = g->rowptr[w]; e < g->rowptr[w + 1]; ++e) {
            int32_t p = g->colidx[e];
            if (x->d[p] == x->d[w] - 1) {
                acc += x->sigma[p];
                if (acc > r) { pick = p; break; }
            }
        }
        if (x->d[pick] > 0) out[len++] = pick;
        w = pick;
        ++t;
    }
    return len;
}

static int cmp_i32(const void *a, const void *b) {
    int32_t x = *(const int32_t *)a, y = *(const int32_t *)b;
    return (x > y) - (x < y);
}

/*
 * One sample: a uniformly random shortest u-v path, found by a balanced
 * bidirectional breadth-first search with path counting.
 *
 * Search: side A grows from u, side B from v, one whole level at a time;
 * the side whose deepest level has fewer leaving arcs grows next (A on
 * ties).  The first time a new level of one side contains vertices already
 * reached by the other side, those vertices M are exactly the vertices at
 * distance d_A(z) from u on shortest u-v paths (every vertex of M has the
 * other side's deepest distance), and sigma_uv = sum over z in M of
 * sigma_A(z) * sigma_B(z).  A side whose new level is empty has exhausted
 * its component: v is unreachable.
 *
 * Path: z in M is taken with probability sigma_A(z) sigma_B(z) / sigma_uv
 * (the first z in increasing id order whose running weight sum exceeds a
 * choice in [0, sigma_uv), stream 4); then a walk from z to v on side B
 * (stream 5) and one from z to u on side A (stream 3), each choosing
 * predecessors in proportion to their path counts.  The walk factors
 * telescope to 1 / (sigma_A(z) sigma_B(z)), so every shortest path is drawn
 * with probability 1 / sigma_uv.
 *
 * Interior vertices are written from v's side towards u.  Returns their
 * number, -1 if v is unreachable, or OR_E_SIGMA_OVERFLOW - 100 when a path
 * count (or sigma_uv) reaches 2^64.
 */
static int32_t sample_one(const graph_t *g, chooser_t *ch, int32_t u, int32_t v, side_t *A, side_t *B,
                          int32_t *interior, int32_t *scratch) {
    side_start(g, A, u);
    side_start(g, B, v);
    int32_t result = -1;
    for (;;) {
        side_t *X = (A->cost <= B->cost) ? A : B;
        side_t *Y = (X == A) ? B : A;
        int32_t fresh = expand_level(g, X);
        if (fresh < 0) { result = OR_E_SIGMA_OVERFLOW - 100; break; }
        if (fresh == 0) { result = -1; break; }
        /* meeting vertices, in increasing id order */
        int32_t lo = X->lvl[X->depth], hi = X->lvl[X->depth + 1], nm = 0;
        for (int32_t i = lo; i < hi; ++i)
            if (Y->d[X->S[i]] >= 0) scratch[nm++] = X->S[i];
        if (nm == 0) continue;
        qsort(scratch, (size_t)nm, sizeof(int32_t), cmp_i32);
        unsigned __int128 total = 0;
        for (int32_t a = 0; a < nm; ++a)
            total += (unsigned __int128)A->sigma[scratch[a]] * B->sigma[scratch[a]];
        if (total >> 64) { result = OR_E_SIGMA_OVERFLOW - 100; break; }
        uint64_t r = choose(ch, 4, 0, (uint64_t)total);
        unsigned __int128 acc = 0;
        int32_t z = -1;
        for (int32_t a = 0; a < nm; ++a) {
            acc += (unsigned __int128)A->sigma[scratch[a]] * B->sigma[scratch[a]];
            if (acc > r) { z = scratch[a]; break; }
        }
        /* v's side first, reversed so the list runs from v towards u */
        int32_t len = walk_to_root(g, B, z, ch, 5, scratch);
        for (int32_t a = 0; a < len; ++a) interior[a] = scratch[len - 1 - a];
        if (z != u && z != v) interior[len++] = z;
        len += walk_to_root(g, A, z, ch, 3, interior + len);
        result = len;
        break;
    }
    side_reset(A);
    side_reset(B);
    return result;
}

typedef struct {
    int32_t *d[2], *S[2], *lvl[2], *scratch;
    uint64_t *sigma[2];
    side_t A, B;
} pair_work_t;

static int pair_work_alloc(pair_work_t *w, int32_t n) {
    size_t nn = (size_t)(n > 0 ? n : 1);
    memset(w, 0, sizeof(*w));
    for (int k = 0; k < 2; ++k) {
        w->d[k] = (int32_t *)malloc(nn * sizeof(int32_t));
        w->S[k] = (int32_t *)malloc(nn * sizeof(int32_t));
        w->lvl[k] = (int32_t *)malloc((nn + 2) * sizeof(int32_t));
        w->sigma[k] = (uint64_t *)calloc(nn, sizeof(uint64_t));
        if (!w->d[k] || !w->S[k] || !w->lvl[k] || !w->sigma[k]) return OR_E_NO_MEMORY;
        for (int32_t i = 0; i < n; ++i) w->d[k][i] = -1;
    }
    w->scratch = (int32_t *)malloc(nn * sizeof(int32_t));
    if (!w->scratch) return OR_E_NO_MEMORY;
    side_t A = {w->d[0], w->sigma[0], w->S[0], w->lvl[0], 0, 0};
    side_t B = {w->d[1], w->sigma[1], w->S[1], w->lvl[1], 0, 0};
    w->A = A;
    w->B = B;
    return OR_OK;
}

static void pair_work_free(pair_work_t *w) {
    for (int k = 0; k < 2; ++k) { free(w->d[k]); free(w->S[k]); free(w->lvl[k]); free(w->sigma[k]); }
    free(w->scratch);
}

/* The path sample j draws for an explicit pair (u, v) (for inspection). */
int or_sample_path_uv(int32_t n, int64_t m, const int32_t *rowptr, const int32_t *colidx,
                      uint64_t seed, int64_t j, int32_t u, int32_t v, int32_t *interior, int32_t *len) {
    int st = or_validate(n, m, rowptr, colidx);
    if (st != OR_OK) return st;
    if (u < 0 || u >= n || v < 0 || v >= n || u == v) return OR_E_INVALID_ARG;
    graph_t g = {n, rowptr, colidx};
    pair_work_t w;
    if (pair_work_alloc(&w, n) != OR_OK) { pair_work_free(&w); return OR_E_NO_MEMORY; }
    chooser_t ch = {seed, j, NULL, 0, 0, NULL, NULL, 0, 0};
    int32_t l = sample_one(&g, &ch, u, v, &w.A, &w.B, interior, w.scratch);
    pair_work_free(&w);
    if (l < -1) return OR_E_SIGMA_OVERFLOW;
    *len = l;
    return OR_OK;
}

/*
 * The path an explicit pair (u, v) yields when the sample's choices are the
 * given values (in request order; missing ones are 0) instead of draws: for
 * enumerating every outcome of the procedure.  ranges[i] receives the range
 * N of request i and keys[i] its generator index stream << 32 | t (up to
 * cap entries each), *nused the number of requests made.  A given value
 * outside its range is an invalid argument.
 */
int or_sample_path_given(int32_t n, int64_t m, const int32_t *rowptr, const int32_t *colidx, int32_t u, int32_t v,
                         const uint64_t *given, int32_t ngiven, uint64_t *ranges, uint64_t *keys, int32_t cap,
                         int32_t *nused, int32_t *interior, int32_t *len) {
    int st = or_validate(n, m, rowptr, colidx);
    if (st != OR_OK) return st;
    if (u < 0 || u >= n || v < 0 || v >= n || u == v || ngiven < 0 || cap < 0) return OR_E_INVALID_ARG;
    graph_t g = {n, rowptr, colidx};
    pair_work_t w;
    if (pair_work_alloc(&w, n) != OR_OK) { pair_work_free(&w); return OR_E_NO_MEMORY; }
    chooser_t ch = {0, 0, given, ngiven, 0, ranges, keys, cap, 0};
    int32_t l = sample_one(&g, &ch, u, v, &w.A, &w.B, interior, w.scratch);
    pair_work_free(&w);
    if (l < -1) return OR_E_SIGMA_OVERFLOW;
    if (ch.bad) return OR_E_INVALID_ARG;
    *nused = ch.used;
    *len = l;
    return OR_OK;
}

/* The sampled pair and path of sample j (for inspection). */
int or_sample_path(int32_t n, int64_t m, const int32_t *rowptr, const int32_t *colidx,
                   uint64_t seed, int64_t j, int32_t *uv, int32_t *interior, int32_t *len) {
    int st = or_validate(n, m, rowptr, colidx);
    if (st != OR_OK) return st;
    if (n < 2) return OR_E_INVALID_ARG;
    graph_t g = {n, rowptr, colidx};
    pair_work_t w;
    if (pair_work_alloc(&w, n) != OR_OK) { pair_work_free(&w); return OR_E_NO_MEMORY; }
    pair_of(seed, j, n, &uv[0], &uv[1]);
    chooser_t ch = {seed, j, NULL, 0, 0, NULL, NULL, 0, 0};
    int32_t l = sample_one(&g, &ch, uv[0], uv[1], &w.A, &w.B, interior, w.scratch);
    pair_work_free(&w);
    if (l < -1) return OR_E_SIGMA_OVERFLOW;
    *len = l;
    return OR_OK;
}

/* Counts cnt[p] = number of samples j in [j0, j1) whose path has p inside
 * (added into counts). */
typedef struct {
    const graph_t *g;
    uint64_t seed;
    int64_t j0, j1;
    uint32_t *counts;
    int status;
} pair_job_t;

static void *run_pair_job(void *arg) {
    pair_job_t *jb = (pair_job_t *)arg;
    const graph_t *g = jb->g;
    pair_work_t w;
    int32_t *interior = (int32_t *)malloc(sizeof(int32_t) * (size_t)g->n);
    if (pair_work_alloc(&w, g->n) != OR_OK || !interior) {
        pair_work_free(&w);
        free(interior);
        jb->status = OR_E_NO_MEMORY;
        return NULL;
    }
    jb->status = OR_OK;
    for (int64_t j = jb->j0; j < jb->j1; ++j) {
        int32_t u, v;
        pair_of(jb->seed, j, g->n, &u, &v);
        chooser_t ch = {jb->seed, j, NULL, 0, 0, NULL, NULL, 0, 0};
        int32_t l = sample_one(g, &ch, u, v, &w.A, &w.B, interior, w.scratch);
        if (l < -1) { jb->status = OR_E_SIGMA_OVERFLOW; break; }
        for (int32_t i = 0; i < l; ++i) jb->counts[interior[i]]++;
    }
    pair_work_free(&w);
    free(interior);
    return NULL;
}

/* Counts cnt[p] = number of samples j in [0, r) whose path has p inside.
 * The timing mode splits [0, r) into nthreads contiguous blocks with
 * private counts, added at the end (integer sums: the result does not
 * depend on nthreads). */
int or_pair_counts(int32_t n, int64_t m, const int32_t *rowptr, const int32_t *colidx,
                   int64_t r, uint64_t seed, uint32_t *counts, int32_t nthreads) {
    int st = or_validate(n, m, rowptr, colidx);
    if (st != OR_OK) return st;
    for (int32_t i = 0; i < n; ++i) counts[i] = 0;
    if (n < 2 || r <= 0) return OR_OK;
    graph_t g = {n, rowptr, colidx};
    if (nthreads <= 1) {
        pair_job_t jb = {&g, seed, 0, r, counts, OR_OK};
        run_pair_job(&jb);
        return jb.status;
    }
    if ((int64_t)nthreads > r) nthreads = (int32_t)r;
    pair_job_t *jobs = (pair_job_t *)calloc((size_t)nthreads, sizeof(pair_job_t));
    pthread_t *th = (pthread_t *)calloc((size_t)nthreads, sizeof(pthread_t));
    char *started = (char *)calloc((size_t)nthreads, 1);
    if (!jobs || !th || !started) { free(jobs); free(th); free(started); return OR_E_NO_MEMORY; }
    for (int32_t t = 0; t < nthreads; ++t) {
        jobs[t].g = &g;
        jobs[t].seed = seed;
        jobs[t].j0 = r * t / nthreads;
        jobs[t].j1 = r * (t + 1) / nthreads;
        jobs[t].counts = (uint32_t *)calloc((size_t)n, sizeof(uint32_t));
        jobs[t].status = jobs[t].counts ? OR_OK : OR_E_NO_MEMORY;
    }
    for (int32_t t = 0; t < nthreads; ++t)
        if (jobs[t].status == OR_OK) started[t] = pthread_create(&th[t], NULL, run_pair_job, &jobs[t]) == 0;
    for (int32_t t = 0; t < nthreads; ++t)
        if (started[t]) pthread_join(th[t], NULL);
        else if (jobs[t].status == OR_OK) jobs[t].status = OR_E_NO_MEMORY;
    st = OR_OK;
    for (int32_t t = 0; t < nthreads; ++t) {
        if (jobs[t].status != OR_OK && st == OR_OK) st = jobs[t].status;
        if (jobs[t].counts) {
            for (int32_t i = 0; i < n; ++i) counts[i] += jobs[t].counts[i];
            free(jobs[t].counts);
        }
    }
    free(started);
    free(jobs);
    free(th);
    return st;
}

/*
 * Full pair-sampling estimate: VD bound, sample size r, counts, and
 * bc[v] = counts[v] / r * n (n - 1) (ordered-pair scale).
 */
int or_pair_sample(int32_t n, int64_t m, const int32_t *rowptr, const int32_t *colidx,
                   double eps, double delta, uint64_t seed, uint32_t *counts, double *bc,
                   int64_t *r_out, int32_t *vd_out) {
    if (!(eps > 0.0 && eps < 1.0) || !(delta > 0.0 && delta < 1.0)) return OR_E_INVALID_ARG;
    int st = or_validate(n, m, rowptr, colidx);
    if (st != OR_OK) return st;
    int32_t info[8];
    st = or_vd_bound(n, m, rowptr, colidx, info);
    if (st != OR_OK) return st;
    int64_t r = n >= 2 ? or_rk_sample_size(eps, delta, info[4]) : 0;
    *r_out = r;
    *vd_out = info[4];
    st = or_pair_counts(n, m, rowptr, colidx, r, seed, counts, 1);
    if (st != OR_OK) return st;
    double scale = r > 0 ? (double)n * (double)(n - 1) / (double)r : 0.0;
    for (int32_t i = 0; i < n; ++i) bc[i] = (double)counts[i] * scale;
    return OR_OK;
}
