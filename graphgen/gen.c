/*
 * Seeded synthetic graph generators and a CSR builder.
 *
 * This file produces inputs only: edge lists drawn from named random-graph
 * models and their conversion to a symmetric, sorted, duplicate-free CSR.
 * It contains no shortest-path or centrality arithmetic.
 *
 * Randomness: a counter-based generator built from SplitMix64 (Steele, Lea,
 * Flood, "Fast splittable pseudorandom number generators", OOPSLA 2014).
 * mix64 is the SplitMix64 output function; the k-th output (k >= 1) of a
 * SplitMix64 stream seeded with x is mix64(x + k * GAMMA).  A draw indexed by
 * (seed, stream, j, t) is output t+1 of a stream whose seed is output j+1 of
 * a stream whose seed is output stream+1 of the stream seeded with `seed`.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define GAMMA 0x9E3779B97F4A7C15ULL

static inline uint64_t mix64(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

uint64_t gg_draw(uint64_t seed, uint64_t stream, uint64_t j, uint64_t t) {
    uint64_t k1 = mix64(seed + (stream + 1) * GAMMA);
    uint64_t k2 = mix64(k1 + (j + 1) * GAMMA);
    return mix64(k2 + (t + 1) * GAMMA);
}

/* floor(x * N / 2^64): Lemire's multiply-shift range reduction, no rejection. */
static inline uint64_t bounded(uint64_t x, uint64_t N) {
    return (uint64_t)(((unsigned __int128)x * N) >> 64);
}

/* out[i] = bounded(gg_draw(seed, stream, keys[i], 0), N) for i < count. */
int gg_bounded_draws(uint64_t seed, uint64_t stream, const int64_t *keys, int64_t count, uint64_t N, int32_t *out) {
    if (count < 0 || N == 0 || N > 0x7fffffffULL) return -1;
    for (int64_t i = 0; i < count; ++i) out[i] = (int32_t)bounded(gg_draw(seed, stream, (uint64_t)keys[i], 0), N);
    return 0;
}

/* uniform double in the open interval (0, 1) */
static inline double unit_open(uint64_t x) {
    return ((double)(x >> 11) + 0.5) * (1.0 / 9007199254740992.0);
}

/* uniform double in [0, 1) */
static inline double unit_half(uint64_t x) {
    return (double)(x >> 11) * (1.0 / 9007199254740992.0);
}

/* ---- open-addressing set of 64-bit keys (keys are never ~0) ---- */
typedef struct { uint64_t *slot; uint64_t mask; } kset;

static int kset_init(kset *s, int64_t expected) {
    uint64_t cap = 16;
    while (cap < (uint64_t)(expected * 2 + 16)) cap <<= 1;
    s->slot = (uint64_t *)malloc(cap * sizeof(uint64_t));
    if (!s->slot) return -1;
    memset(s->slot, 0xff, cap * sizeof(uint64_t));
    s->mask = cap - 1;
    return 0;
}

/* returns 1 if inserted, 0 if already present */
static int kset_insert(kset *s, uint64_t key) {
    uint64_t h = mix64(key) & s->mask;
    for (;;) {
        if (s->slot[h] == ~0ULL) { s->slot[h] = key; return 1; }
        if (s->slot[h] == key) return 0;
        h = (h + 1) & s->mask;
    }
}

/*
 * Erdos-Renyi G(n, m): m distinct unordered pairs {u, v}, u != v, each drawn
 * uniformly by rejection.  Candidate j uses draws (seed, 10, j, 0..1).
 * Returns 0, or -1 on bad arguments / allocation failure.
 */
int gg_er(int32_t n, int64_t m, uint64_t seed, int32_t *out_u, int32_t *out_v) {
    if (n < 0 || m < 0) return -1;
    if (n < 2) return m == 0 ? 0 : -1;
    if ((double)m > 0.5 * (double)n * (double)(n - 1)) return -1;
    kset s;
    if (kset_init(&s, m) != 0) return -1;
    int64_t got = 0;
    for (uint64_t j = 0; got < m; ++j) {
        uint64_t a = bounded(gg_draw(seed, 10, j, 0), (uint64_t)n);
        uint64_t b = bounded(gg_draw(seed, 10, j, 1), (uint64_t)n);
        if (a == b) continue;
        uint64_t lo = a < b ? a : b, hi = a < b ? b : a;
        if (!kset_insert(&s, (lo << 32) | hi)) continue;
        out_u[got] = (int32_t)lo;
        out_v[got] = (int32_t)hi;
        ++got;
    }
    free(s.slot);
    return 0;
}

/*
 * R-MAT (Chakrabarti, Zhan, Faloutsos 2004): each edge descends `scale`
 * levels of the recursive 2x2 partition, choosing quadrant (0,0), (0,1),
 * (1,0), (1,1) with probabilities a, b, c, 1-a-b-c.  Edge e, level l uses
 * draw (seed, 20, e, l).  No noise, no relabelling.  Self-loops and
 * duplicates are left for the CSR builder to drop.
 */
int gg_rmat(int32_t scale, int64_t nedges, double a, double b, double c, uint64_t seed,
            int32_t *out_u, int32_t *out_v) {
    if (scale < 1 || scale > 30 || nedges < 0) return -1;
    double ab = a + b, abc = a + b + c;
    for (int64_t e = 0; e < nedges; ++e) {
        uint32_t u = 0, v = 0;
        for (int l = 0; l < scale; ++l) {
            double x = unit_half(gg_draw(seed, 20, (uint64_t)e, (uint64_t)l));
            uint32_t bu, bv;
            if (x < a) { bu = 0; bv = 0; }
            else if (x < ab) { bu = 0; bv = 1; }
            else if (x < abc) { bu = 1; bv = 0; }
            else { bu = 1; bv = 1; }
            u = (u << 1) | bu;
            v = (v << 1) | bv;
        }
        out_u[e] = (int32_t)u;
        out_v[e] = (int32_t)v;
    }
    return 0;
}

/*
 * Chung-Lu random graph with expected degrees w_i (sorted non-increasing),
 * edge {u, v} present independently with probability min(1, w_u w_v / S),
 * S = sum w.  Generated with the O(n + m) skipping method of Miller and
 * Hagberg ("Efficient generation of networks with given expected degrees",
 * WAW 2011).  Row u consumes draws (seed, 30, u, 0, 1, 2, ...).
 * Weights: w_i = mean * (g-2)/(g-1) * (n/(i+1))^(1/(g-1)).
 * Writes up to `cap` edges; returns the edge count, or -(needed) if `cap`
 * was too small (the caller retries with a larger buffer), or -1 on error
 * when n < 1.
 */
int64_t gg_chung_lu(int32_t n, double gamma_exp, double mean_deg, uint64_t seed,
                    int32_t *out_u, int32_t *out_v, int64_t cap) {
    if (n < 1 || !(gamma_exp > 2.0) || !(mean_deg > 0.0)) return -1;
    double *w = (double *)malloc(sizeof(double) * (size_t)n);
    if (!w) return -1;
    double ex = 1.0 / (gamma_exp - 1.0);
    double pre = mean_deg * (gamma_exp - 2.0) / (gamma_exp - 1.0);
    double S = 0.0;
    for (int32_t i = 0; i < n; ++i) {
        w[i] = pre * pow((double)n / (double)(i + 1), ex);
        S += w[i];
    }
    int64_t cnt = 0;
    for (int32_t u = 0; u + 1 < n; ++u) {
        uint64_t t = 0;
        int64_t v = u + 1;
        double p = w[u] * w[v] / S;
        if (p > 1.0) p = 1.0;
        while (v < n && p > 0.0) {
            if (p != 1.0) {
                double r = unit_open(gg_draw(seed, 30, (uint64_t)u, t++));
                v += (int64_t)floor(log(r) / log1p(-p));
            }
            if (v < n) {
                double q = w[u] * w[v] / S;
                if (q > 1.0) q = 1.0;
                double r = unit_open(gg_draw(seed, 30, (uint64_t)u, t++));
                if (r < q / p) {
                    if (cnt < cap) { out_u[cnt] = u; out_v[cnt] = (int32_t)v; }
                    ++cnt;
                }
                p = q;
                v += 1;
            }
        }
    }
    free(w);
    return cnt <= cap ? cnt : -cnt;
}

/*
 * Barabasi-Albert preferential attachment: start from the complete graph on
 * m0+1 vertices; each later vertex v attaches to m0 distinct earlier vertices,
 * each chosen with probability proportional to current degree (uniform pick
 * from the list of edge endpoints; repeats are redrawn).  Vertex v uses draws
 * (seed, 40, v, 0, 1, ...).  Edge count: (m0+1)m0/2 + (n-m0-1)m0.
 */
int gg_ba(int32_t n, int32_t m0, uint64_t seed, int32_t *out_u, int32_t *out_v) {
    if (m0 < 1 || n < m0 + 1) return -1;
    int64_t ne_total = (int64_t)(m0 + 1) * m0 / 2 + (int64_t)(n - m0 - 1) * m0;
    int32_t *ends = (int32_t *)malloc(sizeof(int32_t) * (size_t)(2 * ne_total));
    int32_t *pick = (int32_t *)malloc(sizeof(int32_t) * (size_t)m0);
    if (!ends || !pick) { free(ends); free(pick); return -1; }
    int64_t ne = 0, nends = 0;
    for (int32_t i = 0; i <= m0; ++i)
        for (int32_t j = i + 1; j <= m0; ++j) {
            out_u[ne] = i; out_v[ne] = j; ++ne;
            ends[nends++] = i; ends[nends++] = j;
        }
    for (int32_t v = m0 + 1; v < n; ++v) {
        uint64_t t = 0;
        int32_t got = 0;
        while (got < m0) {
            int32_t c = ends[bounded(gg_draw(seed, 40, (uint64_t)v, t++), (uint64_t)nends)];
            int dup = 0;
            for (int32_t q = 0; q < got; ++q) dup |= (pick[q] == c);
            if (!dup) pick[got++] = c;
        }
        for (int32_t q = 0; q < m0; ++q) {
            out_u[ne] = pick[q]; out_v[ne] = v; ++ne;
            ends[nends++] = pick[q]; ends[nends++] = v;
        }
    }
    free(ends);
    free(pick);
    return 0;
}

/*
 * k distinct sources out of [0, n) by a partial Fisher-Yates shuffle; step i
 * swaps position i with i + bounded(draw(seed, 50, i, 0), n - i).
 */
int gg_sample_sources(int32_t n, int32_t k, uint64_t seed, int32_t *out) {
    if (k < 0 || k > n) return -1;
    int32_t *perm = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    if (!perm) return -1;
    for (int32_t i = 0; i < n; ++i) perm[i] = i;
    for (int32_t i = 0; i < k; ++i) {
        int32_t j = i + (int32_t)bounded(gg_draw(seed, 50, (uint64_t)i, 0), (uint64_t)(n - i));
        int32_t tmp = perm[i]; perm[i] = perm[j]; perm[j] = tmp;
        out[i] = perm[i];
    }
    free(perm);
    return 0;
}

static int cmp_i32(const void *a, const void *b) {
    int32_t x = *(const int32_t *)a, y = *(const int32_t *)b;
    return (x > y) - (x < y);
}

/*
 * Undirected CSR from an edge list: each edge {u, v} with u != v is stored as
 * arcs u->v and v->u; self-loops are dropped, each adjacency list is sorted
 * ascending and duplicates are removed.  rowptr has n+1 entries; colidx must
 * hold 2*ne entries (the final arc count may be smaller).  Returns the arc
 * count, or -1 on a vertex id out of range / allocation failure.
 */
int64_t gg_csr(int32_t n, int64_t ne, const int32_t *u, const int32_t *v,
               int32_t *rowptr, int32_t *colidx) {
    int64_t *cnt = (int64_t *)calloc((size_t)n + 1, sizeof(int64_t));
    if (!cnt) return -1;
    for (int64_t e = 0; e < ne; ++e) {
        if (u[e] < 0 || u[e] >= n || v[e] < 0 || v[e] >= n) { free(cnt); return -1; }
        if (u[e] == v[e]) continue;
        cnt[u[e] + 1]++;
        cnt[v[e] + 1]++;
    }
    for (int32_t i = 0; i < n; ++i) cnt[i + 1] += cnt[i];
    if (cnt[n] > 2147483647LL) { free(cnt); return -1; }
    int64_t *pos = (int64_t *)malloc(sizeof(int64_t) * ((size_t)n + 1));
    if (!pos) { free(cnt); return -1; }
    memcpy(pos, cnt, sizeof(int64_t) * ((size_t)n + 1));
    for (int64_t e = 0; e < ne; ++e) {
        if (u[e] == v[e]) continue;
        colidx[pos[u[e]]++] = v[e];
        colidx[pos[v[e]]++] = u[e];
    }
    free(pos);
    int64_t w = 0;
    rowptr[0] = 0;
    for (int32_t i = 0; i < n; ++i) {
        int64_t b = cnt[i], e = cnt[i + 1];
        qsort(colidx + b, (size_t)(e - b), sizeof(int32_t), cmp_i32);
        int64_t start = w;
        for (int64_t q = b; q < e; ++q) {
            if (q > b && colidx[q] == colidx[q - 1]) continue;
            colidx[w++] = colidx[q];
        }
        (void)start;
        rowptr[i + 1] = (int32_t)w;
    }
    free(cnt);
    return w;
}
