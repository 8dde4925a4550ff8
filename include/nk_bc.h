/*
 * nk_bc.h -- Brandes betweenness centrality on one AMD Instinct MI355X
 * (gfx950): the C ABI of libnkbc.so.
 *
 * The method is the one the NetworKit paper (Staudt, Sazonovs, Meyerhenke,
 * arXiv 1403.3005) uses for betweenness (section "Heuristics and
 * Approximation Algorithms"; Table 1): Brandes' algorithm for unweighted
 * graphs, O(nm) for all sources -- per source a breadth-first search that
 * counts shortest paths (distance d, path count sigma), then a reverse-level
 * dependency accumulation (delta) -- summed over all sources, over a sampled
 * source set (O(sm), scaled), or replaced by Riondato-Kornaropoulos pair
 * sampling with an additive error guarantee epsilon at probability 1-delta.
 *
 * Graphs.  Undirected, unweighted, simple.  CSR with int32 indices:
 *   rowptr  int32[n+1], rowptr[0] = 0, non-decreasing, rowptr[n] = m;
 *   colidx  int32[m], entries in [0, n); every edge {u,v} appears as the two
 *           arcs u->v and v->u; adjacency lists sorted ascending, no
 *           self-loops, no duplicates (preconditions; the structural checks
 *           run on every call, the simple-graph checks in
 *           nk_validate_graph(strict=1)).
 *   n       vertex count, 0 <= n < 2^31;  m  arc count, 0 <= m <= 2^31 - 2^16.
 *
 * Conventions (the paper does not fix them):
 *   - scores sum over ORDERED pairs (s, t), s != v != t (twice the
 *     unordered-pair value some libraries report);
 *   - sigma is uint64; a path count that needs 2^64 or more is an error
 *     (NK_E_SIGMA_OVERFLOW), never saturated;
 *   - scores are FP64; unreachable vertices contribute nothing.
 *
 * Memory.  Unless stated otherwise every array argument is a DEVICE pointer
 * (memory from hipMalloc or a PyTorch CUDA/HIP tensor) on the current HIP
 * device.  The caller owns all inputs and outputs.  The library owns its
 * scratch (pooled per device, released by nk_shutdown).
 *
 * Streams.  `stream` is a hipStream_t passed as void* (NULL = the null
 * stream).  Every call except the nk_server_* family enqueues its work on
 * `stream` and synchronises that stream before it returns, so the returned
 * status -- including a sigma overflow found on the GPU -- is final.
 * Different host threads may call concurrently on different streams.
 *
 * Errors.  Functions return nk_status: 0 on success, a negative code on
 * failure.  No C++ exception crosses this interface.  On failure the
 * contents of output arrays are unspecified; nk_last_error() gives a message
 * for the calling thread's last failure.  Argument checks come first, then
 * graph checks, then the run.
 */
#ifndef NK_BC_H
#define NK_BC_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t nk_status;

enum {
    NK_OK = 0,
    NK_E_INVALID_ARG = -1,     /* null pointer, negative size, bad epsilon ... */
    NK_E_INVALID_GRAPH = -2,   /* CSR structure check failed                  */
    NK_E_SIGMA_OVERFLOW = -3,  /* a shortest-path count needs >= 2^64         */
    NK_E_NO_MEMORY = -4,       /* device allocation failed                    */
    NK_E_HIP = -5,             /* a HIP runtime call failed                   */
    NK_E_BUDGET = -6,          /* request can never fit the HBM budget        */
    NK_E_TIMEOUT = -7,         /* nk_server_wait ran out of time              */
    NK_E_INTERNAL = -8         /* internal capacity check tripped             */
};

/* Message for the calling thread's last failure ("" if none).  The pointer
 * stays valid until the thread's next nk_* call. */
const char *nk_last_error(void);

/* Library version string. */
const char *nk_version(void);

/* Frees pooled device scratch on every device.  Optional; calls after it
 * allocate again. */
void nk_shutdown(void);

/*
 * CSR checks.  strict = 0: rowptr[0] = 0, rowptr non-decreasing,
 * rowptr[n] = m, 0 <= colidx < n (the checks every call runs).
 * strict = 1 adds: no self-loop, adjacency strictly ascending, every arc
 * has its reverse.  Returns NK_OK or NK_E_INVALID_GRAPH.
 */
nk_status nk_validate_graph(const int32_t *rowptr, const int32_t *colidx, int32_t n, int64_t m,
                            int32_t strict, void *stream);

/*
 * Exact betweenness (Brandes' algorithm over every source, the paper's
 * exact "Betweenness"; Table 1, O(nm)).
 *   bc  FP64[n], overwritten: bc[v] = sum over ordered pairs (s,t),
 *       s != v != t, of sigma_st(v) / sigma_st.
 * n = 0 returns NK_OK and writes nothing.
 */
nk_status nk_bc_exact(const int32_t *rowptr, const int32_t *colidx, int32_t n, int64_t m,
                      double *bc, void *stream);

/*
 * Betweenness summed over an explicit source list, times `scale` (the
 * paper's sampled-source approximation: k shortest-path trees instead of n,
 * O(km); scale = n/k gives the plain unbiased estimate).
 *   sources  int32[k] DEVICE array of vertex ids in [0, n); a repeated id
 *            counts once per occurrence; an id out of range is
 *            NK_E_INVALID_ARG (detected on the device).
 *   bc       FP64[n], overwritten.  k = 0 writes zeros.
 */
nk_status nk_bc_sources(const int32_t *rowptr, const int32_t *colidx, int32_t n, int64_t m,
                        const int32_t *sources, int32_t k, double scale, double *bc, void *stream);

/*
 * nk_bc_sources for callers that cannot allocate device memory: code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc.
 * Same arguments, results (within the score tolerance: the summation order
 * differs) and errors as nk_bc_sources.  It calls no hipMalloc, hipFree or
 * allocating library routine: its scratch (status block, isolated-vertex
 * bitmap, per-workgroup state of the persistent kernel) is carved from one
 * fixed 128 MiB array in device memory that each device the library runs
 * on holds until the process ends; the graph runs under the caller's ids
 * (no degree relabelling) and the grid shrinks until the workgroups' state
 * fits.  A graph whose state for one workgroup does not fit (n above about
 * 2.9 million vertices) is NK_E_BUDGET, reported before any launch.  Every
 * call on a device shares that device's array: calls that overlap on one
 * device (other threads or streams) race and must be serialised by the
 * caller.  Synchronises `stream` before returning.
 */
nk_status nk_bc_sources_noalloc(const int32_t *rowptr, const int32_t *colidx, int32_t n, int64_t m,
                                const int32_t *sources, int32_t k, double scale, double *bc, void *stream);

/*
 * Linear-scaling estimator of Geisberger, Sanders and Schultes (the
 * reference the paper cites for approximating betweenness from a few
 * shortest-path trees, "Heuristics and Approximation Algorithms"): every
 * pair (s, t) with s in the source list adds sigma_st(v) / sigma_st times
 * d(s, v) / d(s, t) to v, so vertices near the sampled sources are not
 * over-counted.  Summed over every vertex as a source this is half of
 * exact betweenness; scale = 2 n / k gives the estimate of the exact
 * (ordered-pair) scores.
 *   sources  int32[k] DEVICE array as for nk_bc_sources (NULL with k = n:
 *            every vertex);
 *   bc       FP64[n] DEVICE, overwritten.
 * Same errors as nk_bc_sources.
 */
nk_status nk_bc_sources_linear(const int32_t *rowptr, const int32_t *colidx, int32_t n, int64_t m,
                               const int32_t *sources, int32_t k, double scale, double *bc, void *stream);

/*
 * Bisection estimator of the same paper by Geisberger, Sanders and
 * Schultes: a pair (s, t) with s in the source list counts
 * sigma_st(v) / sigma_st for the vertices v on the far half of its
 * shortest paths (2 d(s, v) > d(s, t)), half of it for a vertex exactly in
 * the middle, nothing on the near half.  As for linear scaling the weights
 * of a path seen from its two ends add to 1: over every vertex as a source
 * this is half of exact betweenness, and scale = 2 n / k estimates the
 * exact scores.  A source whose search reaches depth L does about
 * 1 + L/4 times the dependency-sweep work of nk_bc_sources.
 *   sources, bc, errors as for nk_bc_sources_linear.
 */
nk_status nk_bc_sources_bisect(const int32_t *rowptr, const int32_t *colidx, int32_t n, int64_t m,
                               const int32_t *sources, int32_t k, double scale, double *bc, void *stream);

/*
 * Betweenness of a DIRECTED graph (the paper's graph model allows directed
 * edges, section "Graph data structure"): shortest paths follow arcs, the
 * score of v sums sigma_st(v) / sigma_st over ordered pairs (s, t) with a
 * directed s -> t path, s != v != t, over the listed sources, times scale.
 *   rowptr, colidx     out-arc CSR (int32[n+1], int32[m] DEVICE; no symmetry
 *                      required; simple: no self-loops, no duplicate arcs);
 *   trowptr, tcolidx   the in-arc CSR of the same graph (nk_transpose builds
 *                      it) or both NULL.  With them, levels with a large
 *                      frontier run bottom-up over in-arcs; without, every
 *                      level runs top-down.  A supplied pair is checked for
 *                      structure and for every vertex's in-degree
 *                      (NK_E_INVALID_GRAPH otherwise);
 *   sources, k, scale  as nk_bc_sources (NULL with k = n: every vertex, the
 *                      exact scores);
 *   bc                 FP64[n] DEVICE, overwritten.
 * The dependency sweep pulls over out-arcs or, with the in-arc CSR, pushes
 * over in-arcs where the next level is much smaller.  The run renames the
 * vertices by out-degree internally (scores come back by the caller's ids).
 * Same errors as nk_bc_sources.
 */
nk_status nk_bc_directed(const int32_t *rowptr, const int32_t *colidx, const int32_t *trowptr,
                         const int32_t *tcolidx, int32_t n, int64_t m, const int32_t *sources, int32_t k,
                         double scale, double *bc, void *stream);

/*
 * Betweenness with positive integer arc weights (the paper's graph model
 * carries edge weights, section "Graph data structure"): shortest paths
 * minimise the weight sum, sigma counts the minimum-weight paths, and the
 * score of v sums sigma_st(v) / sigma_st over ordered pairs (s, t), s != v
 * != t, over the listed sources, times scale.
 *   rowptr, colidx  out-arc CSR, DEVICE; an undirected weighted graph is
 *                   given as both arcs of every edge with the same weight
 *                   (no symmetry is required: a directed weighted graph
 *                   works as is);
 *   weights         int32[m] DEVICE, weights[e] >= 1 for arc e
 *                   (NK_E_INVALID_GRAPH otherwise); distances are 64-bit;
 *   sources, k, scale, bc  as nk_bc_sources (NULL with k = n: exact).
 * Integer weights keep "d(s, v) + w = d(s, x)" exact on both sides of a
 * comparison.  The run renames the vertices by out-degree internally,
 * carrying each arc's weight along (scores come back by the caller's ids).
 * Same errors as nk_bc_sources.
 */
nk_status nk_bc_weighted(const int32_t *rowptr, const int32_t *colidx, const int32_t *weights, int32_t n,
                         int64_t m, const int32_t *sources, int32_t k, double scale, double *bc, void *stream);

/*
 * In-arc CSR of a directed graph given by its out-arcs: trowptr int32[n+1]
 * and tcolidx int32[m] DEVICE, caller-allocated, overwritten; every row
 * sorted ascending.  The input is validated first (NK_E_INVALID_GRAPH).
 * Synchronises the stream; scratch of about 16 m bytes.
 */
nk_status nk_transpose(const int32_t *rowptr, const int32_t *colidx, int32_t n, int64_t m, int32_t *trowptr,
                       int32_t *tcolidx, void *stream);

/*
 * Edge betweenness (section "Edge Centrality, Sparsification and Link
 * Prediction"): for the undirected edge {u, v}, the sum over ordered pairs
 * (s, t), s in the source list, of the share of shortest s-t paths that
 * use the edge, times `scale`.
 *   sources  int32[k] DEVICE array, or NULL with k = n for every vertex
 *            (exact edge betweenness);
 *   ebc      FP64[m] DEVICE, overwritten: ebc[e] for arc e = u -> v holds
 *            the score of edge {u, v}; both arcs of an edge hold the same
 *            value;
 *   bc       FP64[n] DEVICE or NULL: the vertex scores of the same run,
 *            times `scale`.
 * Needs the reverse of every arc and ascending adjacency (the CSR rules
 * above); a missing reverse arc is NK_E_INVALID_GRAPH.  The run renames the
 * vertices by degree internally; edge and vertex scores come back in the
 * caller's arc order and vertex ids.
 */
nk_status nk_edge_bc(const int32_t *rowptr, const int32_t *colidx, int32_t n, int64_t m, const int32_t *sources,
                     int32_t k, double scale, double *ebc, double *bc, void *stream);

/*
 * Closeness (Table 1, "closeness": one shortest-path search from each
 * node), generalised to disconnected graphs: with r the number of vertices
 * reachable from v (v included) and F the sum of their distances,
 *     out[v] = (r - 1) / (n - 1) * (r - 1) / F,  0 for an isolated vertex,
 * which is (n - 1) / F on a connected graph.
 *   out  FP64[n] DEVICE, overwritten.
 */
nk_status nk_closeness(const int32_t *rowptr, const int32_t *colidx, int32_t n, int64_t m, double *out,
                       void *stream);

/*
 * Sampled closeness of Eppstein and Wang (Table 1, "ap. closeness"): the
 * farness of v is estimated as F(v) = n / k * sum over the k sources of
 * d(s, v) (an unreachable pair adds 0; the sums are exact integers), and
 *     out[v] = (n - 1) / F(v),  0 where no source reaches v.
 *   sources  int32[k] DEVICE array (repeats count once per occurrence);
 *   out      FP64[n] DEVICE, overwritten; k = 0 writes zeros.
 */
nk_status nk_closeness_sampled(const int32_t *rowptr, const int32_t *colidx, int32_t n, int64_t m,
                               const int32_t *sources, int32_t k, double *out, void *stream);

/*
 * Forward phase only, for inspection: distance and shortest-path count from
 * each of k sources (the breadth-first search with path counting that
 * Brandes' algorithm runs per source).
 *   sources  int32[k] DEVICE array;
 *   d        int32[k*n] DEVICE, row i = source i, -1 = unreachable;
 *   sigma    uint64[k*n] DEVICE, 0 = unreachable.
 * Results are exact integers (bit-identical to any correct BFS).
 */
nk_status nk_sssp_counts(const int32_t *rowptr, const int32_t *colidx, int32_t n, int64_t m,
                         const int32_t *sources, int32_t k, int32_t *d, uint64_t *sigma, void *stream);

/*
 * Vertex-diameter bound for pair sampling (HOST output info[8]):
 *   info = {x0, e1, a, e2, vd_ub, vd_lb, c0, c2} where x0 = vertex of
 *   maximum degree (lowest id on ties), e1 = eccentricity of x0, a = lowest
 *   id at distance e1 from x0, e2 = eccentricity of a (double sweep),
 *   c0 = size of x0's component, c2 = largest other component,
 *   vd_ub = max(min(2*e1+1, c0), c2) >= true vertex diameter,
 *   vd_lb = e2 + 1.
 * n = 0 gives all zeros.
 */
nk_status nk_vd_bound(const int32_t *rowptr, const int32_t *colidx, int32_t n, int64_t m,
                      int32_t *info, void *stream);

/*
 * Riondato-Kornaropoulos sample size (host computation, constant c = 0.5):
 *   r = ceil(0.5 / eps^2 * (floor(log2(max(vd - 2, 1))) + 1 + ln(1/delta))).
 * Returns r, or -1 when eps or delta lies outside (0, 1).
 */
int64_t nk_rk_sample_size(double eps, double delta, int32_t vd);

/*
 * Pair-sampling betweenness with an additive guarantee (the paper's
 * epsilon-approximation, Riondato and Kornaropoulos): r uniform ordered
 * pairs (u, v), u != v, one uniformly chosen shortest u-v path each; with
 * probability >= 1 - delta every |bc[v]/(n(n-1)) - BC(v)/(n(n-1))| <= eps.
 *   eps, delta in (0, 1); seed selects the sample (counter-based
 *   SplitMix64: pair j draws u from stream 1 and v from stream 2; its path
 *   comes from a balanced bidirectional search with path counts on both
 *   sides, which draws the meeting vertex from stream 4 (weight
 *   sigma_u(z) * sigma_v(z)), then step t of the walk from the meeting
 *   vertex towards v from stream 5 and step t of the walk towards u from
 *   stream 3, each choosing a predecessor with probability proportional to
 *   its path count).
 *   bc      FP64[n] DEVICE, counts[v] / r * n * (n-1);
 *   counts  uint32[n] DEVICE or NULL: samples whose path has v inside;
 *   r_out   HOST int64 or NULL: number of samples r;
 *   vd_out  HOST int32 or NULL: the vertex-diameter bound used.
 * n < 2 writes zeros and r = 0.
 */
nk_status nk_bc_pair_sample(const int32_t *rowptr, const int32_t *colidx, int32_t n, int64_t m,
                            double eps, double delta, uint64_t seed, double *bc, uint32_t *counts,
                            int64_t *r_out, int32_t *vd_out, void *stream);

/*
 * Pair-sampling counts for an explicit sample count r (no bound, no
 * scaling): counts uint32[n] DEVICE.  Same sample sequence as
 * nk_bc_pair_sample for the same seed.
 */
nk_status nk_pair_counts(const int32_t *rowptr, const int32_t *colidx, int32_t n, int64_t m,
                         int64_t r, uint64_t seed, uint32_t *counts, void *stream);

/*
 * Inspection of individual samples j0 .. j0+count-1 (DEVICE outputs):
 *   uv     int32[count*2]  the pair (u, v);
 *   len    int32[count]    number of interior path vertices, -1 if v is
 *                          unreachable from u, -2 if more than maxlen;
 *   path   int32[count*maxlen] interior vertices from v's side towards u.
 */
nk_status nk_sample_paths(const int32_t *rowptr, const int32_t *colidx, int32_t n, int64_t m,
                          uint64_t seed, int64_t j0, int32_t count, int32_t maxlen,
                          int32_t *uv, int32_t *len, int32_t *path, void *stream);

/*
 * Exact betweenness of G independent graphs (the paper's recommended use on
 * large batches of smaller networks): one persistent launch of the
 * all-in-LDS kernel for the graphs that fit one workgroup's LDS, one of the
 * global-memory kernel for the rest, and one of the group kernel for the
 * sparse graphs of 10^5 to 3 * 10^5 vertices (see nk_tuning flags bits 3
 * and 4), each draining (graph, source) tasks, largest graphs first.
 *   vtx_off  HOST int64[G+1]: graph g has vertices vtx_off[g] .. vtx_off[g+1]-1
 *            of the concatenated vertex space;
 *   arc_off  HOST int64[G+1]: its arcs are colidx_cat[arc_off[g] .. arc_off[g+1]);
 *   rowptr_cat DEVICE int32[vtx_off[G] + G]: graph g's local rowptr (n_g+1
 *            entries, starting at 0) at offset vtx_off[g] + g;
 *   colidx_cat DEVICE int32[arc_off[G]]: local vertex ids;
 *   bc_cat   DEVICE FP64[vtx_off[G]], overwritten.
 * Every graph obeys the CSR rules above; all sources of all graphs run.
 */
nk_status nk_bc_exact_batched(int32_t G, const int64_t *vtx_off, const int64_t *arc_off,
                              const int32_t *rowptr_cat, const int32_t *colidx_cat, double *bc_cat,
                              void *stream);

/*
 * The batched run above as a captured HIP graph, for a batch that is run
 * again and again (same graphs, same output buffer).  nk_batch_plan_create
 * does all host work once -- argument checks, offset and schedule uploads,
 * the split between the two kernels, kernel plans and every scratch
 * buffer (held by the plan until it is destroyed) -- and records the run's
 * kernels (status reset, batch validation, output clear, the two
 * persistent launches; no memory-set or copy nodes) into a graph on a
 * stream of its own.  nk_batch_plan_run replays it on `stream`, then reads
 * the status (synchronises the stream): the same scores as
 * nk_bc_exact_batched on the same batch, within the stated tolerance.
 *   Arguments of create as nk_bc_exact_batched (HOST offset tables are
 *   copied; rowptr_cat, colidx_cat and bc_cat must stay allocated while
 *   the plan lives, and every run reads the graphs' current contents and
 *   overwrites bc_cat).  *out receives the plan (NULL on error).
 *   Runs of one plan must not overlap; a plan is bound to the device that
 *   was current at creation (NK_E_INVALID_ARG from another).
 * nk_batch_plan_destroy waits for the plan's own stream and releases it.
 */
typedef struct nk_batch_plan nk_batch_plan;
nk_status nk_batch_plan_create(int32_t G, const int64_t *vtx_off, const int64_t *arc_off,
                               const int32_t *rowptr_cat, const int32_t *colidx_cat, double *bc_cat,
                               nk_batch_plan **out);
nk_status nk_batch_plan_run(nk_batch_plan *plan, void *stream);
void nk_batch_plan_destroy(nk_batch_plan *plan);

/*
 * The same run in two halves, for long batches whose caller wants to see
 * the run advance: nk_batch_plan_launch enqueues the graph on `stream` and
 * returns at once; nk_batch_plan_progress reports *done = sources whose
 * dependency sweep has finished so far (read from the device while the run
 * goes on, on the plan's own stream), *total = all sources of the batch,
 * and *finished = 1 once the launch has completed; nk_batch_plan_finish
 * (same stream) waits, reads the status and records the statistics, as
 * nk_batch_plan_run does.  A launched plan must be finished before it is
 * launched again (NK_E_INVALID_ARG otherwise).  The progress read needs
 * `stream` not to be the legacy default stream, which waits for every
 * other stream.
 */
nk_status nk_batch_plan_launch(nk_batch_plan *plan, void *stream);
nk_status nk_batch_plan_progress(nk_batch_plan *plan, int64_t *done, int64_t *total, int32_t *finished);
nk_status nk_batch_plan_finish(nk_batch_plan *plan, void *stream);

/*
 * Statistics of the calling thread's last nk_bc_exact / nk_bc_sources /
 * nk_bc_exact_batched / pair-sampling call (HOST out[32]):
 *   out[0] sources (or samples) processed     out[1] vertices reached
 *   out[2] arcs scanned, forward              out[3] arcs scanned, backward
 *   out[4] shortest-path DAG arcs             out[5] levels run top-down
 *   out[6] levels run bottom-up               out[7] workgroups launched
 *   out[8] main kernel time in microseconds (HIP events on the call's stream)
 *   out[9] threads per workgroup
 *   out[10] kernel placement: 0 visited bitmap in global memory, 1 bitmap in
 *           LDS, 2 whole graph in LDS (all-in-LDS kernel), 3 a batch split
 *           between the all-in-LDS kernel and the LDS-bitmap kernel, 4 the
 *           multi-source kernel, 5 a batch split between the all-in-LDS and
 *           multi-source kernels, 6 the group kernel (the workgroups of one
 *           XCD share a source), 7 a batch split between the all-in-LDS and
 *           group kernels
 *   out[11] arcs of reached vertices (sum of their degrees, over sources)
 *   out[12] dependency-sweep levels run by push
 *   out[13] sources per workgroup task (multi-source kernel; else 1)
 *   out[14] pair samples that could outgrow their slot's hashed records
 *           and ran again with one record per vertex (flags bit 6)
 *   out[15] reserved
 *   (pair sampling: out[1] counts the vertices the searches listed; a
 *   search's probed last level is read, and only its meeting vertices,
 *   which the other side listed, are written)
 *   (nk_bc_weighted: out[2] arcs relaxed in the distance rounds, out[5]
 *   distance rounds, out[6] shortest-path DAG layers, out[4] DAG arcs)
 *   out[16..23] shader-clock cycles per phase, summed over workgroups:
 *           task set-up, top-down levels, bottom-up levels, level marking,
 *           pull levels, push levels, path-count reset, everything else
 *   out[24..29] cycles inside bottom-up levels (staging and scans, arc loop,
 *           finalize) and pull levels (same three); pair sampling reports
 *           in out[24..27] the bidirectional search, the meeting-vertex
 *           choice, the two walks and the clearing; out[30..31] reserved
 */
nk_status nk_last_stats(int64_t *out);

/*
 * Tuning of the per-source kernel: direction switches and tiling.
 *   block      threads per workgroup: 256, 512 or 1024 (0 = automatic);
 *   bu_ratio   run a level bottom-up when the arcs of still-unvisited
 *              vertices are below bu_ratio x the frontier's arcs
 *              (0 = never bottom-up; default 16);
 *   wg_per_cu  resident workgroups per compute unit requested (0 = as many
 *              as fit);
 *   flags      bit 0: keep the visited bitmap in global memory even when it
 *              would fit in LDS (for testing that placement);
 *              bit 1: run single graphs under their own vertex ids instead
 *              of the internal degree-descending relabelling;
 *              bit 2: never use the all-in-LDS kernel (which otherwise runs
 *              betweenness on every graph whose CSR plus one source's state,
 *              about 16 n + 4 m bytes, fits one workgroup's LDS);
 *              bit 3: run exact and source-set betweenness (plain and linear
 *              scaling) of undirected graphs that the all-in-LDS kernel does
 *              not take on the group kernel, where the workgroups of one XCD
 *              run one source together with its path counts in that XCD's
 *              L2 (graphs whose visited bitmap fits LDS: up to about 1.1
 *              million vertices); block 512 makes two groups per XCD;
 *              bit 4: never use the group kernel (the automatic choice runs
 *              it on sparse graphs of 10^5 to 3 * 10^5 vertices);
 *              bit 5: pair sampling always keeps one record per vertex per
 *              workgroup slot; bit 6: it keeps a hash table of the reached
 *              vertices per slot instead (n/16 entries, rounded up to a
 *              power of two in [2^14, 2^18]; graphs above 4x that) and runs
 *              the samples that could fill more than half of it again with
 *              one record per vertex -- which it does by itself when records
 *              per vertex (68 bytes per vertex per slot) would leave fewer
 *              slots than compute units in half the device memory;
 *   bw_ratio   in the dependency sweep, handle level l by pushing from level
 *              l+1 when the arcs of level l+1 are below bw_ratio x the arcs
 *              of level l (0 = always pull; default 0.1);
 *   scratch_mib  cap, in MiB, on the per-call scratch of the persistent
 *              kernel's workgroup slots (about 44 bytes per vertex per slot,
 *              72 in pair sampling); 0 = 85% of the device memory that is
 *              free or idle in the library's pool.  The grid shrinks to fit;
 *              if a single slot does not fit the call fails with
 *              NK_E_NO_MEMORY.
 *   batch      sources per workgroup task in exact and source-set
 *              betweenness (plain and linear scaling) of graphs the
 *              all-in-LDS kernel does not take: 1 = one source per task;
 *              4, 8 or 16 = the multi-source kernel, which runs that many
 *              sources level by level over the union of their frontiers,
 *              reading each adjacency row once per union level and keeping
 *              the sources' path counts of a vertex side by side; 0 =
 *              chosen by graph size.
 *   group      workgroups per group in the group kernel (flags bit 3): 1,
 *              2, 4, 8, 16, 32 or 64, capped at the workgroups of one XCD
 *              (0 = chosen by graph size).  Each group runs one source at a
 *              time; fewer workgroups per group means more sources in
 *              flight, more workgroups per group keeps fewer sources'
 *              path counts in the caches.
 * nk_set_tuning applies to later calls from every thread.
 */
typedef struct {
    int32_t block;
    float bu_ratio;
    int32_t wg_per_cu;
    int32_t flags;
    float bw_ratio;
    int32_t scratch_mib;
    int32_t batch;
    int32_t group;
} nk_tuning;

nk_status nk_set_tuning(const nk_tuning *t);
nk_status nk_get_tuning(nk_tuning *t);

/*
 * Autotuner: times with nk_bc_sources on the given sample of sources
 * (DEVICE int32[k]) every setting of block in {256, 512, 1024}, bu_ratio in
 * {0, 2, 8, 16, 64} and bw_ratio in {0, 0.1, 0.25, 1} (one source per task),
 * on the one-source kernel (flags bit 4), then from the fastest of those
 * one resident workgroup per compute unit, batch = 4, 8 and 16 sources per
 * task (block 1024) and, where its bitmap fits LDS, the group kernel
 * (flags bit 3) with group = 2, 4 and 8 workgroups per source, and returns
 * the fastest in *best (HOST).  The current tuning is left unchanged.  If
 * cache_path is not NULL the winner is stored there under the graph's
 * shape bucket (floor log2 n, round log2 mean degree, round log2 max
 * degree / mean degree) in a flat JSON object
 * {"bucket": [block, bu_ratio, bw_ratio, wg_per_cu, batch, ms,
 * kernel_flags, group]}, kernel_flags being the winner's flag bits 3 and 4
 * (8 or 16).  Entries of six values (no kernel choice) and of four
 * ([block, bu_ratio, bw_ratio, ms]) are read as well.
 */
nk_status nk_autotune(const int32_t *rowptr, const int32_t *colidx, int32_t n, int64_t m, const int32_t *sources,
                      int32_t k, const char *cache_path, nk_tuning *best, void *stream);

/* Cached tuning for a graph shape (n vertices, m arcs, maximum degree
 * max_deg) from an autotuner cache file; NK_E_INVALID_ARG if absent.  Host
 * only: needs no GPU. */
nk_status nk_tuning_lookup(const char *cache_path, int32_t n, int64_t m, int64_t max_deg, nk_tuning *out);

/*
 * Registers an autotuner cache file (NULL or "" unregisters): from then on
 * every nk_bc_exact / nk_bc_sources / linear / bisection / edge / directed
 * call, every batched call or plan (for the launch of its graphs
 * too large for the all-in-LDS kernel, by the largest of them) and every
 * server graph added later (for its source requests) whose shape bucket has
 * an entry runs under that entry's block, bu_ratio, bw_ratio, wg_per_cu,
 * batch and, for eight-value entries, group and flag bits 3 and 4 (the
 * other flags and scratch_mib stay those of nk_set_tuning), found by one
 * maximum-degree reduction per call; other graphs run under the global
 * tuning.  The file is read when registered and re-read when nk_autotune
 * writes it.  NK_E_INVALID_ARG if it cannot be read.
 */
nk_status nk_set_tuning_cache(const char *cache_path);

/*
 * Serving: betweenness queries on a resident pool of graphs with continuous
 * batching and admission by HBM budget (the paper's use case of many
 * analyses over many networks, run as a long-lived service).
 *
 * nk_server_create: hbm_budget_bytes bounds the device memory of resident
 *   graphs plus running requests; n_slots (1..16, 0 = 4) requests run at once,
 *   each on its own stream with 1/n_slots of the workgroups the GPU can hold
 *   at once for its kernel (fewer when that share's scratch does not fit
 *   the budget beside the resident graphs).
 * nk_server_add_graph: copies the CSR (DEVICE pointers, same rules as above)
 *   into server memory, relabels it, computes its vertex-diameter bound.
 *   NK_E_BUDGET if it does not fit.  Not concurrent with other calls on the
 *   same server.
 * nk_server_submit: queues a request and returns at once.
 *   sources  HOST int32[k] (copied), k > 0: betweenness summed over these
 *            sources, scaled by n / k;
 *   k = 0:   pair sampling with eps, delta and seed (as nk_bc_pair_sample);
 *   bc_out   HOST double[n] that receives the scores; it must stay valid
 *            until nk_server_wait returns for the ticket.
 *   NK_E_BUDGET if the request can never fit beside the resident graphs.
 * Requests start in arrival order as soon as a slot is free and their
 *   footprint fits the budget left by the graphs and the running requests.
 * nk_server_wait: blocks until the request is done (timeout_s < 0: no limit),
 *   returns its status (NK_E_TIMEOUT if not done in time; the ticket stays
 *   valid then) and its latency from submit to scores in host memory
 *   (latency_s, HOST, may be NULL).  A ticket is released once waited.
 * nk_server_poll: *done = 1 when the request has finished.
 * nk_server_stats: HOST out[8] = {completed, failed, p50 latency ms, p99
 *   latency ms, max latency ms, GTEPS (sources or samples x undirected edges
 *   over the span from first submit to last completion), most requests in
 *   flight, device bytes in use}.  nk_server_reset_stats clears them.
 * nk_server_destroy: waits for running requests, drops queued ones, frees
 *   everything.
 */
typedef struct nk_server nk_server;

nk_status nk_server_create(size_t hbm_budget_bytes, int32_t n_slots, nk_server **out);
nk_status nk_server_add_graph(nk_server *server, const int32_t *rowptr, const int32_t *colidx, int32_t n,
                              int64_t m, int32_t *graph_id);
nk_status nk_server_submit(nk_server *server, int32_t graph_id, const int32_t *sources, int32_t k, double eps,
                           double delta, uint64_t seed, double *bc_out, int64_t *ticket);
nk_status nk_server_wait(nk_server *server, int64_t ticket, double timeout_s, double *latency_s);
nk_status nk_server_poll(nk_server *server, int64_t ticket, int32_t *done);
nk_status nk_server_stats(nk_server *server, double *out);
nk_status nk_server_reset_stats(nk_server *server);
void nk_server_destroy(nk_server *server);

#ifdef __cplusplus
}
#endif

#endif /* NK_BC_H */
