// Internal interface between the HIP kernels (nk_kernels.hip) and the host
// runtime (nk_api.cpp, nk_server.cpp).  Not part of the public C ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "nk_device.h"

namespace nk {

// What a persistent Brandes launch computes per task.
enum Mode : int {
    kModeBC = 0,    // forward + dependency sweep, scores into bc
    kModeSSSP = 1,  // forward only, d and sigma written out per task
    kModePair = 2,  // one sampled pair: bidirectional search and path walk
    kModeClose = 3,  // forward with unit path counts; distance sums for closeness
    kModeBisect = 4,  // betweenness with the bisection estimator
    kModeWeighted = 5,  // betweenness over positive integer arc weights
    kModePairHash = 6   // pair mode with each slot's records in a hash table keyed by vertex
};

// Pair mode with hashed records: a table of 2^ph_log2 entries per slot,
// ph_log2 in [kPairHashMinLog2, kPairHashMaxLog2] chosen from the graph's
// size; a sample that could list more than half of it is left to a later
// launch with one record per vertex, and no probe passes kPairHashProbes
// entries.
constexpr int kPairHashMinLog2 = 14;
constexpr int kPairHashMaxLog2 = 18;
constexpr int kPairHashProbes = 128;

// Weighted mode: distinct distances the bucket layering handles; its
// histogram takes kDistBuckets ints of dynamic LDS.
constexpr int kDistBuckets = 4096;

// Bisection: cutoff depths served by one truncated pass (coefficients per
// vertex; one vector fills an aligned line of 8 * kBisK bytes).
constexpr int kBisK = 4;

// Everything a persistent launch reads.  Per-slot scratch arrays hold
// `stride` elements per workgroup slot (slot = blockIdx.x).
struct Params {
    // graph: single graph, or G > 0 concatenated graphs
    const int32_t *rowptr;
    const int32_t *colidx;
    int32_t n;
    int32_t m;
    int32_t G;
    int32_t pad0;
    const long long *g_vtx;    // [G+1] vertex offsets
    const long long *g_arc;    // [G+1] arc offsets
    const long long *g_task;   // [G+1] task prefix in processing order
    const int32_t *g_order;    // [G] processing order -> graph id
    // tasks
    long long ntasks;
    const int32_t *sources;    // task -> source (NULL: task id is the source)
    int32_t pad2;
    int32_t maxlen;            // pair inspection
    // outputs
    double *bc;
    int32_t *d_out;
    unsigned long long *sigma_out;
    uint32_t *counts;
    int32_t *p_uv;
    int32_t *p_len;
    int32_t *p_path;
    unsigned long long seed;
    long long j0;
    // relabelling (degree order): perm maps original -> internal ids, inv
    // internal -> original; both NULL when the graph runs as given
    const int32_t *perm;
    const int32_t *inv;
    // scratch
    unsigned long long *sigma;
    double *dacc;
    int32_t *ldeg;
    int32_t *d;
    int32_t *lv;
    int32_t *la;
    int32_t *ld;
    int32_t *lvl;
    int32_t *cand;
    uint32_t *bmg;             // global bitmaps (when not in LDS; weighted mode: settled vertices)
    const uint32_t *iso;       // isolated-vertex bitmap of a single graph, or NULL
    long long stride;          // per-slot elements of the n-sized arrays
    long long bm_words;        // per-slot words of a global bitmap
    float bu_ratio;
    float bw_ratio;
    DevStatus *st;
    // estimator variants (BC mode): linear != 0 weights each pair (s, t)
    // by d(s, v) / d(s, t) (linear scaling); ebc != NULL also accumulates
    // the per-arc edge terms (single graph, sweep down to level 0)
    int32_t linear;
    // directed graph (single graph, BC modes): rowptr/colidx are the out-
    // arcs; trowptr/tcolidx the in-arcs for bottom-up levels and push sweep
    // levels (NULL: top-down levels and pull sweep levels only).
    int32_t directed;
    double *ebc;
    const int32_t *trowptr;
    const int32_t *tcolidx;
    // weighted mode (single graph, out-arcs): arc weights >= 1; per-slot
    // distances (u64, all-ones = unreached between sources), worklist
    // membership epochs and two worklists
    const int32_t *wts;
    unsigned long long *dist;
    int32_t *mark;
    int32_t *wl0;
    int32_t *wl1;
    int32_t *wl2;              // far pile of the near-far distance rounds
    long long wdelta;          // threshold step of the near-far rounds (0: one bucket)
    double *bvec;              // bisection: kBisK cutoff coefficients per vertex (kBisK * stride per slot)
    uint32_t *dagm;            // per-slot bitmap over the arcs: shortest-path DAG arcs of
    long long dag_words;       // the current source (all clear between sources); words per slot
    // pair mode: 32-byte per-vertex records of both search sides (path
    // counts and distances from u and from v, and, one record per vertex,
    // the vertex's degree; `stride` records per slot) and the level lists
    // of the side grown from the target; pair_blk is the pooled block that
    // holds the records (host side only)
    void *pair_rec;
    void *pair_blk;
    int32_t *lv2;
    int32_t *la2;
    int32_t *ld2;
    // closeness mode: per-source closeness by original id (exact form), or
    // per-vertex integer distance sums over the sources (sampled form)
    double *close_out;
    unsigned long long *close_acc;
    // multi-source mode (nk_multi.hip): ms_b sources per task with their
    // path counts interleaved (sigma[v * ms_b + b]); per slot the masks of
    // sources newly reaching each vertex (nx), the union level lists' source
    // masks (lm, ms_cap entries per slot, as lv/la/ld), and the visited
    // masks of vertices ms_nl and up (visg; those below ms_nl sit in LDS)
    int32_t ms_b;
    int32_t ms_nl;
    long long ms_cap;
    long long nsources;        // sources of a single-graph task list (tasks = ceil(nsources / ms_b))
    uint32_t *nx;
    uint32_t *lm;
    uint32_t *visg;
    long long visg_words;      // per-slot words of visg
    // group mode (nk_group.hip): the workgroups of one XCD share a source;
    // per group (not per slot) `stride` elements of sigma, lv, la, ld, lvl;
    // xg_gpx groups per XCD, xg_groups groups allocated, their control
    // blocks (group_ctl_bytes() each, zeroed before the launch), 17
    // registration counters (zeroed), and the longest wait allowed, in
    // wall-clock ticks
    int32_t xg_gpx;
    int32_t xg_groups;
    int32_t xg_nxcc;           // XCDs of the device (each must hold workgroups of the launch)
    int32_t pad4;
    void *xg_ctl;
    unsigned int *xg_reg;
    long long xg_timeout;
    long long xg_cand_stride;  // per-group entries of the bottom-up candidate array (cand)
    // pair modes: task_list (if not NULL) maps launch task t to sample
    // task_list[t] (outputs indexed by the sample); hashed records: each
    // listed vertex's table slot for both sides (ls, ls2, `stride` entries
    // per slot) and the samples left for a launch with one record per vertex
    // (defer, *defer_count)
    const long long *task_list;
    int32_t ph_log2;           // hashed records: log2 of the entries per slot (stride = 2^ph_log2)
    int32_t pad3;
    int32_t *ls;
    int32_t *ls2;
    long long *defer;
    unsigned long long *defer_count;
};

// Kernel handle for one (mode, block, bitmap placement) instantiation.
struct KernelRef {
    const void *fn;
    void (*launch)(dim3 grid, dim3 block, size_t lds, hipStream_t s, const Params &p);
};

KernelRef brandes_kernel(int mode, int block, bool bitmap_in_lds);

// All-in-LDS betweenness kernel for graphs whose CSR and per-source state
// fit one workgroup's LDS (nk_lds.hip); lds_graph_bytes is its dynamic LDS
// size for a graph of n vertices and m arcs.
KernelRef brandes_lds_kernel(int block);

// Multi-source kernel (nk_multi.hip) for `b` sources per task (4, 8 or
// 16); its dynamic LDS holds the visited masks of the first vertices.
KernelRef brandes_ms_kernel(int block, int b);
// Bytes of visited mask per vertex for b sources per task.
int ms_mask_bytes(int b);
// Group kernel (nk_group.hip): the workgroups of one XCD run one source
// together; its dynamic LDS holds the visited bitmap (4 * ceil(n / 32)
// bytes).  Every workgroup of the launch must be resident at once.
KernelRef brandes_group_kernel(int block);
size_t group_ctl_bytes();
size_t lds_graph_bytes(int32_t n, int64_t m);
hipError_t launch_validate_batched(const int32_t *rowptr_cat, const int32_t *colidx_cat, const long long *g_vtx,
                                   const long long *g_arc, int32_t G, DevStatus *st, hipStream_t s);
hipError_t launch_reset_head(DevStatus *st, hipStream_t s);
// Edge scores: ebc[e] = ebc[rev(e)] = (ebc[e] + ebc[rev(e)]) * scale for
// every arc; a missing reverse arc raises kErrGraph.
hipError_t launch_edge_symmetrize(const int32_t *rowptr, const int32_t *colidx, int32_t n, double *ebc,
                                  double scale, DevStatus *st, hipStream_t s);

// Small helper launches (all asynchronous on `s`).
hipError_t launch_status_init(DevStatus *st, hipStream_t s);
hipError_t launch_validate(const int32_t *rowptr, const int32_t *colidx, int32_t n, int64_t m, int32_t strict,
                           DevStatus *st, hipStream_t s);
hipError_t launch_iso_bitmap(const int32_t *rowptr, int32_t n, uint32_t *iso, hipStream_t s);
hipError_t launch_fill_f64(double *p, double v, long long count, hipStream_t s);
hipError_t launch_fill_u32(uint32_t *p, uint32_t v, long long count, hipStream_t s);
hipError_t launch_fill_i32(int32_t *p, int32_t v, long long count, hipStream_t s);
hipError_t launch_validate_weights(const int32_t *wts, long long m, DevStatus *st, hipStream_t s);
// *sum (zeroed by the caller) += sum of the m weights
hipError_t launch_sum_weights(const int32_t *wts, long long m, unsigned long long *sum, hipStream_t s);
hipError_t launch_fill_u64(unsigned long long *p, unsigned long long v, long long count, hipStream_t s);
hipError_t launch_scale_f64(double *p, double scale, long long count, hipStream_t s);
hipError_t launch_counts_to_bc(const uint32_t *counts, double *bc, double scale, long long count, hipStream_t s);
hipError_t launch_argmax_degree(const int32_t *rowptr, int32_t n, unsigned long long *key, hipStream_t s);
// Pair-mode record block, one record per vertex per slot: a 256-byte head
// (int32 [0] = n of the row pointers kept, [1] = stale flag), the row
// pointers the degree fields were filled from (stride + 1 entries, padded
// to 256 bytes), then the records of every whole slot that fits.
__host__ __device__ inline long long pair_block_head_bytes(long long stride) {
    return 256 + ((stride + 1) * 4 + 255) / 256 * 256;
}
// Prepares a record block of `bytes` bytes for the graph rowptr (n
// vertices): every record of every whole slot unreached (path counts 0,
// distances -1) with its vertex's degree (0 past n), rowptr[0..n] kept.
hipError_t launch_pair_block_init(void *blk, size_t bytes, long long stride, const int32_t *rowptr, int32_t n,
                                  hipStream_t s);
// A block last prepared (or refreshed) for some graph with this stride:
// if the kept row pointers differ from rowptr[0..n], rewrites every
// record's degree field and the kept row pointers (the records stay
// unreached).  Three launches; no host synchronisation.
hipError_t launch_pair_block_refresh(void *blk, size_t bytes, long long stride, const int32_t *rowptr, int32_t n,
                                     hipStream_t s);
// Hashed pair mode: every table entry free and unreached.
hipError_t launch_pair_table_init(void *rec, long long count, hipStream_t s);
// Sampled closeness: out[o] = (n-1) / (n/k * acc[perm[o]]) (0 where acc = 0).
hipError_t launch_close_finish(const unsigned long long *acc, const int32_t *perm, int32_t n, int32_t k, double *out,
                               hipStream_t s);
// Degree-descending relabelling of a single graph (nk_relabel.hip).
struct Relabeled {
    const int32_t *rowptr;  // CSR in internal ids (the input when not relabelled)
    const int32_t *colidx;
    const int32_t *perm;    // original -> internal, or NULL
    const int32_t *inv;     // internal -> original, or NULL
};

}  // namespace nk
