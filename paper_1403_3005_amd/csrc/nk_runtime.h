// Host runtime shared by the C ABI (nk_api.hip) and the serving loop
// (nk_server.hip): error reporting, device properties, the pooled scratch
// allocator, tuning state and the persistent-kernel runner.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>
#include <vector>

#include "../../include/nk_bc.h"
#include "nk_kernels.h"

namespace nk {

nk_status fail(nk_status code, const char *fmt, ...);
void clear_error();

#define NK_HIP(expr)                                                                              \
    do {                                                                                          \
        hipError_t e_ = (expr);                                                                   \
        if (e_ != hipSuccess) return ::nk::fail(NK_E_HIP, "%s failed: %s", #expr, hipGetErrorString(e_)); \
    } while (0)

struct DevInfo {
    int device;
    int cus;
    size_t lds_per_block;
};
nk_status dev_info(DevInfo *out);

// Pooled device scratch.  Blocks return to the pool when the holder is
// destroyed; the pool keeps them for later calls until nk_shutdown.
// Scratch block tags (contents that stay meaningful across calls).
// Pair-mode record blocks: every record unreached, and the degree field of
// every record of every whole slot filled from the row pointers kept at the
// block's head, for the record layout of the stride the tag carries.
constexpr uint64_t kTagPairRecords = 1;
inline uint64_t pair_records_tag(long long stride) { return kTagPairRecords | ((uint64_t)stride << 8); }
// Pair-mode hash tables: every entry free and unreached.
constexpr uint64_t kTagPairTables = 2;

class Scratch {
public:
    Scratch() = default;
    ~Scratch();
    Scratch(const Scratch &) = delete;
    Scratch &operator=(const Scratch &) = delete;
    // Returns NK_OK and a device pointer of at least `bytes` bytes (256-byte aligned).
    nk_status get(size_t bytes, void **out);
    template <typename T>
    nk_status get(long long count, T **out) {
        return get((size_t)(count > 0 ? count : 1) * sizeof(T), (void **)out);
    }
    void release_all();
    // A block that keeps a meaning across calls: `tag` != 0 asks for a free
    // block last marked with that tag (*clean = true if one was found; its
    // contents are as the marking call left them).  *block_bytes is the
    // whole block's size, which may exceed `bytes`: a caller that marks the
    // block must have prepared all of it.  Any block handed out loses its
    // tag until mark() sets it again.
    nk_status get_tagged(size_t bytes, uint64_t tag, void **out, bool *clean, size_t *block_bytes);
    void mark(void *p, uint64_t tag);

private:
    std::vector<void *> held_;
};
void pool_clear();
size_t pool_bytes_in_use();
size_t pool_bytes_idle();   // idle pooled bytes on the current device

nk_tuning tuning_get();
void tuning_set(const nk_tuning &t);

// While alive, tuning_get() on this thread returns *t (nothing changes when
// t is NULL); scopes nest.
class TuningOverride {
public:
    explicit TuningOverride(const nk_tuning *t);
    ~TuningOverride();
    TuningOverride(const TuningOverride &) = delete;
    TuningOverride &operator=(const TuningOverride &) = delete;

private:
    const nk_tuning *prev_;
};

// Autotuner cache (nk_tune.hip): the tuning registered for graphs shaped
// like (n, m, max degree), merged into the global tuning (flags and
// scratch cap stay global); false when no cache is registered or it has no
// entry for the shape.
bool cached_tuning(int32_t n, int64_t m, int64_t max_deg, nk_tuning *out);
bool tuning_cache_active();
// Maximum degree of a CSR (one reduction kernel; synchronises s).
nk_status graph_max_degree(const int32_t *rowptr, int32_t n, hipStream_t s, int64_t *out);

// Per-thread statistics of the last call (nk_last_stats).
// lds: 0 global bitmap, 1 bitmap in LDS, 2 whole graph in LDS
void stats_record(const DevStatus &st, int grid, int block, int lds, float kernel_ms);
void stats_clear();

// Launch configuration chosen for a persistent Brandes launch.
struct LaunchPlan {
    int mode;
    int block;
    bool lds;
    int grid;
    size_t dyn_lds;
    long long stride;
    long long bm_words;
    KernelRef kernel;
    void *pair_rec;   // pair mode: the record block the launch used (set by the caller after the launch)
    long long dag_words;   // weighted mode: per-slot words of the DAG-arc bitmap
};
// The tag a pair-mode record block of `plan` carries after a successful
// launch (records or hash tables, by the plan's mode and stride).
inline uint64_t pair_block_tag(const LaunchPlan &plan) {
    return plan.mode == kModePairHash ? kTagPairTables : pair_records_tag(plan.stride);
}

// Picks block size, bitmap placement and grid for graphs of at most n_max
// vertices and `ntasks` tasks.  max_slots > 0 caps the grid.  m_arcs: the
// arcs of the graph (weighted mode sizes its DAG-arc bitmap by them).
nk_status plan_launch(int mode, int32_t n_max, long long ntasks, int max_slots, LaunchPlan *plan,
                      int64_t m_arcs = 0);
// Block size of a persistent launch over graphs of at most n_max vertices
// when the tuning leaves it open.
int auto_block(int32_t n_max);

// Multi-source launch (nk_multi.hip): b sources per task.
struct MsPlan {
    LaunchPlan lp;
    int b;
    int32_t nl;            // vertices whose visited masks sit in LDS
    long long stride;      // per-slot vertex capacity
    long long cap;         // per-slot union-list capacity (stride * b)
    long long visg_words;  // per-slot words of global masks
    long long ntasks;      // tasks of the launch (set by plan_ms for a single graph)
};
// Sources per task for a graph of at most n_max vertices (the tuning's
// batch, or the automatic choice); 1 means the one-source kernels.
int ms_batch_for(int32_t n_max, long long nsources);
// Plan for graphs of at most n_max vertices and `nsources` sources in all
// (tasks = ceil(nsources / b)).
nk_status plan_ms(int b, int32_t n_max, long long nsources, MsPlan *mp);
nk_status ms_alloc(const MsPlan &mp, Params &p, Scratch &scr);
// Clears the path counts, new-source masks and global visited masks, then
// launches (p.ntasks is replaced by the plan's task count).
nk_status ms_enqueue(const MsPlan &mp, const Params &p, hipStream_t s, hipEvent_t ev0, hipEvent_t ev1);
void stats_set_batch(int b);

// Group launch (nk_group.hip): one source per group of workgroups sharing
// an XCD's L2.
struct GroupPlan {
    LaunchPlan lp;
    int gpx;               // groups per XCD
    int groups;            // groups allocated (XCDs x gpx)
    int nxcc;              // XCDs of the device
    long long stride;      // per-group vertex capacity
    long long timeout;     // wall-clock ticks a wait may last
};
// Whether the group kernel takes a graph of n_max vertices and m_arcs arcs:
// automatically for sparse graphs of 10^5 to 3 * 10^5 vertices, for every
// graph under tuning flag bit 3, never under bit 4 or an explicit
// multi-source batch; and only if its visited bitmap fits LDS.
bool group_wanted(int32_t n_max, int64_t m_arcs);
nk_status plan_group(int32_t n_max, GroupPlan *gp);
nk_status group_alloc(const GroupPlan &gp, Params &p, Scratch &scr);
// Clears the path counts, control blocks and registration counters, then
// launches (cooperatively unless the stream is being captured).
nk_status group_enqueue(const GroupPlan &gp, const Params &p, hipStream_t s, hipEvent_t ev0, hipEvent_t ev1);

// Grid-wide direction-optimising breadth-first search (nk_bfs.hip).
struct BfsWork {
    int32_t *d;        // n distances from the source (-1 unreached)
    int32_t *f0, *f1;  // frontier lists, n entries each
    int32_t *f2;       // n + 1: deferred vertices, or a frontier's degrees
    int32_t *off;      // n + 1 arc offsets of a top-down frontier
    long long *cnt;    // 9 words: two level counter sets and one spare
    void *tmp;         // prefix-sum temporary storage
    size_t tmp_bytes;
};
nk_status bfs_work_get(Scratch &scr, int32_t n, hipStream_t s, BfsWork *w);
// Distances from src into w.d; out = {eccentricity of src, lowest id at
// that distance (-1 unless want_lowest), vertices reached}.  src_deg: the
// source's degree if the caller knows it (else -1: read from rowptr).
// Synchronises s.
nk_status grid_bfs(const int32_t *rowptr, const int32_t *colidx, int32_t n, int64_t m, int32_t src,
                   const BfsWork &w, hipStream_t s, int32_t out[3], int32_t src_deg = -1, bool want_lowest = true);
// Size of the largest connected component among the vertices with
// skip[v] < 0 (label, size: n ints of scratch; flag: one int).
nk_status largest_unreached_component(const int32_t *rowptr, const int32_t *colidx, int32_t n, const int32_t *skip,
                                      int32_t *label, int32_t *size, int32_t *flag, hipStream_t s, int32_t *out);

// All-in-LDS betweenness plan for graphs needing at most `dyn_bytes` of
// dynamic LDS; returns false (and plans nothing) when they do not fit or
// tuning flag bit 2 turns the path off.
bool plan_lds(size_t dyn_bytes, int32_t n_max, long long ntasks, LaunchPlan *plan);

// Allocates per-slot scratch for `plan`, clears the path counts, fills the
// scratch fields of `p` and launches the persistent kernel on `s`,
// recording HIP events around it when ev0/ev1 are non-null.
nk_status launch_persistent(const LaunchPlan &plan, Params &p, Scratch &scr, hipStream_t s, hipEvent_t ev0,
                            hipEvent_t ev1);
// The two halves of launch_persistent: persistent_alloc takes the scratch
// and fills the scratch fields of `p` (it enqueues nothing, except in pair
// mode the fill of a record block that is not clean); persistent_enqueue
// clears what the kernel expects clear and launches it -- kernels only, so
// a non-pair launch can be captured into a HIP graph and replayed.
nk_status persistent_alloc(const LaunchPlan &plan, Params &p, Scratch &scr, hipStream_t s);
nk_status persistent_enqueue(const LaunchPlan &plan, const Params &p, hipStream_t s, hipEvent_t ev0,
                             hipEvent_t ev1);

// Copies the status block to the host, synchronises `s` and maps error bits
// to a status code.
nk_status finish(DevStatus *dst, DevStatus *host, hipStream_t s);

nk_status map_err(int32_t err);

// Per-thread pinned status buffer and timing events.
DevStatus *host_status();
nk_status thread_events(hipEvent_t *ev0, hipEvent_t *ev1);

// Graph argument checks shared by every entry point.
nk_status check_graph_args(const int32_t *rowptr, const int32_t *colidx, int32_t n, int64_t m);

// Degree-order relabelling (nk_relabel.hip).  Kernels skip their work when
// the structural check already failed.
// Directed graphs (nk_directed.hip): the in-arc CSR of out-arcs (rows
// sorted by tail), and a check that trowptr's row lengths are the
// in-degrees of colidx (sets kErrGraph in dst otherwise).
nk_status transpose_graph(const int32_t *rowptr, const int32_t *colidx, int32_t n, int64_t m, int32_t *trowptr,
                          int32_t *tcolidx, Scratch &scr, hipStream_t s);
nk_status check_transpose(const int32_t *colidx, int32_t n, int64_t m, const int32_t *trowptr, DevStatus *dst,
                          Scratch &scr, hipStream_t s);

nk_status relabel_graph(const int32_t *rowptr, const int32_t *colidx, int32_t n, int64_t m, const DevStatus *st,
                        Scratch &scr, hipStream_t s, Relabeled *out);
// The same renaming applied to per-arc int32 values (arc weights), and to a
// second CSR over the same vertices (the in-arcs of a directed graph; its
// rows get the renamed in-neighbours, in their original order).
nk_status relabel_weights(const int32_t *wts, const int32_t *rowptr, int32_t n, int64_t m, const Relabeled &g,
                          const DevStatus *st, Scratch &scr, hipStream_t s, int32_t **out);
nk_status relabel_second_csr(const int32_t *rowptr2, const int32_t *colidx2, int32_t n, int64_t m, const Relabeled &g,
                             const DevStatus *st, Scratch &scr, hipStream_t s, int32_t **rp_out, int32_t **ci_out);
hipError_t launch_map_sources(const int32_t *src, int32_t k, const int32_t *perm, int32_t n, int32_t *out,
                              hipStream_t s);
hipError_t launch_arcs_back(const double *in, const int32_t *rp_new, const int32_t *inv, const int32_t *rowptr,
                            int32_t n, double *out, hipStream_t s);
hipError_t launch_gather_scale(const double *in, const int32_t *perm, int32_t n, double scale, double *out,
                               hipStream_t s);
hipError_t launch_gather_u32(const uint32_t *in, const int32_t *perm, int32_t n, uint32_t *out, hipStream_t s);

// Vertex-diameter bound (see nk_vd_bound); runs synchronously on `s`.
// lower = false skips the second sweep, which gives only the lower bound
// (info[3] is then -1 and info[5] 0): the upper bound info[4] is the same.
nk_status vd_bound_impl(const int32_t *rowptr, const int32_t *colidx, int32_t n, int64_t m, int32_t *info,
                        hipStream_t s, bool lower = true);

}  // namespace nk
