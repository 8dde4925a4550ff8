// Host runtime and C ABI of libnkbc.so (declarations and contracts in
// include/nk_bc.h).
#include <stdarg.h>
#include <stdio.h>
#include <string.h>

#include <algorithm>
#include <cmath>
#include <mutex>
#include <numeric>
#include <string>
#include <vector>

#include "nk_runtime.h"

namespace nk {

// ------------------------------------------------------------------ errors --

static thread_local std::string t_err;
static thread_local int64_t t_stats[32];

nk_status fail(nk_status code, const char *fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    t_err = buf;
    return code;
}

void clear_error() { t_err.clear(); }

nk_status map_err(int32_t err) {
    if (err & kErrGraph) return fail(NK_E_INVALID_GRAPH, "CSR structure check failed");
    if (err & kErrArg) return fail(NK_E_INVALID_ARG, "a source or sample index is out of range");
    if (err & kErrOverflow) return fail(NK_E_SIGMA_OVERFLOW, "a shortest-path count needs 2^64 or more");
    if (err & kErrInternal) return fail(NK_E_INTERNAL, "internal capacity check tripped");
    return NK_OK;
}

// ------------------------------------------------------------ device info --

static std::mutex g_dev_mu;
static DevInfo g_dev[64];
static bool g_dev_ok[64];

nk_status dev_info(DevInfo *out) {
    int dev = 0;
    NK_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= 64) return fail(NK_E_HIP, "device index %d out of range", dev);
    std::lock_guard<std::mutex> lk(g_dev_mu);
    if (!g_dev_ok[dev]) {
        DevInfo d;
        d.device = dev;
        int cus = 0, lds = 0;
        NK_HIP(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
        NK_HIP(hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev));
        d.cus = cus;
        d.lds_per_block = (size_t)lds;
        g_dev[dev] = d;
        g_dev_ok[dev] = true;
    }
    *out = g_dev[dev];
    return NK_OK;
}

// ------------------------------------------------------------ scratch pool --

struct PoolBlock {
    void *ptr;
    size_t bytes;
    int device;
    bool busy;
    uint64_t tag;   // meaning of the contents kept across calls (0 = none)
};
static std::mutex g_pool_mu;
static std::vector<PoolBlock> g_pool;

nk_status Scratch::get(size_t bytes, void **out) {
    int dev = 0;
    NK_HIP(hipGetDevice(&dev));
    bytes = (bytes + 255) & ~(size_t)255;
    {
        std::lock_guard<std::mutex> lk(g_pool_mu);
        int best = -1;
        for (size_t i = 0; i < g_pool.size(); ++i) {
            const PoolBlock &b = g_pool[i];
            if (b.busy || b.device != dev || b.bytes < bytes || b.bytes > 2 * bytes + (64u << 20)) continue;
            if (best < 0 || b.bytes < g_pool[best].bytes) best = (int)i;
        }
        if (best >= 0) {
            g_pool[best].busy = true;
            g_pool[best].tag = 0;
            held_.push_back(g_pool[best].ptr);
            *out = g_pool[best].ptr;
            return NK_OK;
        }
    }
    void *p = nullptr;
    hipError_t e = hipMalloc(&p, bytes);
    if (e != hipSuccess) {
        (void)hipGetLastError();
        // release idle blocks of this device and retry once
        std::vector<void *> idle;
        {
            std::lock_guard<std::mutex> lk(g_pool_mu);
            for (size_t i = 0; i < g_pool.size();) {
                if (!g_pool[i].busy && g_pool[i].device == dev) {
                    idle.push_back(g_pool[i].ptr);
                    g_pool.erase(g_pool.begin() + i);
                } else {
                    ++i;
                }
            }
        }
        for (void *q : idle) (void)hipFree(q);
        e = hipMalloc(&p, bytes);
        if (e != hipSuccess) {
            (void)hipGetLastError();
            return fail(NK_E_NO_MEMORY, "hipMalloc of %zu bytes failed", bytes);
        }
    }
    {
        std::lock_guard<std::mutex> lk(g_pool_mu);
        g_pool.push_back(PoolBlock{p, bytes, dev, true, 0});
    }
    held_.push_back(p);
    *out = p;
    return NK_OK;
}

nk_status Scratch::get_tagged(size_t bytes, uint64_t tag, void **out, bool *clean, size_t *block_bytes) {
    int dev = 0;
    NK_HIP(hipGetDevice(&dev));
    const size_t need = (bytes + 255) & ~(size_t)255;
    *clean = false;
    *block_bytes = need;
    {
        std::lock_guard<std::mutex> lk(g_pool_mu);
        int best = -1;
        for (size_t i = 0; i < g_pool.size(); ++i) {
            const PoolBlock &b = g_pool[i];
            if (b.busy || b.device != dev || b.tag != tag || b.bytes < need || b.bytes > 2 * need + (64u << 20))
                continue;
            if (best < 0 || b.bytes < g_pool[best].bytes) best = (int)i;
        }
        if (best >= 0) {
            g_pool[best].busy = true;
            g_pool[best].tag = 0;   // dirty until marked again
            held_.push_back(g_pool[best].ptr);
            *out = g_pool[best].ptr;
            *clean = true;
            *block_bytes = g_pool[best].bytes;
            return NK_OK;
        }
    }
    nk_status st = get(bytes, out);
    if (st != NK_OK) return st;
    // a reused untagged block may be larger than asked for; the caller
    // prepares all of it, so that a later mark() covers the whole block
    std::lock_guard<std::mutex> lk(g_pool_mu);
    for (const auto &b : g_pool)
        if (b.ptr == *out) *block_bytes = b.bytes;
    return NK_OK;
}

void Scratch::mark(void *p, uint64_t tag) {
    std::lock_guard<std::mutex> lk(g_pool_mu);
    for (auto &b : g_pool)
        if (b.ptr == p) b.tag = tag;
}

void Scratch::release_all() {
    std::lock_guard<std::mutex> lk(g_pool_mu);
    for (void *p : held_)
        for (auto &b : g_pool)
            if (b.ptr == p) b.busy = false;
    held_.clear();
}

Scratch::~Scratch() { release_all(); }

void pool_clear() {
    std::vector<PoolBlock> keep, drop;
    {
        std::lock_guard<std::mutex> lk(g_pool_mu);
        for (auto &b : g_pool) (b.busy ? keep : drop).push_back(b);
        g_pool = keep;
    }
    int cur = 0;
    (void)hipGetDevice(&cur);
    for (auto &b : drop) {
        (void)hipSetDevice(b.device);
        (void)hipFree(b.ptr);
    }
    (void)hipSetDevice(cur);
}

size_t pool_bytes_idle() {
    int dev = 0;
    (void)hipGetDevice(&dev);
    std::lock_guard<std::mutex> lk(g_pool_mu);
    size_t s = 0;
    for (auto &b : g_pool)
        if (!b.busy && b.device == dev) s += b.bytes;
    return s;
}

size_t pool_bytes_in_use() {
    std::lock_guard<std::mutex> lk(g_pool_mu);
    size_t s = 0;
    for (auto &b : g_pool)
        if (b.busy) s += b.bytes;
    return s;
}

// ------------------------------------------------------------------ tuning --

static std::mutex g_tune_mu;
static nk_tuning g_tune = {0, 16.0f, 0, 0, 0.1f, 0, 0, 0};

// A call running under a cached per-graph-shape tuning sees it instead of
// the global one (thread-local, set for the duration of the call).
static thread_local const nk_tuning *t_override = nullptr;

nk_tuning tuning_get() {
    if (t_override) return *t_override;
    std::lock_guard<std::mutex> lk(g_tune_mu);
    return g_tune;
}

TuningOverride::TuningOverride(const nk_tuning *t) : prev_(t_override) {
    if (t) t_override = t;
}
TuningOverride::~TuningOverride() { t_override = prev_; }

void tuning_set(const nk_tuning &t) {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune = t;
}

// ------------------------------------------------------------------- stats --

void stats_clear() { memset(t_stats, 0, sizeof(t_stats)); }

void stats_set_batch(int b) { t_stats[13] = b; }

void stats_record(const DevStatus &st, int grid, int block, int lds, float kernel_ms) {
    t_stats[0] = (int64_t)st.stat[kStSources];
    t_stats[1] = (int64_t)st.stat[kStReached];
    t_stats[2] = (int64_t)st.stat[kStArcsFwd];
    t_stats[3] = (int64_t)st.stat[kStArcsBwd];
    t_stats[4] = (int64_t)st.stat[kStDag];
    t_stats[5] = (int64_t)st.stat[kStTd];
    t_stats[6] = (int64_t)st.stat[kStBu];
    t_stats[7] = grid;
    t_stats[8] = (int64_t)llround((double)kernel_ms * 1000.0);
    t_stats[9] = block;
    t_stats[10] = lds;
    t_stats[11] = (int64_t)st.stat[kStArcsReached];
    t_stats[12] = (int64_t)st.stat[kStBwPush];
    t_stats[13] = 1;
    t_stats[14] = (int64_t)st.stat[kStDeferred];
    t_stats[15] = 0;
    for (int i = 0; i < kNumPhases; ++i) t_stats[16 + i] = (int64_t)st.cycles[i];
    for (int i = 0; i < 8; ++i) t_stats[24 + i] = (int64_t)st.sub[i];
}

static thread_local DevStatus *t_host_status = nullptr;
static thread_local hipEvent_t t_ev[2] = {nullptr, nullptr};

DevStatus *host_status() {
    if (!t_host_status) {
        void *p = nullptr;
        if (hipHostMalloc(&p, sizeof(DevStatus), hipHostMallocDefault) != hipSuccess) {
            (void)hipGetLastError();
            return nullptr;
        }
        t_host_status = (DevStatus *)p;
    }
    return t_host_status;
}

nk_status thread_events(hipEvent_t *ev0, hipEvent_t *ev1) {
    if (!t_ev[0]) {
        NK_HIP(hipEventCreate(&t_ev[0]));
        NK_HIP(hipEventCreate(&t_ev[1]));
    }
    *ev0 = t_ev[0];
    *ev1 = t_ev[1];
    return NK_OK;
}

nk_status finish(DevStatus *dst, DevStatus *host, hipStream_t s) {
    NK_HIP(hipMemcpyAsync(host, dst, sizeof(DevStatus), hipMemcpyDeviceToHost, s));
    NK_HIP(hipStreamSynchronize(s));
    return map_err(host->err);
}

// Arc indices inside a tile are int32 and run up to 4 * BLOCK past the
// tile's arc count, so m keeps a margin below 2^31.
static const long long kMaxArcs = 2147483647LL - 65536;

nk_status check_graph_args(const int32_t *rowptr, const int32_t *colidx, int32_t n, int64_t m) {
    if (n < 0) return fail(NK_E_INVALID_ARG, "n = %d is negative", n);
    if (m < 0 || m > kMaxArcs) return fail(NK_E_INVALID_ARG, "m = %lld outside [0, 2^31 - 2^16]", (long long)m);
    if (n > 0 && !rowptr) return fail(NK_E_INVALID_ARG, "rowptr is NULL");
    if (m > 0 && !colidx) return fail(NK_E_INVALID_ARG, "colidx is NULL");
    return NK_OK;
}

// ----------------------------------------------------------------- planner --

int auto_block(int32_t n_max) {
    if (n_max < 20000) return 256;
    if (n_max < 200000) return 512;
    return 1024;
}

// Words of a per-slot bitmap over m arcs, rounded to 256 bytes.
static long long dag_words_of(int64_t m) { return ((m + 31) / 32 + 63) / 64 * 64; }

nk_status plan_launch(int mode, int32_t n_max, long long ntasks, int max_slots, LaunchPlan *plan, int64_t m_arcs) {
    DevInfo di;
    nk_status st = dev_info(&di);
    if (st != NK_OK) return st;
    nk_tuning t = tuning_get();
    int block = t.block;
    if (block != 256 && block != 512 && block != 1024) {
        block = auto_block(n_max);
        // a pair sample's search levels are small: more concurrent samples
        // of 256 threads hide more memory latency than fewer wide ones
        if (mode == kModePair || mode == kModePairHash) block = 256;
    }
    const long long words = ((long long)n_max + 31) / 32;
    const size_t bm_bytes = (size_t)words * 4;
    bool lds = false;
    // weighted mode: the distance-bucket histogram shares the dynamic LDS
    // with the settled-vertex bitmap (or has it alone)
    const size_t hist_bytes = mode == kModeWeighted ? (size_t)kDistBuckets * 4 : 0;
    {
        KernelRef probe = brandes_kernel(mode, block, true);
        hipFuncAttributes attr;
        NK_HIP(hipFuncGetAttributes(&attr, probe.fn));
        // pair mode keeps two visited bitmaps (one per search side) in global memory
        lds = attr.sharedSizeBytes + std::max(bm_bytes, hist_bytes) <= di.lds_per_block && !(t.flags & 1) &&
              mode != kModePair && mode != kModePairHash;
    }
    KernelRef kr = brandes_kernel(mode, block, lds);
    size_t dyn = std::max(lds ? bm_bytes : 0, hist_bytes);
    if (dyn > 0) NK_HIP(hipFuncSetAttribute(kr.fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)dyn));
    int occ = 0;
    NK_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, kr.fn, block, dyn));
    if (occ < 1) return fail(NK_E_INTERNAL, "kernel does not fit a compute unit (block %d, lds %zu)", block, dyn);
    if (t.wg_per_cu > 0 && t.wg_per_cu < occ) occ = t.wg_per_cu;
    long long grid = (long long)di.cus * occ;
    // max_slots < 0: a 1/|max_slots| share of the resident-workgroup capacity
    if (max_slots < 0) grid = std::max(1LL, grid / (-(long long)max_slots));
    if (ntasks < grid) grid = ntasks;
    if (max_slots > 0 && grid > max_slots) grid = max_slots;
    if (grid < 1) grid = 1;
    // Cap the grid so the slots' scratch fits.
    {
        const long long stride = (((long long)n_max + 2) + 63) / 64 * 64;
        const long long wordsr = (words + 63) / 64 * 64;
        // pair sampling: 32-byte records, 8 (weights) and 6 x 4 (two sides'
        // lists) + 4 (meeting list); otherwise 8 + 8 + 7 x 4 and a global
        // bitmap when it does not sit in LDS
        // weighted: + u64 distances, round marks, two worklists and the far pile (24)
        // bisection: + kBisK cutoff coefficients per vertex
        // hashed pair records: + the two sides' table slots (8)
        size_t per_slot = (size_t)stride * (mode == kModePair       ? 68
                                            : mode == kModePairHash ? 76
                                            : mode == kModeWeighted ? 68
                                            : mode == kModeBisect   ? 44 + 8 * kBisK
                                                                    : 44);
        if (mode != kModePair && mode != kModePairHash && !lds) per_slot += (size_t)wordsr * 4;
        // weighted: one bit per arc marks the shortest-path DAG
        if (mode == kModeWeighted) per_slot += (size_t)dag_words_of(m_arcs) * 4;
        size_t avail;
        if (t.scratch_mib > 0) {
            avail = (size_t)t.scratch_mib << 20;
        } else {
            size_t fr = 0, tot = 0;
            NK_HIP(hipMemGetInfo(&fr, &tot));
            avail = (size_t)((double)(fr + pool_bytes_idle()) * 0.85);
            // pair samples touch their slots' records at random: beyond
            // about half the device's memory, more slots add address-
            // translation misses faster than they hide latency
            if ((mode == kModePair || mode == kModePairHash) && avail > tot / 2) avail = tot / 2;
        }
        const long long fit = (long long)(avail / per_slot);
        if (fit < 1)
            return fail(NK_E_NO_MEMORY, "one workgroup slot needs %zu bytes of scratch; %zu available", per_slot,
                        avail);
        // a memory-capped grid keeps the same number of workgroups on
        // every compute unit
        if (grid > fit) grid = fit > di.cus ? fit / di.cus * di.cus : fit;
    }
    plan->mode = mode;
    plan->block = block;
    plan->lds = lds;
    plan->grid = (int)grid;
    plan->dyn_lds = dyn;
    plan->stride = (((long long)n_max + 2) + 63) / 64 * 64;
    plan->bm_words = (words + 63) / 64 * 64;
    plan->kernel = kr;
    plan->pair_rec = nullptr;
    plan->dag_words = mode == kModeWeighted ? dag_words_of(m_arcs) : 0;
    return NK_OK;
}

bool plan_lds(size_t dyn_bytes, int32_t n_max, long long ntasks, LaunchPlan *plan) {
    nk_tuning t = tuning_get();
    if (t.flags & 4) return false;
    DevInfo di;
    if (dev_info(&di) != NK_OK) {
        clear_error();
        return false;
    }
    int block = t.block;
    // levels of graphs above ~1500 vertices fill a 1024-thread tile; smaller
    // ones leave room for two 512-thread workgroups per compute unit
    if (block != 256 && block != 512 && block != 1024) block = n_max >= 1500 ? 1024 : 512;
    KernelRef kr = brandes_lds_kernel(block);
    hipFuncAttributes attr;
    if (hipFuncGetAttributes(&attr, kr.fn) != hipSuccess) return false;
    if (attr.sharedSizeBytes + dyn_bytes > di.lds_per_block) return false;
    if (hipFuncSetAttribute(kr.fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)dyn_bytes) != hipSuccess)
        return false;
    int occ = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, kr.fn, block, dyn_bytes) != hipSuccess || occ < 1)
        return false;
    if (t.wg_per_cu > 0 && t.wg_per_cu < occ) occ = t.wg_per_cu;
    long long grid = (long long)di.cus * occ;
    if (ntasks < grid) grid = ntasks;
    if (grid < 1) grid = 1;
    plan->mode = kModeBC;
    plan->block = block;
    plan->lds = true;
    plan->grid = (int)grid;
    plan->dyn_lds = dyn_bytes;
    plan->stride = 0;
    plan->bm_words = 0;
    plan->kernel = kr;
    return true;
}

// ------------------------------------------------------ multi-source plan --

int ms_batch_for(int32_t n_max, long long nsources) {
    const int t = tuning_get().batch;
    if (t == 1 || t == 4 || t == 8 || t == 16) return t;
    (void)n_max;
    (void)nsources;
    return 1;
}

nk_status plan_ms(int b, int32_t n_max, long long nsources, MsPlan *mp) {
    DevInfo di;
    nk_status st = dev_info(&di);
    if (st != NK_OK) return st;
    const nk_tuning t = tuning_get();
    int block = t.block;
    if (block != 256 && block != 512 && block != 1024) block = 1024;
    KernelRef kr = brandes_ms_kernel(block, b);
    hipFuncAttributes attr;
    NK_HIP(hipFuncGetAttributes(&attr, kr.fn));
    const int per_word = 4 / ms_mask_bytes(b);
    const size_t room = di.lds_per_block > attr.sharedSizeBytes ? di.lds_per_block - attr.sharedSizeBytes : 0;
    long long nl = (long long)(room / 4) * per_word;
    const long long n_round = ((long long)n_max + per_word - 1) / per_word * per_word;
    if (nl > n_round) nl = n_round;
    const size_t dyn = (size_t)(nl / per_word) * 4;
    NK_HIP(hipFuncSetAttribute(kr.fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)dyn));
    int occ = 0;
    NK_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, kr.fn, block, dyn));
    if (occ < 1) return fail(NK_E_INTERNAL, "multi-source kernel does not fit a compute unit (block %d)", block);
    if (t.wg_per_cu > 0 && t.wg_per_cu < occ) occ = t.wg_per_cu;
    const long long ntasks = (nsources + b - 1) / b;
    long long grid = (long long)di.cus * occ;
    if (ntasks < grid) grid = ntasks;
    if (grid < 1) grid = 1;
    const long long stride = (((long long)n_max + 2) + 63) / 64 * 64;
    const long long cap = stride * b;
    const long long visg_words = ((stride + per_word - 1) / per_word + 63) / 64 * 64;
    // per slot: interleaved path counts, new-source masks, four list arrays
    // of cap entries, level offsets, bottom-up candidates, global masks
    const size_t per_slot = (size_t)stride * b * 8 + (size_t)stride * 4 * 3 + (size_t)cap * 4 * 4 +
                            (size_t)visg_words * 4;
    size_t avail;
    if (t.scratch_mib > 0) {
        avail = (size_t)t.scratch_mib << 20;
    } else {
        size_t fr = 0, tot = 0;
        NK_HIP(hipMemGetInfo(&fr, &tot));
        avail = (size_t)((double)(fr + pool_bytes_idle()) * 0.85);
    }
    const long long fit = (long long)(avail / per_slot);
    if (fit < 1)
        return fail(NK_E_NO_MEMORY, "one multi-source workgroup slot needs %zu bytes of scratch; %zu available",
                    per_slot, avail);
    if (grid > fit) grid = fit > di.cus ? fit / di.cus * di.cus : fit;
    mp->b = b;
    mp->nl = (int32_t)nl;
    mp->stride = stride;
    mp->cap = cap;
    mp->visg_words = visg_words;
    mp->ntasks = ntasks;
    mp->lp.mode = kModeBC;
    mp->lp.block = block;
    mp->lp.lds = true;
    mp->lp.grid = (int)grid;
    mp->lp.dyn_lds = dyn;
    mp->lp.stride = stride;
    mp->lp.bm_words = 0;
    mp->lp.kernel = kr;
    mp->lp.pair_rec = nullptr;
    mp->lp.dag_words = 0;
    return NK_OK;
}

nk_status ms_alloc(const MsPlan &mp, Params &p, Scratch &scr) {
    const long long slots = mp.lp.grid;
    nk_status st;
    if ((st = scr.get(slots * mp.stride * mp.b, &p.sigma)) != NK_OK) return st;
    if ((st = scr.get(slots * mp.stride, &p.nx)) != NK_OK) return st;
    if ((st = scr.get(slots * mp.stride, &p.lvl)) != NK_OK) return st;
    if ((st = scr.get(slots * mp.stride, &p.cand)) != NK_OK) return st;
    if ((st = scr.get(slots * mp.cap, &p.lv)) != NK_OK) return st;
    if ((st = scr.get(slots * mp.cap, &p.la)) != NK_OK) return st;
    if ((st = scr.get(slots * mp.cap, &p.ld)) != NK_OK) return st;
    if ((st = scr.get(slots * mp.cap, &p.lm)) != NK_OK) return st;
    if ((st = scr.get(slots * mp.visg_words, &p.visg)) != NK_OK) return st;
    p.stride = mp.stride;
    p.ms_b = mp.b;
    p.ms_nl = mp.nl;
    p.ms_cap = mp.cap;
    p.visg_words = mp.visg_words;
    p.bu_ratio = tuning_get().bu_ratio;
    p.bw_ratio = tuning_get().bw_ratio;
    return NK_OK;
}

nk_status ms_enqueue(const MsPlan &mp, const Params &p, hipStream_t s, hipEvent_t ev0, hipEvent_t ev1) {
    const long long slots = mp.lp.grid;
    NK_HIP(launch_fill_u64(p.sigma, 0ULL, slots * mp.stride * mp.b, s));
    NK_HIP(launch_fill_u32(p.nx, 0u, slots * mp.stride, s));
    NK_HIP(launch_fill_u32(p.visg, 0u, slots * mp.visg_words, s));
    if (ev0) NK_HIP(hipEventRecord(ev0, s));
    mp.lp.kernel.launch(dim3(mp.lp.grid), dim3(mp.lp.block), mp.lp.dyn_lds, s, p);
    NK_HIP(hipGetLastError());
    if (ev1) NK_HIP(hipEventRecord(ev1, s));
    return NK_OK;
}

// ------------------------------------------------------------- group plan --

bool group_wanted(int32_t n_max, int64_t m_arcs) {
    const nk_tuning t = tuning_get();
    if ((t.flags & 16) || n_max < 1 || t.batch > 1) return false;
    // automatic: sparse graphs of 10^5 to 3 * 10^5 vertices, where sharing
    // a source between a few workgroups measured faster than one source per
    // workgroup (mean-degree-8 random and preferential-attachment graphs);
    // flag bit 3 asks for the group kernel on every graph it can take
    const bool autosel = n_max >= 100000 && n_max <= 300000 && m_arcs <= 12LL * n_max;
    if (!(t.flags & 8) && !autosel) return false;
    DevInfo di;
    if (dev_info(&di) != NK_OK) return false;
    const int block = t.block == 512 ? 512 : 1024;
    hipFuncAttributes attr;
    if (hipFuncGetAttributes(&attr, brandes_group_kernel(block).fn) != hipSuccess) return false;
    const size_t bm = (size_t)(((long long)n_max + 31) / 32) * 4;
    return attr.sharedSizeBytes + bm <= di.lds_per_block;
}

nk_status plan_group(int32_t n_max, GroupPlan *gp) {
    DevInfo di;
    nk_status st = dev_info(&di);
    if (st != NK_OK) return st;
    const nk_tuning t = tuning_get();
    const int block = t.block == 512 ? 512 : 1024;
    KernelRef kr = brandes_group_kernel(block);
    hipFuncAttributes attr;
    NK_HIP(hipFuncGetAttributes(&attr, kr.fn));
    const size_t dyn = (size_t)(((long long)n_max + 31) / 32) * 4;
    if (attr.sharedSizeBytes + dyn > di.lds_per_block)
        return fail(NK_E_INTERNAL, "group kernel: a bitmap of %d vertices does not fit LDS", n_max);
    NK_HIP(hipFuncSetAttribute(kr.fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)dyn));
    int occ = 0;
    NK_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, kr.fn, block, dyn));
    if (occ < 1) return fail(NK_E_INTERNAL, "group kernel does not fit a compute unit (block %d)", block);
    // one 1024-thread workgroup per compute unit, or two of 512 (one per
    // group of each XCD's two groups)
    const int per_cu = block == 512 ? std::min(occ, 2) : 1;
    int nxcc = 0;
    if (hipDeviceGetAttribute(&nxcc, hipDeviceAttributeNumberOfXccs, di.device) != hipSuccess || nxcc < 1) nxcc = 1;
    (void)hipGetLastError();
    int rate_khz = 0;
    if (hipDeviceGetAttribute(&rate_khz, hipDeviceAttributeWallClockRate, di.device) != hipSuccess || rate_khz < 1)
        rate_khz = 100000;
    (void)hipGetLastError();
    // workgroups per group: the tuning's, else 4 (measured fastest on the
    // mid-size graphs; whole-XCD groups leave each workgroup too few tiles
    // per level)
    const int per_xcd = std::max(1, di.cus * per_cu / nxcc);   // (one XCD has per_cu fewer)
    int gsz = t.group > 0 ? t.group : 4;
    if (gsz > per_xcd) gsz = per_xcd;
    gp->gpx = std::max(1, per_xcd / gsz);
    gp->groups = nxcc * gp->gpx;
    gp->nxcc = nxcc;
    gp->stride = (((long long)n_max + 2) + 63) / 64 * 64;
    gp->timeout = (long long)rate_khz * 1000LL * 20LL;   // 20 s
    gp->lp.mode = kModeBC;
    gp->lp.block = block;
    gp->lp.lds = true;
    // one compute unit stays free: a workgroup fills its compute unit's
    // vector registers, and the runtime's copy kernels (a progress read
    // while the launch runs) need a place to run
    gp->lp.grid = std::max(1, di.cus - 1) * per_cu;
    gp->lp.dyn_lds = dyn;
    gp->lp.stride = gp->stride;
    gp->lp.bm_words = 0;
    gp->lp.kernel = kr;
    gp->lp.pair_rec = nullptr;
    gp->lp.dag_words = 0;
    return NK_OK;
}

nk_status group_alloc(const GroupPlan &gp, Params &p, Scratch &scr) {
    const long long cells = (long long)gp.groups * gp.stride;
    nk_status st;
    if ((st = scr.get(cells, &p.sigma)) != NK_OK) return st;
    if ((st = scr.get(cells, &p.lv)) != NK_OK) return st;
    if ((st = scr.get(cells, &p.la)) != NK_OK) return st;
    if ((st = scr.get(cells, &p.ld)) != NK_OK) return st;
    if ((st = scr.get(cells, &p.lvl)) != NK_OK) return st;
    // bottom-up candidates: each member's segment holds the vertices of
    // every G-th bitmap word (G <= 64 members)
    const long long cstride = gp.stride + 64 * 32 + 64;
    if ((st = scr.get((long long)gp.groups * cstride, &p.cand)) != NK_OK) return st;
    p.xg_cand_stride = cstride;
    unsigned long long *ctl;
    if ((st = scr.get((long long)(gp.groups * group_ctl_bytes() / 8), &ctl)) != NK_OK) return st;
    if ((st = scr.get(32, &p.xg_reg)) != NK_OK) return st;
    p.xg_ctl = ctl;
    p.stride = gp.stride;
    p.xg_gpx = gp.gpx;
    p.xg_groups = gp.groups;
    p.xg_nxcc = gp.nxcc;
    p.xg_timeout = gp.timeout;
    p.bu_ratio = tuning_get().bu_ratio;
    p.bw_ratio = tuning_get().bw_ratio;
    return NK_OK;
}

nk_status group_enqueue(const GroupPlan &gp, const Params &p, hipStream_t s, hipEvent_t ev0, hipEvent_t ev1) {
    NK_HIP(launch_fill_u64(p.sigma, 0ULL, (long long)gp.groups * gp.stride, s));
    NK_HIP(launch_fill_u64(static_cast<unsigned long long *>(p.xg_ctl), 0ULL,
                           (long long)(gp.groups * group_ctl_bytes() / 8), s));
    NK_HIP(launch_fill_u32(p.xg_reg, 0u, 32, s));
    if (ev0) NK_HIP(hipEventRecord(ev0, s));
    hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
    NK_HIP(hipStreamIsCapturing(s, &cap));
    if (cap == hipStreamCaptureStatusNone) {
        // the runtime checks that the whole grid can be resident at once
        Params arg = p;
        void *args[] = {&arg};
        NK_HIP(hipLaunchCooperativeKernel(gp.lp.kernel.fn, dim3(gp.lp.grid), dim3(gp.lp.block), args,
                                          (unsigned int)gp.lp.dyn_lds, s));
    } else {
        // a captured plan runs alone on its stream, after the launches
        // before it, with the device otherwise idle; the registration
        // count inside the kernel still checks residency
        gp.lp.kernel.launch(dim3(gp.lp.grid), dim3(gp.lp.block), gp.lp.dyn_lds, s, p);
        NK_HIP(hipGetLastError());
    }
    if (ev1) NK_HIP(hipEventRecord(ev1, s));
    return NK_OK;
}

nk_status persistent_alloc(const LaunchPlan &plan, Params &p, Scratch &scr, hipStream_t s) {
    const long long slots = plan.grid;
    const long long cells = slots * plan.stride;
    nk_status st;
    const bool pair = plan.mode == kModePair || plan.mode == kModePairHash;
    p.sigma = nullptr;
    p.ls = p.ls2 = nullptr;
    p.ldeg = nullptr;
    p.d = nullptr;
    p.lvl = nullptr;
    p.bmg = nullptr;
    p.pair_rec = p.pair_blk = nullptr;
    p.lv2 = p.la2 = p.ld2 = nullptr;
    p.dist = nullptr;
    p.mark = nullptr;
    p.wl0 = p.wl1 = p.wl2 = nullptr;
    p.dagm = nullptr;
    p.dag_words = plan.dag_words;
    p.bvec = nullptr;
    if ((st = scr.get(cells, &p.dacc)) != NK_OK) return st;
    if ((st = scr.get(cells, &p.lv)) != NK_OK) return st;
    if ((st = scr.get(cells, &p.la)) != NK_OK) return st;
    if ((st = scr.get(cells, &p.ld)) != NK_OK) return st;
    if ((st = scr.get(cells, &p.cand)) != NK_OK) return st;
    if (pair) {
        // 32-byte records of both search sides, the target side's lists.
        // Every sample resets the records it touched, so a block left by a
        // successful pair launch is still all-unreached and needs no fill;
        // one record per vertex also holds the vertex's degree, refreshed
        // on the device when the graph's row pointers differ from the ones
        // the block was filled from (tables hold no degree).
        const bool hashed = plan.mode == kModePairHash;
        const long long head = hashed ? 0 : pair_block_head_bytes(plan.stride);
        bool clean = false;
        size_t blk_bytes = 0;
        void *blk = nullptr;
        if ((st = scr.get_tagged((size_t)cells * 32 + (size_t)head, pair_block_tag(plan), &blk, &clean,
                                 &blk_bytes)) != NK_OK)
            return st;
        p.pair_blk = blk;
        p.pair_rec = static_cast<char *>(blk) + head;
        if ((st = scr.get(cells, &p.lv2)) != NK_OK) return st;
        if ((st = scr.get(cells, &p.la2)) != NK_OK) return st;
        if ((st = scr.get(cells, &p.ld2)) != NK_OK) return st;
        if (hashed) {
            if ((st = scr.get(cells, &p.ls)) != NK_OK) return st;
            if ((st = scr.get(cells, &p.ls2)) != NK_OK) return st;
            if (!clean) NK_HIP(launch_pair_table_init(blk, (long long)(blk_bytes / 32), s));
        } else if (clean) {
            NK_HIP(launch_pair_block_refresh(blk, blk_bytes, plan.stride, p.rowptr, p.n, s));
        } else {
            NK_HIP(launch_pair_block_init(blk, blk_bytes, plan.stride, p.rowptr, p.n, s));
        }
    } else {
        if ((st = scr.get(cells, &p.sigma)) != NK_OK) return st;
        if ((st = scr.get(cells, &p.ldeg)) != NK_OK) return st;
        if ((st = scr.get(cells, &p.d)) != NK_OK) return st;
        if ((st = scr.get(cells, &p.lvl)) != NK_OK) return st;
        if (plan.mode == kModeWeighted) {
            if ((st = scr.get(cells, &p.dist)) != NK_OK) return st;
            if ((st = scr.get(cells, &p.mark)) != NK_OK) return st;
            if ((st = scr.get(cells, &p.wl0)) != NK_OK) return st;
            if ((st = scr.get(cells, &p.wl1)) != NK_OK) return st;
            if ((st = scr.get(cells, &p.wl2)) != NK_OK) return st;
            if ((st = scr.get(slots * plan.dag_words, &p.dagm)) != NK_OK) return st;
        }
        if (plan.mode == kModeBisect)
            if ((st = scr.get(cells * kBisK, &p.bvec)) != NK_OK) return st;
        if (!plan.lds)
            if ((st = scr.get(slots * plan.bm_words, &p.bmg)) != NK_OK) return st;
    }
    p.stride = plan.stride;
    p.bm_words = plan.bm_words;
    // a directed run without in-arcs grows every level top-down
    p.bu_ratio = (p.directed && !p.trowptr) ? 0.0f : tuning_get().bu_ratio;
    p.bw_ratio = tuning_get().bw_ratio;
    return NK_OK;
}

nk_status persistent_enqueue(const LaunchPlan &plan, const Params &p, hipStream_t s, hipEvent_t ev0, hipEvent_t ev1) {
    if (plan.mode != kModePair && plan.mode != kModePairHash) {
        const long long cells = (long long)plan.grid * plan.stride;
        if (plan.mode == kModeWeighted) {
            NK_HIP(launch_fill_u64(p.dist, ~0ULL, cells, s));
            NK_HIP(launch_fill_i32(p.mark, -1, cells, s));
            NK_HIP(launch_fill_i32(p.d, 0, cells, s));   // far-pile flags
            NK_HIP(launch_fill_u32(p.dagm, 0u, (long long)plan.grid * plan.dag_words, s));
        }
        NK_HIP(launch_fill_u64(p.sigma, 0ULL, cells, s));
        // the push accumulator of the dependency sweep must start at zero
        if (plan.mode == kModeBC || plan.mode == kModeBisect) NK_HIP(launch_fill_f64(p.dacc, 0.0, cells, s));
    }
    if (ev0) NK_HIP(hipEventRecord(ev0, s));
    plan.kernel.launch(dim3(plan.grid), dim3(plan.block), plan.dyn_lds, s, p);
    NK_HIP(hipGetLastError());
    if (ev1) NK_HIP(hipEventRecord(ev1, s));
    return NK_OK;
}

nk_status launch_persistent(const LaunchPlan &plan, Params &p, Scratch &scr, hipStream_t s, hipEvent_t ev0,
                            hipEvent_t ev1) {
    nk_status st = persistent_alloc(plan, p, scr, s);
    if (st != NK_OK) return st;
    return persistent_enqueue(plan, p, s, ev0, ev1);
}

// --------------------------------------------------------- vertex diameter --

// Vertex-diameter bound: the maximum-degree vertex, a grid-wide sweep from
// it, the largest component it missed, and a second sweep from the lowest
// far vertex (info layout as nk_vd_bound).
nk_status vd_bound_impl(const int32_t *rowptr, const int32_t *colidx, int32_t n, int64_t m, int32_t *info,
                        hipStream_t s, bool lower) {
    for (int i = 0; i < 8; ++i) info[i] = 0;
    if (n == 0) return NK_OK;
    Scratch scr;
    DevStatus *dst;
    unsigned long long *key;
    int32_t *label, *size, *flag;
    BfsWork w;
    nk_status st;
    if ((st = scr.get(1, &dst)) != NK_OK) return st;
    if ((st = scr.get(1, &key)) != NK_OK) return st;
    if ((st = bfs_work_get(scr, n, s, &w)) != NK_OK) return st;
    if ((st = scr.get(n, &label)) != NK_OK) return st;
    if ((st = scr.get(n, &size)) != NK_OK) return st;
    if ((st = scr.get(2, &flag)) != NK_OK) return st;
    DevStatus *h = host_status();
    if (!h) return fail(NK_E_NO_MEMORY, "pinned status buffer");
    NK_HIP(launch_status_init(dst, s));
    NK_HIP(launch_validate(rowptr, colidx, n, m, 0, dst, s));
    NK_HIP(launch_fill_u64(key, 0ULL, 1, s));
    NK_HIP(launch_argmax_degree(rowptr, n, key, s));
    // (the status read synchronises the stream, so the key has arrived too)
    unsigned long long k = 0;
    NK_HIP(hipMemcpyAsync(&k, key, 8, hipMemcpyDeviceToHost, s));
    if ((st = finish(dst, h, s)) != NK_OK) return st;
    const int32_t x0 = (int32_t)(0xffffffffULL - (k & 0xffffffffULL));
    // first sweep from x0 (its degree is the key's high word): e1, the
    // lowest far vertex a (for the second sweep only), and |C(x0)|
    int32_t r1[3], r2[3];
    if ((st = grid_bfs(rowptr, colidx, n, m, x0, w, s, r1, (int32_t)(k >> 32), lower)) != NK_OK) return st;
    const int32_t e1 = r1[0], a = r1[1], c0 = r1[2];
    // largest component among the vertices the first sweep did not reach
    int32_t c2 = 0;
    if (c0 < n)
        if ((st = largest_unreached_component(rowptr, colidx, n, w.d, label, size, flag, s, &c2)) != NK_OK) return st;
    // second sweep from a (the lower bound only)
    int32_t e2 = -1;
    if (lower) {
        if ((st = grid_bfs(rowptr, colidx, n, m, a, w, s, r2)) != NK_OK) return st;
        e2 = r2[0];
    }
    int32_t ub = 2 * e1 + 1;
    if (ub > c0) ub = c0;
    if (c2 > ub) ub = c2;
    info[0] = x0;
    info[1] = e1;
    info[2] = a;
    info[3] = e2;
    info[4] = ub;
    info[5] = e2 + 1;
    info[6] = c0;
    info[7] = c2;
    return NK_OK;
}

}  // namespace nk

using namespace nk;

// ==================================================================== C ABI ==

extern "C" {

const char *nk_last_error(void) { return t_err.c_str(); }

const char *nk_version(void) { return "nkbc 0.1 (gfx950)"; }

void nk_shutdown(void) { pool_clear(); }

nk_status nk_last_stats(int64_t *out) {
    if (!out) return fail(NK_E_INVALID_ARG, "out is NULL");
    memcpy(out, t_stats, sizeof(t_stats));
    return NK_OK;
}

nk_status nk_set_tuning(const nk_tuning *t) {
    clear_error();
    if (!t) return fail(NK_E_INVALID_ARG, "tuning is NULL");
    if (t->block != 0 && t->block != 256 && t->block != 512 && t->block != 1024)
        return fail(NK_E_INVALID_ARG, "block must be 0, 256, 512 or 1024");
    if (!(t->bu_ratio >= 0.0f) || !(t->bw_ratio >= 0.0f) || t->wg_per_cu < 0 || t->scratch_mib < 0)
        return fail(NK_E_INVALID_ARG, "bad tuning values");
    if (t->batch != 0 && t->batch != 1 && t->batch != 4 && t->batch != 8 && t->batch != 16)
        return fail(NK_E_INVALID_ARG, "batch must be 0, 1, 4, 8 or 16");
    if (t->group < 0 || t->group > 64 || (t->group & (t->group - 1)) != 0)
        return fail(NK_E_INVALID_ARG, "group must be 0 or a power of two up to 64");
    tuning_set(*t);
    return NK_OK;
}

nk_status nk_get_tuning(nk_tuning *t) {
    if (!t) return fail(NK_E_INVALID_ARG, "tuning is NULL");
    *t = tuning_get();
    return NK_OK;
}

nk_status nk_validate_graph(const int32_t *rowptr, const int32_t *colidx, int32_t n, int64_t m, int32_t strict,
                            void *stream) {
    clear_error();
    nk_status st = check_graph_args(rowptr, colidx, n, m);
    if (st != NK_OK || n == 0) return st;
    hipStream_t s = (hipStream_t)stream;
    Scratch scr;
    DevStatus *dst;
    if ((st = scr.get(1, &dst)) != NK_OK) return st;
    NK_HIP(launch_status_init(dst, s));
    NK_HIP(launch_validate(rowptr, colidx, n, m, strict, dst, s));
    DevStatus *h = host_status();
    if (!h) return fail(NK_E_NO_MEMORY, "pinned status buffer");
    return finish(dst, h, s);
}

// The graph a single-graph call runs on: degree-relabelled unless tuning
// flag bit 1 is set or the graph is tiny.
static nk_status prepare_graph(const int32_t *rowptr, const int32_t *colidx, int32_t n, int64_t m, DevStatus *dst,
                               Scratch &scr, hipStream_t s, Relabeled *g) {
    g->rowptr = rowptr;
    g->colidx = colidx;
    g->perm = nullptr;
    g->inv = nullptr;
    if ((tuning_get().flags & 2) || n < 256) return NK_OK;
    return relabel_graph(rowptr, colidx, n, m, dst, scr, s, g);
}

// Estimators of the source-sampled sweep.
enum Estimator : int { kEstPlain = 0, kEstLinear = 1, kEstBisect = 2 };

// A directed run: rowptr/colidx are out-arcs; trp/tci the in-arcs or NULL.
struct DirectedArgs {
    const int32_t *trp;
    const int32_t *tci;
};

// Shared body of nk_bc_exact / nk_bc_sources / nk_bc_sources_linear /
// nk_bc_sources_bisect / nk_edge_bc.  est selects the estimator; ebc !=
// NULL also computes edge scores (global kernel, graph under its own ids).
static nk_status bc_sources_impl(const int32_t *rowptr, const int32_t *colidx, int32_t n, int64_t m,
                                 const int32_t *sources, long long k, double scale, double *bc, void *stream,
                                 int est = kEstPlain, double *ebc = nullptr, const DirectedArgs *dir = nullptr) {
    clear_error();
    stats_clear();
    nk_status st = check_graph_args(rowptr, colidx, n, m);
    if (st != NK_OK) return st;
    if (n == 0) return NK_OK;
    if (!bc) return fail(NK_E_INVALID_ARG, "bc is NULL");
    if (k < 0) return fail(NK_E_INVALID_ARG, "k is negative");
    if (k > 0 && !sources && k != n) return fail(NK_E_INVALID_ARG, "sources is NULL");
    hipStream_t s = (hipStream_t)stream;
    // a registered autotuner cache supplies the tuning for this graph's shape
    nk_tuning cached;
    bool use_cached = false;
    if (tuning_cache_active()) {
        int64_t dmax = 0;
        if ((st = graph_max_degree(rowptr, n, s, &dmax)) != NK_OK) return st;
        use_cached = cached_tuning(n, m, dmax, &cached);
    }
    TuningOverride cached_scope(use_cached ? &cached : nullptr);
    Scratch scr;
    DevStatus *dst;
    uint32_t *iso;
    const long long words = ((long long)n + 31) / 32;
    if ((st = scr.get(1, &dst)) != NK_OK) return st;
    if ((st = scr.get(words, &iso)) != NK_OK) return st;
    DevStatus *h = host_status();
    if (!h) return fail(NK_E_NO_MEMORY, "pinned status buffer");
    NK_HIP(launch_status_init(dst, s));
    NK_HIP(launch_validate(rowptr, colidx, n, m, 0, dst, s));
    if (dir && dir->trp) {
        // the in-arcs must be the out-arcs' transpose (checked: structure
        // and every vertex's in-degree)
        NK_HIP(launch_validate(dir->trp, dir->tci, n, m, 0, dst, s));
        if ((st = check_transpose(colidx, n, m, dir->trp, dst, scr, s)) != NK_OK) return st;
    }
    NK_HIP(launch_fill_f64(bc, 0.0, n, s));
    if (ebc) NK_HIP(launch_fill_f64(ebc, 0.0, m, s));
    LaunchPlan plan = {};
    float ms = 0.0f;
    int where = 0;
    // (the all-in-LDS kernel has no bisection sweeps)
    if (k > 0 && !ebc && est != kEstBisect && plan_lds(lds_graph_bytes(n, m), n, k, &plan)) {
        // the whole graph fits one workgroup's LDS: no relabelling, no scratch
        Params p;
        memset(&p, 0, sizeof(p));
        p.rowptr = rowptr;
        p.colidx = colidx;
        p.n = n;
        p.m = (int32_t)m;
        p.ntasks = k;
        p.sources = sources;
        p.bc = bc;
        p.st = dst;
        p.linear = est == kEstLinear;
        hipEvent_t ev0, ev1;
        if ((st = thread_events(&ev0, &ev1)) != NK_OK) return st;
        NK_HIP(hipEventRecord(ev0, s));
        plan.kernel.launch(dim3(plan.grid), dim3(plan.block), plan.dyn_lds, s, p);
        NK_HIP(hipGetLastError());
        NK_HIP(hipEventRecord(ev1, s));
        if (scale != 1.0) NK_HIP(launch_scale_f64(bc, scale, n, s));
        st = finish(dst, h, s);
        NK_HIP(hipEventElapsedTime(&ms, ev0, ev1));
        where = 2;
    } else if (k > 0) {
        where = -1;
        Relabeled g = {rowptr, colidx, nullptr, nullptr};
        if ((st = prepare_graph(rowptr, colidx, n, m, dst, scr, s, &g)) != NK_OK) return st;
        // a directed run renames its in-arcs with the same permutation
        DirectedArgs dir_run = {nullptr, nullptr};
        if (dir) {
            dir_run = *dir;
            if (dir->trp && g.perm) {
                int32_t *trp_new, *tci_new;
                if ((st = relabel_second_csr(dir->trp, dir->tci, n, m, g, dst, scr, s, &trp_new, &tci_new)) != NK_OK)
                    return st;
                dir_run = {trp_new, tci_new};
            }
            dir = &dir_run;
        }
        // edge scores of a relabelled run go to the relabelled arc order
        // first, then back to the caller's
        double *ebc_run = ebc;
        if (ebc && g.perm) {
            if ((st = scr.get(m > 0 ? m : 1, &ebc_run)) != NK_OK) return st;
            NK_HIP(launch_fill_f64(ebc_run, 0.0, m, s));
        }
        // vertices no search can reach: no arcs (undirected) or no in-arcs
        // (directed; unknown without the in-arc CSR)
        if (dir)
            iso = dir->trp ? iso : nullptr;
        if (iso) NK_HIP(launch_iso_bitmap(dir ? dir->trp : g.rowptr, n, iso, s));
        const int32_t *src = sources;
        double *acc = bc;
        if (g.perm) {
            if (sources) {
                int32_t *mapped;
                if ((st = scr.get(k, &mapped)) != NK_OK) return st;
                NK_HIP(launch_map_sources(sources, (int32_t)k, g.perm, n, mapped, s));
                src = mapped;
            }
            if ((st = scr.get(n, &acc)) != NK_OK) return st;
            NK_HIP(launch_fill_f64(acc, 0.0, n, s));
        }
        // plain and linear-scaling sweeps of undirected graphs without edge
        // scores may run one source per XCD group of workgroups
        if (!ebc && !dir && est != kEstBisect && group_wanted(n, m)) {
            GroupPlan gp;
            if ((st = plan_group(n, &gp)) != NK_OK) return st;
            Params p;
            memset(&p, 0, sizeof(p));
            p.rowptr = g.rowptr;
            p.colidx = g.colidx;
            p.n = n;
            p.m = (int32_t)m;
            p.sources = src;
            p.ntasks = k;
            p.bc = acc;
            p.iso = iso;
            p.st = dst;
            p.linear = est == kEstLinear;
            if ((st = group_alloc(gp, p, scr)) != NK_OK) return st;
            hipEvent_t ev0, ev1;
            if ((st = thread_events(&ev0, &ev1)) != NK_OK) return st;
            if ((st = group_enqueue(gp, p, s, ev0, ev1)) != NK_OK) return st;
            if (g.perm)
                NK_HIP(launch_gather_scale(acc, g.perm, n, scale, bc, s));
            else if (scale != 1.0)
                NK_HIP(launch_scale_f64(bc, scale, n, s));
            st = finish(dst, h, s);
            NK_HIP(hipEventElapsedTime(&ms, ev0, ev1));
            stats_record(*h, gp.lp.grid, gp.lp.block, 6, ms);
            return st;
        }
        // or several sources per task
        const int msb = (!ebc && !dir && est != kEstBisect) ? ms_batch_for(n, k) : 1;
        if (msb > 1) {
            MsPlan mp;
            if ((st = plan_ms(msb, n, k, &mp)) != NK_OK) return st;
            Params p;
            memset(&p, 0, sizeof(p));
            p.rowptr = g.rowptr;
            p.colidx = g.colidx;
            p.n = n;
            p.m = (int32_t)m;
            p.sources = src;
            p.nsources = k;
            p.ntasks = mp.ntasks;
            p.bc = acc;
            p.iso = iso;
            p.st = dst;
            p.linear = est == kEstLinear;
            if ((st = ms_alloc(mp, p, scr)) != NK_OK) return st;
            hipEvent_t ev0, ev1;
            if ((st = thread_events(&ev0, &ev1)) != NK_OK) return st;
            if ((st = ms_enqueue(mp, p, s, ev0, ev1)) != NK_OK) return st;
            if (g.perm)
                NK_HIP(launch_gather_scale(acc, g.perm, n, scale, bc, s));
            else if (scale != 1.0)
                NK_HIP(launch_scale_f64(bc, scale, n, s));
            st = finish(dst, h, s);
            NK_HIP(hipEventElapsedTime(&ms, ev0, ev1));
            stats_record(*h, mp.lp.grid, mp.lp.block, 4, ms);
            stats_set_batch(msb);
            return st;
        }
        if ((st = plan_launch(est == kEstBisect ? kModeBisect : kModeBC, n, k, 0, &plan)) != NK_OK) return st;
        Params p;
        memset(&p, 0, sizeof(p));
        p.rowptr = g.rowptr;
        p.colidx = g.colidx;
        p.n = n;
        p.m = (int32_t)m;
        p.ntasks = k;
        p.sources = src;
        p.bc = acc;
        p.iso = iso;
        p.st = dst;
        p.linear = est == kEstLinear;
        p.ebc = ebc_run;
        p.directed = dir != nullptr;
        p.trowptr = dir ? dir->trp : nullptr;
        p.tcolidx = dir ? dir->tci : nullptr;
        hipEvent_t ev0, ev1;
        if ((st = thread_events(&ev0, &ev1)) != NK_OK) return st;
        if ((st = launch_persistent(plan, p, scr, s, ev0, ev1)) != NK_OK) return st;
        if (g.perm)
            NK_HIP(launch_gather_scale(acc, g.perm, n, scale, bc, s));
        else if (scale != 1.0)
            NK_HIP(launch_scale_f64(bc, scale, n, s));
        if (ebc && g.perm) NK_HIP(launch_arcs_back(ebc_run, g.rowptr, g.inv, rowptr, n, ebc, s));
        if (ebc) NK_HIP(launch_edge_symmetrize(rowptr, colidx, n, ebc, scale, dst, s));
        st = finish(dst, h, s);
        NK_HIP(hipEventElapsedTime(&ms, ev0, ev1));
    } else {
        st = finish(dst, h, s);
    }
    if (where < 0) where = plan.lds ? 1 : 0;
    stats_record(*h, plan.grid, plan.block, where, ms);
    return st;
}

nk_status nk_bc_exact(const int32_t *rowptr, const int32_t *colidx, int32_t n, int64_t m, double *bc,
                      void *stream) {
    return bc_sources_impl(rowptr, colidx, n, m, nullptr, n, 1.0, bc, stream);
}

nk_status nk_bc_sources(const int32_t *rowptr, const int32_t *colidx, int32_t n, int64_t m, const int32_t *sources,
                        int32_t k, double scale, double *bc, void *stream) {
    if (k > 0 && !sources) {
        clear_error();
        return fail(NK_E_INVALID_ARG, "sources is NULL");
    }
    return bc_sources_impl(rowptr, colidx, n, m, sources, k, scale, bc, stream);
}

nk_status nk_bc_sources_linear(const int32_t *rowptr, const int32_t *colidx, int32_t n, int64_t m,
                               const int32_t *sources, int32_t k, double scale, double *bc, void *stream) {
    if (k > 0 && !sources && k != n) {
        clear_error();
        return fail(NK_E_INVALID_ARG, "sources is NULL");
    }
    return bc_sources_impl(rowptr, colidx, n, m, sources, k, scale, bc, stream, kEstLinear);
}

nk_status nk_bc_directed(const int32_t *rowptr, const int32_t *colidx, const int32_t *trowptr,
                         const int32_t *tcolidx, int32_t n, int64_t m, const int32_t *sources, int32_t k,
                         double scale, double *bc, void *stream) {
    clear_error();
    if (k > 0 && !sources && k != n) return fail(NK_E_INVALID_ARG, "sources is NULL");
    if ((!trowptr && tcolidx) || (trowptr && !tcolidx && m > 0))
        return fail(NK_E_INVALID_ARG, "give both in-arc arrays or neither");
    const DirectedArgs dir = {trowptr, tcolidx};
    return bc_sources_impl(rowptr, colidx, n, m, sources, k, scale, bc, stream, kEstPlain, nullptr, &dir);
}

nk_status nk_bc_weighted(const int32_t *rowptr, const int32_t *colidx, const int32_t *weights, int32_t n,
                         int64_t m, const int32_t *sources, int32_t k, double scale, double *bc, void *stream) {
    clear_error();
    stats_clear();
    nk_status st = check_graph_args(rowptr, colidx, n, m);
    if (st != NK_OK) return st;
    if (n == 0) return NK_OK;
    if (!bc) return fail(NK_E_INVALID_ARG, "bc is NULL");
    if (m > 0 && !weights) return fail(NK_E_INVALID_ARG, "weights is NULL");
    if (k < 0) return fail(NK_E_INVALID_ARG, "k is negative");
    if (k > 0 && !sources && k != n) return fail(NK_E_INVALID_ARG, "sources is NULL");
    hipStream_t s = (hipStream_t)stream;
    Scratch scr;
    DevStatus *dst;
    if ((st = scr.get(1, &dst)) != NK_OK) return st;
    DevStatus *h = host_status();
    if (!h) return fail(NK_E_NO_MEMORY, "pinned status buffer");
    NK_HIP(launch_status_init(dst, s));
    NK_HIP(launch_validate(rowptr, colidx, n, m, 0, dst, s));
    if (m > 0) NK_HIP(launch_validate_weights(weights, m, dst, s));
    NK_HIP(launch_fill_f64(bc, 0.0, n, s));
    LaunchPlan plan = {};
    float ms = 0.0f;
    if (k > 0) {
        // near-far threshold step: an eighth of the mean arc weight (on
        // R-MAT-20 with weights 1..64 the distance rounds relaxed 2.1x the
        // reached arcs in one bucket, 1.8x at the mean weight, 1.25x at a
        // quarter of it; with settled vertices skipped, an eighth (step 4)
        // ran 5% faster than a quarter and a sixteenth (step 2) 2% slower)
        long long wdelta = 0;
        if (m > 0) {
            unsigned long long *wsum;
            if ((st = scr.get(1, &wsum)) != NK_OK) return st;
            NK_HIP(launch_fill_u64(wsum, 0ULL, 1, s));
            NK_HIP(launch_sum_weights(weights, m, wsum, s));
            unsigned long long hsum = 0;
            NK_HIP(hipMemcpyAsync(&hsum, wsum, 8, hipMemcpyDeviceToHost, s));
            NK_HIP(hipStreamSynchronize(s));
            wdelta = (long long)(hsum / (unsigned long long)m) / 8;
            if (wdelta < 1) wdelta = 1;
        }
        // degree order, with the weights carried to the renamed arcs
        Relabeled g = {rowptr, colidx, nullptr, nullptr};
        if ((st = prepare_graph(rowptr, colidx, n, m, dst, scr, s, &g)) != NK_OK) return st;
        const int32_t *wts = weights, *src = sources;
        double *acc = bc;
        if (g.perm) {
            int32_t *w_new;
            if ((st = relabel_weights(weights, rowptr, n, m, g, dst, scr, s, &w_new)) != NK_OK) return st;
            wts = w_new;
            if (sources) {
                int32_t *mapped;
                if ((st = scr.get(k, &mapped)) != NK_OK) return st;
                NK_HIP(launch_map_sources(sources, k, g.perm, n, mapped, s));
                src = mapped;
            }
            if ((st = scr.get(n, &acc)) != NK_OK) return st;
            NK_HIP(launch_fill_f64(acc, 0.0, n, s));
        }
        if ((st = plan_launch(kModeWeighted, n, k, 0, &plan, m)) != NK_OK) return st;
        Params p;
        memset(&p, 0, sizeof(p));
        p.rowptr = g.rowptr;
        p.colidx = g.colidx;
        p.n = n;
        p.m = (int32_t)m;
        p.ntasks = k;
        p.sources = src;
        p.bc = acc;
        p.st = dst;
        p.wts = wts;
        p.wdelta = wdelta;
        hipEvent_t ev0, ev1;
        if ((st = thread_events(&ev0, &ev1)) != NK_OK) return st;
        if ((st = launch_persistent(plan, p, scr, s, ev0, ev1)) != NK_OK) return st;
        if (g.perm)
            NK_HIP(launch_gather_scale(acc, g.perm, n, scale, bc, s));
        else if (scale != 1.0)
            NK_HIP(launch_scale_f64(bc, scale, n, s));
        st = finish(dst, h, s);
        NK_HIP(hipEventElapsedTime(&ms, ev0, ev1));
    } else {
        st = finish(dst, h, s);
    }
    stats_record(*h, plan.grid, plan.block, plan.lds ? 1 : 0, ms);
    return st;
}

nk_status nk_transpose(const int32_t *rowptr, const int32_t *colidx, int32_t n, int64_t m, int32_t *trowptr,
                       int32_t *tcolidx, void *stream) {
    clear_error();
    stats_clear();
    nk_status st = check_graph_args(rowptr, colidx, n, m);
    if (st != NK_OK) return st;
    if (!trowptr || (m > 0 && !tcolidx)) return fail(NK_E_INVALID_ARG, "output arrays are NULL");
    hipStream_t s = (hipStream_t)stream;
    if (n == 0) {
        NK_HIP(launch_fill_i32(trowptr, 0, 1, s));
        NK_HIP(hipStreamSynchronize(s));
        return NK_OK;
    }
    Scratch scr;
    DevStatus *dst;
    if ((st = scr.get(1, &dst)) != NK_OK) return st;
    DevStatus *h = host_status();
    if (!h) return fail(NK_E_NO_MEMORY, "pinned status buffer");
    // the arc heads index the output rows: validate before building
    NK_HIP(launch_status_init(dst, s));
    NK_HIP(launch_validate(rowptr, colidx, n, m, 0, dst, s));
    if ((st = finish(dst, h, s)) != NK_OK) return st;
    if ((st = transpose_graph(rowptr, colidx, n, m, trowptr, tcolidx, scr, s)) != NK_OK) return st;
    NK_HIP(hipStreamSynchronize(s));
    return NK_OK;
}

nk_status nk_bc_sources_bisect(const int32_t *rowptr, const int32_t *colidx, int32_t n, int64_t m,
                               const int32_t *sources, int32_t k, double scale, double *bc, void *stream) {
    if (k > 0 && !sources && k != n) {
        clear_error();
        return fail(NK_E_INVALID_ARG, "sources is NULL");
    }
    return bc_sources_impl(rowptr, colidx, n, m, sources, k, scale, bc, stream, kEstBisect);
}

nk_status nk_edge_bc(const int32_t *rowptr, const int32_t *colidx, int32_t n, int64_t m, const int32_t *sources,
                     int32_t k, double scale, double *ebc, double *bc, void *stream) {
    clear_error();
    if (k > 0 && !sources && k != n) return fail(NK_E_INVALID_ARG, "sources is NULL");
    if (m > 0 && !ebc) return fail(NK_E_INVALID_ARG, "ebc is NULL");
    if (n < 0) return fail(NK_E_INVALID_ARG, "n = %d is negative", n);
    if (n == 0) {
        stats_clear();
        return NK_OK;
    }
    double *vb = bc;
    Scratch scr;
    if (!vb) {
        nk_status st = scr.get(n, &vb);
        if (st != NK_OK) return st;
    }
    if (m == 0) {
        // no arcs: every score is zero (the edge array is empty)
        return bc_sources_impl(rowptr, colidx, n, m, sources, k, scale, vb, stream);
    }
    return bc_sources_impl(rowptr, colidx, n, m, sources, k, scale, vb, stream, 0, ebc);
}

// Shared body of nk_closeness (sources NULL: every vertex, exact form into
// out by source) and nk_closeness_sampled (Eppstein-Wang form over sources).
static nk_status closeness_impl(const int32_t *rowptr, const int32_t *colidx, int32_t n, int64_t m,
                                const int32_t *sources, int32_t k, double *out, void *stream) {
    clear_error();
    stats_clear();
    nk_status st = check_graph_args(rowptr, colidx, n, m);
    if (st != NK_OK) return st;
    if (n == 0) return NK_OK;
    if (!out) return fail(NK_E_INVALID_ARG, "out is NULL");
    const bool sampled = sources != nullptr || k != n;
    if (k < 0 || (sampled && k > 0 && !sources)) return fail(NK_E_INVALID_ARG, "bad sources");
    hipStream_t s = (hipStream_t)stream;
    Scratch scr;
    DevStatus *dst;
    uint32_t *iso;
    unsigned long long *acc = nullptr;
    const long long words = ((long long)n + 31) / 32;
    if ((st = scr.get(1, &dst)) != NK_OK) return st;
    if ((st = scr.get(words, &iso)) != NK_OK) return st;
    DevStatus *h = host_status();
    if (!h) return fail(NK_E_NO_MEMORY, "pinned status buffer");
    NK_HIP(launch_status_init(dst, s));
    NK_HIP(launch_validate(rowptr, colidx, n, m, 0, dst, s));
    NK_HIP(launch_fill_f64(out, 0.0, n, s));
    LaunchPlan plan = {};
    float ms = 0.0f;
    if (k > 0) {
        Relabeled g;
        if ((st = prepare_graph(rowptr, colidx, n, m, dst, scr, s, &g)) != NK_OK) return st;
        NK_HIP(launch_iso_bitmap(g.rowptr, n, iso, s));
        const int32_t *src = sources;
        if (g.perm && sources) {
            int32_t *mapped;
            if ((st = scr.get(k, &mapped)) != NK_OK) return st;
            NK_HIP(launch_map_sources(sources, k, g.perm, n, mapped, s));
            src = mapped;
        }
        if (sampled) {
            if ((st = scr.get(n, &acc)) != NK_OK) return st;
            NK_HIP(launch_fill_u64(acc, 0ULL, n, s));
        }
        if ((st = plan_launch(kModeClose, n, k, 0, &plan)) != NK_OK) return st;
        Params p;
        memset(&p, 0, sizeof(p));
        p.rowptr = g.rowptr;
        p.colidx = g.colidx;
        p.n = n;
        p.m = (int32_t)m;
        p.ntasks = k;
        p.sources = src;
        p.inv = g.inv;
        p.iso = iso;
        p.st = dst;
        p.close_out = sampled ? nullptr : out;
        p.close_acc = acc;
        hipEvent_t ev0, ev1;
        if ((st = thread_events(&ev0, &ev1)) != NK_OK) return st;
        if ((st = launch_persistent(plan, p, scr, s, ev0, ev1)) != NK_OK) return st;
        if (sampled) NK_HIP(launch_close_finish(acc, g.perm, n, k, out, s));
        st = finish(dst, h, s);
        NK_HIP(hipEventElapsedTime(&ms, ev0, ev1));
    } else {
        st = finish(dst, h, s);
    }
    stats_record(*h, plan.grid, plan.block, plan.lds, ms);
    return st;
}

nk_status nk_closeness(const int32_t *rowptr, const int32_t *colidx, int32_t n, int64_t m, double *out,
                       void *stream) {
    return closeness_impl(rowptr, colidx, n, m, nullptr, n, out, stream);
}

nk_status nk_closeness_sampled(const int32_t *rowptr, const int32_t *colidx, int32_t n, int64_t m,
                               const int32_t *sources, int32_t k, double *out, void *stream) {
    if (k > 0 && !sources) {
        clear_error();
        return fail(NK_E_INVALID_ARG, "sources is NULL");
    }
    if (k == 0) {
        // no sources: every estimate is 0 (keeps the exact form out of reach)
        return closeness_impl(rowptr, colidx, n, m, nullptr, 0, out, stream);
    }
    return closeness_impl(rowptr, colidx, n, m, sources, k, out, stream);
}

nk_status nk_sssp_counts(const int32_t *rowptr, const int32_t *colidx, int32_t n, int64_t m,
                         const int32_t *sources, int32_t k, int32_t *d, uint64_t *sigma, void *stream) {
    clear_error();
    stats_clear();
    nk_status st = check_graph_args(rowptr, colidx, n, m);
    if (st != NK_OK) return st;
    if (n == 0 || k == 0) return NK_OK;
    if (k < 0 || !sources || !d || !sigma) return fail(NK_E_INVALID_ARG, "bad sources / outputs");
    hipStream_t s = (hipStream_t)stream;
    Scratch scr;
    DevStatus *dst;
    uint32_t *iso;
    const long long words = ((long long)n + 31) / 32;
    if ((st = scr.get(1, &dst)) != NK_OK) return st;
    if ((st = scr.get(words, &iso)) != NK_OK) return st;
    DevStatus *h = host_status();
    if (!h) return fail(NK_E_NO_MEMORY, "pinned status buffer");
    NK_HIP(launch_status_init(dst, s));
    NK_HIP(launch_validate(rowptr, colidx, n, m, 0, dst, s));
    Relabeled g;
    if ((st = prepare_graph(rowptr, colidx, n, m, dst, scr, s, &g)) != NK_OK) return st;
    NK_HIP(launch_iso_bitmap(g.rowptr, n, iso, s));
    const int32_t *src = sources;
    if (g.perm) {
        int32_t *mapped;
        if ((st = scr.get(k, &mapped)) != NK_OK) return st;
        NK_HIP(launch_map_sources(sources, k, g.perm, n, mapped, s));
        src = mapped;
    }
    NK_HIP(launch_fill_i32(d, -1, (long long)k * n, s));
    NK_HIP(launch_fill_u64((unsigned long long *)sigma, 0ULL, (long long)k * n, s));
    LaunchPlan plan;
    if ((st = plan_launch(kModeSSSP, n, k, 0, &plan)) != NK_OK) return st;
    Params p;
    memset(&p, 0, sizeof(p));
    p.rowptr = g.rowptr;
    p.colidx = g.colidx;
    p.n = n;
    p.m = (int32_t)m;
    p.ntasks = k;
    p.sources = src;
    p.d_out = d;
    p.sigma_out = (unsigned long long *)sigma;
    p.inv = g.inv;
    p.iso = iso;
    p.st = dst;
    if ((st = launch_persistent(plan, p, scr, s, nullptr, nullptr)) != NK_OK) return st;
    st = finish(dst, h, s);
    stats_record(*h, plan.grid, plan.block, plan.lds, 0.0f);
    return st;
}

nk_status nk_vd_bound(const int32_t *rowptr, const int32_t *colidx, int32_t n, int64_t m, int32_t *info,
                      void *stream) {
    clear_error();
    nk_status st = check_graph_args(rowptr, colidx, n, m);
    if (st != NK_OK) return st;
    if (!info) return fail(NK_E_INVALID_ARG, "info is NULL");
    return vd_bound_impl(rowptr, colidx, n, m, info, (hipStream_t)stream);
}

int64_t nk_rk_sample_size(double eps, double delta, int32_t vd) {
    if (!(eps > 0.0 && eps < 1.0) || !(delta > 0.0 && delta < 1.0)) return -1;
    int64_t x = (int64_t)vd - 2;
    if (x < 1) x = 1;
    int32_t fl = 0;
    while ((x >> (fl + 1)) > 0) ++fl;
    const double k = (double)(fl + 1) + (-log(delta));
    const double rr = 0.5 / (eps * eps) * k;
    return (int64_t)ceil(rr);
}

// Runs samples j0 .. j0+count-1 in pair mode.  counts (original ids) is
// accumulated, not cleared.
static nk_status pair_run(const int32_t *rowptr, const int32_t *colidx, int32_t n, int64_t m, long long count,
                          unsigned long long seed, long long j0, uint32_t *counts, int32_t *uv, int32_t *len,
                          int32_t *path, int32_t maxlen, DevStatus *dst, Scratch &scr, hipStream_t s,
                          LaunchPlan *plan_out, hipEvent_t ev0, hipEvent_t ev1) {
    nk_status st;
    // The graph runs under the caller's ids: a pair sample touches a few
    // thousand vertices, and degree relabelling (a pass over every arc per
    // call) left the pair kernel's time unchanged on Chung-Lu, R-MAT and
    // Erdos-Renyi graphs.  (A sample checks its endpoints' degrees itself,
    // so no isolated-vertex bitmap is built.)
    const Relabeled g = {rowptr, colidx, nullptr, nullptr};
    uint32_t *cnt = counts;
    if (counts && g.perm) {
        if ((st = scr.get(n, &cnt)) != NK_OK) return st;
        NK_HIP(launch_fill_u32(cnt, 0u, n, s));
    }
    // Records: one per vertex per slot, unless memory leaves fewer slots
    // than compute units (68 bytes per vertex per slot against half the
    // device memory) -- then each slot keeps a hash table of the vertices
    // its sample reaches (n / 16 entries rounded up to a power of two, in
    // [2^14, 2^18]; a sample lists a few thousand), and samples that could
    // fill more than half of it run afterwards with one record per vertex.
    // Hashing costs a probe per access: on a 4 * 10^6-vertex graph, where
    // 512 slots of records fit, 768 hashed slots were slower.  Tuning flag
    // bit 6 forces the tables, bit 5 forbids them.
    int32_t hlog = kPairHashMinLog2;
    while (hlog < kPairHashMaxLog2 && (1LL << hlog) < (long long)n / 16) ++hlog;
    const long long hcap = 1LL << hlog;
    const int32_t tflags = tuning_get().flags;
    LaunchPlan plan;
    if ((st = plan_launch(kModePair, n, count, 0, &plan)) != NK_OK && st != NK_E_NO_MEMORY) return st;
    DevInfo di;
    if (dev_info(&di) != NK_OK) return NK_E_HIP;
    const bool short_of_slots = st == NK_E_NO_MEMORY || (plan.grid < (long long)di.cus && plan.grid < count);
    clear_error();
    const bool hashed = !(tflags & 32) && (long long)n > 4 * hcap && ((tflags & 64) || short_of_slots);
    if (hashed && (st = plan_launch(kModePairHash, (int32_t)(hcap - 2), count, 0, &plan)) != NK_OK) return st;
    if (!hashed && st == NK_E_NO_MEMORY)
        return fail(NK_E_NO_MEMORY, "one pair-sampling slot with a record per vertex (n = %d) does not fit", n);
    Params p;
    memset(&p, 0, sizeof(p));
    p.rowptr = g.rowptr;
    p.colidx = g.colidx;
    p.n = n;
    p.m = (int32_t)m;
    p.ntasks = count;
    p.seed = seed;
    p.j0 = j0;
    p.counts = cnt;
    p.p_uv = uv;
    p.p_len = len;
    p.p_path = path;
    p.maxlen = maxlen;
    p.perm = g.perm;
    p.inv = g.inv;
    p.st = dst;
    unsigned long long *dcount = nullptr;
    if (hashed) {
        p.ph_log2 = hlog;
        if ((st = scr.get(count, &p.defer)) != NK_OK) return st;
        if ((st = scr.get(1, &dcount)) != NK_OK) return st;
        NK_HIP(launch_fill_u64(dcount, 0ULL, 1, s));
        p.defer_count = dcount;
    }
    if ((st = launch_persistent(plan, p, scr, s, ev0, hashed ? nullptr : ev1)) != NK_OK) return st;
    plan.pair_rec = p.pair_blk;
    if (hashed) {
        unsigned long long nd = 0;
        NK_HIP(hipMemcpyAsync(&nd, dcount, sizeof(nd), hipMemcpyDeviceToHost, s));
        NK_HIP(hipStreamSynchronize(s));
        if (nd > 0) {
            // the deferred samples, one record per vertex, outputs by sample
            LaunchPlan full;
            if ((st = plan_launch(kModePair, n, (long long)nd, 0, &full)) != NK_OK) return st;
            Params q = p;
            q.ntasks = (long long)nd;
            q.task_list = p.defer;
            q.defer = nullptr;
            q.defer_count = nullptr;
            NK_HIP(launch_reset_head(dst, s));
            if ((st = launch_persistent(full, q, scr, s, nullptr, nullptr)) != NK_OK) return st;
            // (its records end all-unreached too, but stay untagged)
        }
        if (ev1) NK_HIP(hipEventRecord(ev1, s));
    }
    if (counts && g.perm) NK_HIP(launch_gather_u32(cnt, g.perm, n, counts, s));
    *plan_out = plan;
    return NK_OK;
}

nk_status nk_pair_counts(const int32_t *rowptr, const int32_t *colidx, int32_t n, int64_t m, int64_t r,
                         uint64_t seed, uint32_t *counts, void *stream) {
    clear_error();
    stats_clear();
    nk_status st = check_graph_args(rowptr, colidx, n, m);
    if (st != NK_OK) return st;
    if (n == 0) return NK_OK;
    if (!counts || r < 0) return fail(NK_E_INVALID_ARG, "counts is NULL or r < 0");
    hipStream_t s = (hipStream_t)stream;
    Scratch scr;
    DevStatus *dst;
    if ((st = scr.get(1, &dst)) != NK_OK) return st;
    DevStatus *h = host_status();
    if (!h) return fail(NK_E_NO_MEMORY, "pinned status buffer");
    NK_HIP(launch_status_init(dst, s));
    NK_HIP(launch_validate(rowptr, colidx, n, m, 0, dst, s));
    NK_HIP(launch_fill_u32(counts, 0u, n, s));
    LaunchPlan plan = {};
    float ms = 0.0f;
    if (n >= 2 && r > 0) {
        hipEvent_t ev0, ev1;
        if ((st = thread_events(&ev0, &ev1)) != NK_OK) return st;
        if ((st = pair_run(rowptr, colidx, n, m, r, seed, 0, counts, nullptr, nullptr, nullptr, 0, dst, scr, s, &plan,
                           ev0, ev1)) != NK_OK)
            return st;
        st = finish(dst, h, s);
        if (st == NK_OK && plan.pair_rec) scr.mark(plan.pair_rec, pair_block_tag(plan));
        NK_HIP(hipEventElapsedTime(&ms, ev0, ev1));
    } else {
        st = finish(dst, h, s);
    }
    stats_record(*h, plan.grid, plan.block, plan.lds, ms);
    return st;
}

nk_status nk_bc_pair_sample(const int32_t *rowptr, const int32_t *colidx, int32_t n, int64_t m, double eps,
                            double delta, uint64_t seed, double *bc, uint32_t *counts, int64_t *r_out,
                            int32_t *vd_out, void *stream) {
    clear_error();
    stats_clear();
    nk_status st = check_graph_args(rowptr, colidx, n, m);
    if (st != NK_OK) return st;
    if (!(eps > 0.0 && eps < 1.0) || !(delta > 0.0 && delta < 1.0))
        return fail(NK_E_INVALID_ARG, "eps and delta must lie in (0, 1)");
    if (n == 0) {
        if (r_out) *r_out = 0;
        if (vd_out) *vd_out = 0;
        return NK_OK;
    }
    if (!bc) return fail(NK_E_INVALID_ARG, "bc is NULL");
    hipStream_t s = (hipStream_t)stream;
    int32_t info[8];
    // the sample size needs the upper bound only
    if ((st = vd_bound_impl(rowptr, colidx, n, m, info, s, false)) != NK_OK) return st;
    const long long r = n >= 2 ? nk_rk_sample_size(eps, delta, info[4]) : 0;
    if (r_out) *r_out = r;
    if (vd_out) *vd_out = info[4];
    Scratch scr;
    DevStatus *dst;
    if ((st = scr.get(1, &dst)) != NK_OK) return st;
    uint32_t *cnt = counts;
    if (!cnt && (st = scr.get(n, &cnt)) != NK_OK) return st;
    DevStatus *h = host_status();
    if (!h) return fail(NK_E_NO_MEMORY, "pinned status buffer");
    NK_HIP(launch_status_init(dst, s));
    NK_HIP(launch_fill_u32(cnt, 0u, n, s));
    LaunchPlan plan = {};
    float ms = 0.0f;
    hipEvent_t ev0 = nullptr, ev1 = nullptr;
    if (r > 0) {
        if ((st = thread_events(&ev0, &ev1)) != NK_OK) return st;
        if ((st = pair_run(rowptr, colidx, n, m, r, seed, 0, cnt, nullptr, nullptr, nullptr, 0, dst, scr, s, &plan,
                           ev0, ev1)) != NK_OK)
            return st;
    }
    const double scale = r > 0 ? (double)n * (double)(n - 1) / (double)r : 0.0;
    NK_HIP(launch_counts_to_bc(cnt, bc, scale, n, s));
    st = finish(dst, h, s);
    if (st == NK_OK && plan.pair_rec) scr.mark(plan.pair_rec, pair_block_tag(plan));
    if (r > 0) NK_HIP(hipEventElapsedTime(&ms, ev0, ev1));
    stats_record(*h, plan.grid, plan.block, plan.lds, ms);
    return st;
}

nk_status nk_sample_paths(const int32_t *rowptr, const int32_t *colidx, int32_t n, int64_t m, uint64_t seed,
                          int64_t j0, int32_t count, int32_t maxlen, int32_t *uv, int32_t *len, int32_t *path,
                          void *stream) {
    clear_error();
    stats_clear();
    nk_status st = check_graph_args(rowptr, colidx, n, m);
    if (st != NK_OK) return st;
    if (n < 2) return fail(NK_E_INVALID_ARG, "pair sampling needs n >= 2");
    if (count < 0 || j0 < 0 || maxlen < 0 || (count > 0 && (!uv || !len || (maxlen > 0 && !path))))
        return fail(NK_E_INVALID_ARG, "bad sample range or outputs");
    if (count == 0) return NK_OK;
    hipStream_t s = (hipStream_t)stream;
    Scratch scr;
    DevStatus *dst;
    if ((st = scr.get(1, &dst)) != NK_OK) return st;
    DevStatus *h = host_status();
    if (!h) return fail(NK_E_NO_MEMORY, "pinned status buffer");
    NK_HIP(launch_status_init(dst, s));
    NK_HIP(launch_validate(rowptr, colidx, n, m, 0, dst, s));
    LaunchPlan plan;
    if ((st = pair_run(rowptr, colidx, n, m, count, seed, j0, nullptr, uv, len, maxlen > 0 ? path : nullptr, maxlen,
                       dst, scr, s, &plan, nullptr, nullptr)) != NK_OK)
        return st;
    st = finish(dst, h, s);
    if (st == NK_OK && plan.pair_rec) scr.mark(plan.pair_rec, pair_block_tag(plan));
    stats_record(*h, plan.grid, plan.block, plan.lds, 0.0f);
    return st;
}

}  // extern "C"

namespace nk {

// Everything a batched exact run launches, planned on the host.
struct BatchSetup {
    DevStatus *dst = nullptr;
    Params p;
    LaunchPlan plan_s = {}, plan_l = {};
    int ms_b = 1;              // sources per task of the large graphs' launch
    MsPlan mplan = {};
    GroupPlan gplan = {};      // the group kernel's launch
    Params pg;                 // its parameters (own scratch)
    long long *t_small = nullptr, *t_large = nullptr, *t_group = nullptr;
    int32_t *o_small = nullptr, *o_large = nullptr, *o_group = nullptr;
    long long k_small = 0, k_large = 0, k_group = 0;
    int32_t g_small = 0, g_large = 0, n_large = 0, g_group = 0, n_group = 0;
    long long *d_vtx = nullptr, *d_arc = nullptr;
    int32_t G = 0;
    long long nv = 0;
    const int32_t *rowptr = nullptr, *colidx = nullptr;
    double *bc = nullptr;
};

// Argument checks, offset and schedule uploads (synchronous), kernel plans
// and all scratch.  nv = 0 means nothing to do.
static nk_status batch_prepare(int32_t G, const int64_t *vtx_off, const int64_t *arc_off, const int32_t *rowptr_cat,
                               const int32_t *colidx_cat, double *bc_cat, Scratch &scr, hipStream_t s,
                               BatchSetup *b) {
    if (G < 0) return fail(NK_E_INVALID_ARG, "G is negative");
    b->G = G;
    b->nv = 0;
    if (G == 0) return NK_OK;
    if (!vtx_off || !arc_off) return fail(NK_E_INVALID_ARG, "offset tables are NULL");
    if (vtx_off[0] != 0 || arc_off[0] != 0) return fail(NK_E_INVALID_ARG, "offsets must start at 0");
    std::vector<long long> work(G);
    for (int32_t g = 0; g < G; ++g) {
        const long long ng = vtx_off[g + 1] - vtx_off[g], mg = arc_off[g + 1] - arc_off[g];
        if (ng < 0 || mg < 0 || ng > 2147483647LL || mg > 2147483647LL)
            return fail(NK_E_INVALID_ARG, "graph %d has bad offsets", g);
        work[g] = ng * std::max<long long>(mg, 1);
    }
    const long long nv = vtx_off[G], na = arc_off[G];
    if (nv == 0) return NK_OK;
    if (!rowptr_cat || (na > 0 && !colidx_cat) || !bc_cat) return fail(NK_E_INVALID_ARG, "NULL graph or output");
    nk_status st;
    if ((st = scr.get(1, &b->dst)) != NK_OK) return st;
    if ((st = scr.get(G + 1, &b->d_vtx)) != NK_OK) return st;
    if ((st = scr.get(G + 1, &b->d_arc)) != NK_OK) return st;
    NK_HIP(hipMemcpyAsync(b->d_vtx, vtx_off, sizeof(long long) * (G + 1), hipMemcpyHostToDevice, s));
    NK_HIP(hipMemcpyAsync(b->d_arc, arc_off, sizeof(long long) * (G + 1), hipMemcpyHostToDevice, s));

    // Graphs whose CSR and per-source state fit one workgroup's LDS run on
    // the all-in-LDS kernel, the others on the global-memory kernel.  Each
    // part takes its largest graphs first, so launch tails are made of
    // small tasks.
    size_t dyn_max = 0;
    LaunchPlan probe;
    const bool lds_ok = plan_lds(0, 1 << 20, 1, &probe);
    size_t budget = 0;
    if (lds_ok) {
        hipFuncAttributes attr;
        NK_HIP(hipFuncGetAttributes(&attr, probe.kernel.fn));
        DevInfo di;
        if ((st = dev_info(&di)) != NK_OK) return st;
        budget = di.lds_per_block > attr.sharedSizeBytes ? di.lds_per_block - attr.sharedSizeBytes : 0;
    }
    // Graphs the group kernel takes (by size, or all large ones under flag
    // bit 3) form a third part with a launch of its own.
    std::vector<int32_t> small, large, grp;
    int32_t n_small = 0;
    for (int32_t g = 0; g < G; ++g) {
        const long long ng = vtx_off[g + 1] - vtx_off[g], mg = arc_off[g + 1] - arc_off[g];
        if (ng == 0) continue;
        const size_t by = lds_graph_bytes((int32_t)ng, mg);
        if (lds_ok && by <= budget) {
            small.push_back(g);
            dyn_max = std::max(dyn_max, by);
            n_small = std::max<int32_t>(n_small, (int32_t)ng);
        } else if (group_wanted((int32_t)ng, mg)) {
            grp.push_back(g);
            b->n_group = std::max<int32_t>(b->n_group, (int32_t)ng);
        } else {
            large.push_back(g);
            b->n_large = std::max<int32_t>(b->n_large, (int32_t)ng);
        }
    }
    auto by_work = [&](int32_t x, int32_t y) { return work[x] > work[y]; };
    std::stable_sort(small.begin(), small.end(), by_work);
    std::stable_sort(large.begin(), large.end(), by_work);
    std::stable_sort(grp.begin(), grp.end(), by_work);
    // task prefix over the graphs in processing order: one task per source,
    // or per group of `per` sources
    auto tables = [&](const std::vector<int32_t> &ids, long long **d_task, int32_t **d_order, long long *ntasks,
                      int per) -> nk_status {
        const int32_t K = (int32_t)ids.size();
        std::vector<long long> pre(K + 1, 0);
        for (int32_t i = 0; i < K; ++i) pre[i + 1] = pre[i] + (vtx_off[ids[i] + 1] - vtx_off[ids[i]] + per - 1) / per;
        nk_status e;
        if ((e = scr.get(K + 1, d_task)) != NK_OK) return e;
        if ((e = scr.get(K, d_order)) != NK_OK) return e;
        NK_HIP(hipMemcpyAsync(*d_task, pre.data(), sizeof(long long) * (K + 1), hipMemcpyHostToDevice, s));
        NK_HIP(hipMemcpyAsync(*d_order, ids.data(), sizeof(int32_t) * K, hipMemcpyHostToDevice, s));
        // the host vectors must outlive the copies
        NK_HIP(hipStreamSynchronize(s));
        *ntasks = pre[K];
        return NK_OK;
    };
    memset(&b->p, 0, sizeof(b->p));
    b->p.rowptr = rowptr_cat;
    b->p.colidx = colidx_cat;
    b->p.g_vtx = b->d_vtx;
    b->p.g_arc = b->d_arc;
    b->p.bc = bc_cat;
    b->p.st = b->dst;
    b->g_small = (int32_t)small.size();
    b->g_large = (int32_t)large.size();
    b->g_group = (int32_t)grp.size();
    if (!small.empty()) {
        if ((st = tables(small, &b->t_small, &b->o_small, &b->k_small, 1)) != NK_OK) return st;
        if (!plan_lds(dyn_max, n_small, b->k_small, &b->plan_s)) return fail(NK_E_INTERNAL, "all-in-LDS plan failed");
    }
    // the large graphs' launch runs under the registered autotuner cache's
    // tuning for the largest of them, if it has one
    nk_tuning cached;
    bool use_cached = false;
    if (!large.empty() && tuning_cache_active()) {
        int32_t gbig = large[0];
        for (int32_t g : large)
            if (vtx_off[g + 1] - vtx_off[g] > vtx_off[gbig + 1] - vtx_off[gbig]) gbig = g;
        int64_t dmax = 0;
        const int32_t nb = (int32_t)(vtx_off[gbig + 1] - vtx_off[gbig]);
        if ((st = graph_max_degree(rowptr_cat + vtx_off[gbig] + gbig, nb, s, &dmax)) != NK_OK) return st;
        use_cached = cached_tuning(nb, arc_off[gbig + 1] - arc_off[gbig], dmax, &cached);
    }
    TuningOverride cached_scope(use_cached ? &cached : nullptr);
    if (!large.empty()) {
        long long nsrc_large = 0;
        for (int32_t g : large) nsrc_large += vtx_off[g + 1] - vtx_off[g];
        b->ms_b = ms_batch_for(b->n_large, nsrc_large);
        if ((st = tables(large, &b->t_large, &b->o_large, &b->k_large, b->ms_b)) != NK_OK) return st;
        if (b->ms_b > 1) {
            if ((st = plan_ms(b->ms_b, b->n_large, nsrc_large, &b->mplan)) != NK_OK) return st;
            b->mplan.ntasks = b->k_large;
            if ((st = ms_alloc(b->mplan, b->p, scr)) != NK_OK) return st;
            b->plan_l = b->mplan.lp;
        } else {
            if ((st = plan_launch(kModeBC, b->n_large, b->k_large, 0, &b->plan_l)) != NK_OK) return st;
            if ((st = persistent_alloc(b->plan_l, b->p, scr, s)) != NK_OK) return st;
        }
    }
    if (!grp.empty()) {
        if ((st = tables(grp, &b->t_group, &b->o_group, &b->k_group, 1)) != NK_OK) return st;
        if ((st = plan_group(b->n_group, &b->gplan)) != NK_OK) return st;
        // the group launch has its own scratch; the one-source launch's
        // pointers in b->p stay as they are
        Params gp_params = b->p;
        if ((st = group_alloc(b->gplan, gp_params, scr)) != NK_OK) return st;
        b->pg = gp_params;
    }
    b->nv = nv;
    b->rowptr = rowptr_cat;
    b->colidx = colidx_cat;
    b->bc = bc_cat;
    return NK_OK;
}

// The run itself: kernels only (status reset, batch validation, output
// clear, the all-in-LDS launch, the global-memory launch), so it can be
// captured into a HIP graph.
static nk_status batch_enqueue(const BatchSetup &b, hipStream_t s, hipEvent_t ev0, hipEvent_t ev1) {
    NK_HIP(launch_status_init(b.dst, s));
    NK_HIP(launch_validate_batched(b.rowptr, b.colidx, b.d_vtx, b.d_arc, b.G, b.dst, s));
    NK_HIP(launch_fill_f64(b.bc, 0.0, b.nv, s));
    if (ev0) NK_HIP(hipEventRecord(ev0, s));
    Params p = b.p;
    if (b.g_small > 0) {
        p.n = 0;
        p.G = b.g_small;
        p.g_task = b.t_small;
        p.g_order = b.o_small;
        p.ntasks = b.k_small;
        b.plan_s.kernel.launch(dim3(b.plan_s.grid), dim3(b.plan_s.block), b.plan_s.dyn_lds, s, p);
        NK_HIP(hipGetLastError());
    }
    if (b.g_large > 0) {
        if (b.g_small > 0) NK_HIP(launch_reset_head(b.dst, s));
        p.n = b.n_large;
        p.G = b.g_large;
        p.g_task = b.t_large;
        p.g_order = b.o_large;
        p.ntasks = b.k_large;
        nk_status st = b.ms_b > 1 ? ms_enqueue(b.mplan, p, s, nullptr, nullptr)
                                  : persistent_enqueue(b.plan_l, p, s, nullptr, nullptr);
        if (st != NK_OK) return st;
    }
    if (b.g_group > 0) {
        if (b.g_small > 0 || b.g_large > 0) NK_HIP(launch_reset_head(b.dst, s));
        Params q = b.pg;
        q.n = b.n_group;
        q.G = b.g_group;
        q.g_task = b.t_group;
        q.g_order = b.o_group;
        q.ntasks = b.k_group;
        nk_status st = group_enqueue(b.gplan, q, s, nullptr, nullptr);
        if (st != NK_OK) return st;
    }
    if (ev1) NK_HIP(hipEventRecord(ev1, s));
    return NK_OK;
}

static void batch_stats(const BatchSetup &b, const DevStatus &h, float ms) {
    int where = b.g_large == 0 ? 2 : (b.g_small == 0 ? (b.plan_l.lds ? 1 : 0) : 3);
    if (b.g_large > 0 && b.ms_b > 1) where = b.g_small == 0 ? 4 : 5;
    if (b.g_group > 0) where = (b.g_small == 0 && b.g_large == 0) ? 6 : 7;
    const LaunchPlan &shown = b.g_large > 0 ? b.plan_l : (b.g_group > 0 ? b.gplan.lp : b.plan_s);
    stats_record(h, shown.grid, shown.block, where, ms);
    if (b.g_large > 0) stats_set_batch(b.ms_b);
}

}  // namespace nk

// A captured batched run (see include/nk_bc.h).
struct nk_batch_plan {
    int device = 0;
    nk::Scratch *scr = nullptr;
    nk::BatchSetup b;
    hipStream_t cs = nullptr;
    hipGraph_t graph = nullptr;
    hipGraphExec_t exec = nullptr;
    hipEvent_t ev0 = nullptr, ev1 = nullptr;   // around the last launch
    unsigned long long *done_h = nullptr;      // pinned: progress counter read back
    bool running = false;
};

extern "C" {

nk_status nk_bc_exact_batched(int32_t G, const int64_t *vtx_off, const int64_t *arc_off, const int32_t *rowptr_cat,
                              const int32_t *colidx_cat, double *bc_cat, void *stream) {
    clear_error();
    stats_clear();
    hipStream_t s = (hipStream_t)stream;
    Scratch scr;
    BatchSetup b;
    nk_status st = batch_prepare(G, vtx_off, arc_off, rowptr_cat, colidx_cat, bc_cat, scr, s, &b);
    if (st != NK_OK || b.nv == 0) return st;
    DevStatus *h = host_status();
    if (!h) return fail(NK_E_NO_MEMORY, "pinned status buffer");
    hipEvent_t ev0, ev1;
    if ((st = thread_events(&ev0, &ev1)) != NK_OK) return st;
    if ((st = batch_enqueue(b, s, ev0, ev1)) != NK_OK) return st;
    st = finish(b.dst, h, s);
    float ms = 0.0f;
    NK_HIP(hipEventElapsedTime(&ms, ev0, ev1));
    batch_stats(b, *h, ms);
    return st;
}

nk_status nk_batch_plan_create(int32_t G, const int64_t *vtx_off, const int64_t *arc_off, const int32_t *rowptr_cat,
                               const int32_t *colidx_cat, double *bc_cat, nk_batch_plan **out) {
    clear_error();
    if (!out) return fail(NK_E_INVALID_ARG, "out is NULL");
    *out = nullptr;
    nk_batch_plan *pl = new nk_batch_plan();
    pl->scr = new Scratch();
    auto bail = [&](nk_status code) {
        nk_batch_plan_destroy(pl);
        return code;
    };
    if (hipGetDevice(&pl->device) != hipSuccess) return bail(fail(NK_E_HIP, "hipGetDevice failed"));
    // a stream of the library's own (default priority): capture cannot run
    // on the legacy default stream
    if (hipStreamCreateWithFlags(&pl->cs, hipStreamNonBlocking) != hipSuccess)
        return bail(fail(NK_E_HIP, "stream creation failed"));
    nk_status st = batch_prepare(G, vtx_off, arc_off, rowptr_cat, colidx_cat, bc_cat, *pl->scr, pl->cs, &pl->b);
    if (st != NK_OK) return bail(st);
    if (hipStreamSynchronize(pl->cs) != hipSuccess) return bail(fail(NK_E_HIP, "stream synchronisation failed"));
    if (pl->b.nv > 0) {
        if (hipStreamBeginCapture(pl->cs, hipStreamCaptureModeThreadLocal) != hipSuccess)
            return bail(fail(NK_E_HIP, "stream capture did not start"));
        st = batch_enqueue(pl->b, pl->cs, nullptr, nullptr);
        hipGraph_t g = nullptr;
        const hipError_t e = hipStreamEndCapture(pl->cs, &g);
        pl->graph = g;
        if (st != NK_OK) return bail(st);
        if (e != hipSuccess || !g) return bail(fail(NK_E_HIP, "stream capture failed"));
        if (hipGraphInstantiate(&pl->exec, pl->graph, nullptr, nullptr, 0) != hipSuccess)
            return bail(fail(NK_E_HIP, "graph instantiation failed"));
    }
    if (hipEventCreate(&pl->ev0) != hipSuccess || hipEventCreate(&pl->ev1) != hipSuccess)
        return bail(fail(NK_E_HIP, "event creation failed"));
    if (hipHostMalloc((void **)&pl->done_h, sizeof(unsigned long long), hipHostMallocDefault) != hipSuccess) {
        pl->done_h = nullptr;
        return bail(fail(NK_E_NO_MEMORY, "pinned progress buffer"));
    }
    *out = pl;
    return NK_OK;
}

static nk_status plan_check(nk_batch_plan *plan) {
    if (!plan) return fail(NK_E_INVALID_ARG, "plan is NULL");
    int dev = 0;
    NK_HIP(hipGetDevice(&dev));
    if (dev != plan->device) return fail(NK_E_INVALID_ARG, "plan was made on device %d, current is %d", plan->device, dev);
    return NK_OK;
}

nk_status nk_batch_plan_launch(nk_batch_plan *plan, void *stream) {
    clear_error();
    nk_status st = plan_check(plan);
    if (st != NK_OK) return st;
    if (plan->running) return fail(NK_E_INVALID_ARG, "the plan's previous run has not been finished");
    if (plan->b.nv == 0) return NK_OK;
    hipStream_t s = (hipStream_t)stream;
    NK_HIP(hipEventRecord(plan->ev0, s));
    NK_HIP(hipGraphLaunch(plan->exec, s));
    NK_HIP(hipEventRecord(plan->ev1, s));
    plan->running = true;
    return NK_OK;
}

nk_status nk_batch_plan_progress(nk_batch_plan *plan, int64_t *done, int64_t *total, int32_t *finished) {
    clear_error();
    nk_status st = plan_check(plan);
    if (st != NK_OK) return st;
    if (!done || !total || !finished) return fail(NK_E_INVALID_ARG, "NULL output");
    *total = plan->b.nv;
    if (!plan->running || plan->b.nv == 0) {
        *done = plan->running ? 0 : plan->b.nv;
        *finished = 1;
        return NK_OK;
    }
    // the counter is read on the plan's own (non-blocking) stream while the
    // run goes on on the caller's
    NK_HIP(hipMemcpyAsync(plan->done_h, &plan->b.dst->stat[kStDone], sizeof(unsigned long long),
                          hipMemcpyDeviceToHost, plan->cs));
    NK_HIP(hipStreamSynchronize(plan->cs));
    const hipError_t q = hipEventQuery(plan->ev1);
    if (q != hipSuccess && q != hipErrorNotReady) return fail(NK_E_HIP, "hipEventQuery failed: %s", hipGetErrorString(q));
    *finished = q == hipSuccess;
    *done = (int64_t)*plan->done_h;
    return NK_OK;
}

nk_status nk_batch_plan_finish(nk_batch_plan *plan, void *stream) {
    clear_error();
    stats_clear();
    nk_status st = plan_check(plan);
    if (st != NK_OK) return st;
    if (plan->b.nv == 0) return NK_OK;
    if (!plan->running) return fail(NK_E_INVALID_ARG, "the plan has no run to finish");
    plan->running = false;
    hipStream_t s = (hipStream_t)stream;
    DevStatus *h = host_status();
    if (!h) return fail(NK_E_NO_MEMORY, "pinned status buffer");
    st = finish(plan->b.dst, h, s);
    float ms = 0.0f;
    NK_HIP(hipEventElapsedTime(&ms, plan->ev0, plan->ev1));
    batch_stats(plan->b, *h, ms);
    return st;
}

nk_status nk_batch_plan_run(nk_batch_plan *plan, void *stream) {
    nk_status st = nk_batch_plan_launch(plan, stream);
    if (st != NK_OK) return st;
    return nk_batch_plan_finish(plan, stream);
}

void nk_batch_plan_destroy(nk_batch_plan *plan) {
    if (!plan) return;
    if (plan->cs) (void)hipStreamSynchronize(plan->cs);
    if (plan->exec) (void)hipGraphExecDestroy(plan->exec);
    if (plan->graph) (void)hipGraphDestroy(plan->graph);
    if (plan->running && plan->ev1) (void)hipEventSynchronize(plan->ev1);
    if (plan->cs) (void)hipStreamDestroy(plan->cs);
    if (plan->ev0) (void)hipEventDestroy(plan->ev0);
    if (plan->ev1) (void)hipEventDestroy(plan->ev1);
    if (plan->done_h) (void)hipHostFree(plan->done_h);
    delete plan->scr;
    delete plan;
}

}  // extern "C"
