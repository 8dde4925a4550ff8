// Serving loop: betweenness queries on a resident pool of graphs.
//
// A server owns device copies of its graphs (relabelled by degree once, with
// their isolated-vertex bitmaps and vertex-diameter bounds) and a small
// number of execution slots, each with its own HIP stream.  A scheduler
// thread admits queued requests in arrival order whenever a slot is free and
// the request's device footprint fits the HBM budget left over by the pool
// and the requests already running, enqueues the whole request on the slot's
// stream (source upload, the persistent Brandes kernel restricted to a share
// of the compute units, scaling, copy of the scores to pinned host memory)
// and polls completion events.  Requests that arrive while others run are
// admitted as soon as a slot and memory free up, so their kernels overlap on
// the device.  Latency runs from submit to scores in host memory.
#include <string.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <deque>
#include <map>
#include <mutex>
#include <thread>
#include <vector>

#include "nk_runtime.h"

namespace nk {

static double now_s() {
    using namespace std::chrono;
    return duration<double>(steady_clock::now().time_since_epoch()).count();
}

struct ServerGraph {
    int32_t n = 0;
    int64_t m = 0;
    int32_t *rowptr = nullptr;   // relabelled CSR (device, server-owned)
    int32_t *colidx = nullptr;
    int32_t *perm = nullptr;     // original -> internal
    int32_t *inv = nullptr;
    uint32_t *iso = nullptr;
    int32_t vd = 0;              // vertex-diameter bound of the original graph
    size_t bytes = 0;
    bool tuned = false;          // an autotuner cache entry matched the graph's shape
    nk_tuning tuning = {};
};

struct Request {
    int64_t ticket = 0;
    int32_t graph = 0;
    // the pooled graph, taken under the server lock at submission; graphs
    // live in a deque, so adding graphs later never moves it
    const ServerGraph *g = nullptr;
    std::vector<int32_t> sources;  // original ids (k-requests)
    double eps = 0.0, delta = 0.0;
    uint64_t seed = 0;
    double *out = nullptr;         // caller's host buffer, n doubles
    long long work = 0;            // sources or samples
    size_t footprint = 0;
    int grid = 1;                  // workgroups of its kernel (set at submission, widened at admission)
    long long tasks = 0;           // sources or samples
    double t_submit = 0, t_start = 0, t_done = 0;
    nk_status status = NK_OK;
    bool done = false;
};

struct Slot {
    hipStream_t stream = nullptr;
    hipEvent_t ev = nullptr;
    Request *req = nullptr;
    DevStatus *dst = nullptr;   // device
    DevStatus *hst = nullptr;   // pinned host
    double *staging = nullptr;  // pinned host, n_max doubles
    size_t staging_n = 0;
    Scratch *scr = nullptr;
    LaunchPlan plan = {};
};

}  // namespace nk

struct nk_server {
    int device = 0;
    size_t budget = 0;
    size_t pool_bytes = 0;       // resident graphs
    size_t running_bytes = 0;    // admitted requests
    int n_share = 1;             // a request's kernel takes 1/n_share of the resident-workgroup capacity
    std::deque<nk::ServerGraph> graphs;   // stable element addresses: requests hold pointers
    std::vector<nk::Slot> slots;
    std::deque<nk::Request *> pending;
    std::map<int64_t, nk::Request *> requests;
    int64_t next_ticket = 1;
    std::mutex mu;
    std::condition_variable cv_work, cv_done;
    std::thread worker;
    bool stop = false;
    // statistics
    std::vector<double> latency;
    double first_submit = 0, last_done = 0;
    long long completed = 0, failed = 0;
    double edge_work = 0;        // sum over completed requests of work x undirected edges
    int max_inflight = 0;
};

namespace nk {

static size_t round256(size_t b) { return (b + 255) & ~(size_t)255; }

// Device bytes a request needs while running (per-slot kernel scratch plus
// its vectors), mirroring what Scratch::get requests.
static size_t request_footprint(const ServerGraph &g, long long k, int grid, bool pair) {
    const long long stride = (((long long)g.n + 2) + 63) / 64 * 64;
    const long long cells = (long long)grid * stride;
    size_t b = 0;
    b += round256(cells * 8);           // weights / push accumulator
    b += round256(cells * 4) * 4;       // lv, la, ld, cand
    b += round256((size_t)g.n * 8);     // accumulator / counts
    b += round256((size_t)std::max<long long>(k, 1) * 4) * 2;
    b += round256(sizeof(DevStatus));
    if (pair) {
        b += round256(cells * 32);          // records of both search sides
        b += round256(cells * 4) * 3;       // the target side's lists
    } else {
        b += round256(cells * 8);           // sigma
        b += round256(cells * 4) * 4;       // ldeg, d, lvl, candidates' spare
        b += round256((size_t)((g.n + 31) / 32) * 4);   // isolated-vertex bitmap
    }
    return b;
}

static void start_request(nk_server *sv, Slot &sl, Request *rq) {
    (void)sv;
    const ServerGraph &g = *rq->g;
    hipStream_t s = sl.stream;
    sl.req = rq;
    sl.scr = new Scratch();
    Scratch &scr = *sl.scr;
    rq->t_start = now_s();
    nk_status st = NK_OK;
    auto bail = [&](nk_status code) {
        rq->status = code;
        (void)hipEventRecord(sl.ev, s);
    };
    const int32_t n = g.n;
    if (sl.staging_n < (size_t)n) {
        if (sl.staging) (void)hipHostFree(sl.staging);
        sl.staging = nullptr;
        sl.staging_n = 0;
        void *h = nullptr;
        if (hipHostMalloc(&h, sizeof(double) * (size_t)n, hipHostMallocDefault) != hipSuccess) {
            (void)hipGetLastError();
            return bail(NK_E_NO_MEMORY);
        }
        sl.staging = (double *)h;
        sl.staging_n = (size_t)n;
    }
    if (launch_status_init(sl.dst, s) != hipSuccess) return bail(NK_E_HIP);
    const bool pair = rq->sources.empty();
    if (!pair) {
        // source requests run under the graph's cached tuning, if any
        TuningOverride tuned(g.tuned ? &g.tuning : nullptr);
        const long long k = (long long)rq->sources.size();
        int32_t *src_host_dev, *src_int;
        double *acc, *outd;
        if ((st = scr.get(k, &src_host_dev)) != NK_OK) return bail(st);
        if ((st = scr.get(k, &src_int)) != NK_OK) return bail(st);
        if ((st = scr.get(n, &acc)) != NK_OK) return bail(st);
        outd = acc;
        if (hipMemcpyAsync(src_host_dev, rq->sources.data(), sizeof(int32_t) * k, hipMemcpyHostToDevice, s) !=
            hipSuccess)
            return bail(NK_E_HIP);
        (void)launch_map_sources(src_host_dev, (int32_t)k, g.perm, n, src_int, s);
        (void)launch_fill_f64(acc, 0.0, n, s);
        if ((st = plan_launch(kModeBC, n, k, rq->grid, &sl.plan)) != NK_OK) return bail(st);
        Params p;
        memset(&p, 0, sizeof(p));
        p.rowptr = g.rowptr;
        p.colidx = g.colidx;
        p.n = n;
        p.m = (int32_t)g.m;
        p.ntasks = k;
        p.sources = src_int;
        p.bc = acc;
        p.iso = g.iso;
        p.st = sl.dst;
        if ((st = launch_persistent(sl.plan, p, scr, s, nullptr, nullptr)) != NK_OK) return bail(st);
        // scores in original ids, scaled by n / k, into a device buffer
        double *res;
        if ((st = scr.get(n, &res)) != NK_OK) return bail(st);
        (void)launch_gather_scale(acc, g.perm, n, (double)n / (double)k, res, s);
        outd = res;
        (void)hipMemcpyAsync(sl.staging, outd, sizeof(double) * n, hipMemcpyDeviceToHost, s);
    } else {
        const long long r = n >= 2 ? nk_rk_sample_size(rq->eps, rq->delta, g.vd) : 0;
        rq->work = r;
        uint32_t *cnt, *cnt_orig;
        double *res;
        if ((st = scr.get(n, &cnt)) != NK_OK) return bail(st);
        if ((st = scr.get(n, &cnt_orig)) != NK_OK) return bail(st);
        if ((st = scr.get(n, &res)) != NK_OK) return bail(st);
        (void)launch_fill_u32(cnt, 0u, n, s);
        if (r > 0) {
            if ((st = plan_launch(kModePair, n, r, rq->grid, &sl.plan)) != NK_OK) return bail(st);
            Params p;
            memset(&p, 0, sizeof(p));
            p.rowptr = g.rowptr;
            p.colidx = g.colidx;
            p.n = n;
            p.m = (int32_t)g.m;
            p.ntasks = r;
            p.seed = rq->seed;
            p.counts = cnt;
            p.perm = g.perm;
            p.inv = g.inv;
            p.iso = g.iso;
            p.st = sl.dst;
            if ((st = launch_persistent(sl.plan, p, scr, s, nullptr, nullptr)) != NK_OK) return bail(st);
            sl.plan.pair_rec = p.pair_blk;
        }
        (void)launch_gather_u32(cnt, g.perm, n, cnt_orig, s);
        const double scale = r > 0 ? (double)n * (double)(n - 1) / (double)r : 0.0;
        (void)launch_counts_to_bc(cnt_orig, res, scale, n, s);
        (void)hipMemcpyAsync(sl.staging, res, sizeof(double) * n, hipMemcpyDeviceToHost, s);
    }
    (void)hipMemcpyAsync(sl.hst, sl.dst, sizeof(DevStatus), hipMemcpyDeviceToHost, s);
    if (hipEventRecord(sl.ev, s) != hipSuccess) rq->status = NK_E_HIP;
}

static void finish_request(nk_server *sv, Slot &sl) {
    Request *rq = sl.req;
    const ServerGraph &g = *rq->g;
    if (rq->status == NK_OK) {
        const int32_t err = sl.hst->err;
        if (err & kErrGraph) rq->status = NK_E_INVALID_GRAPH;
        else if (err & kErrArg) rq->status = NK_E_INVALID_ARG;
        else if (err & kErrOverflow) rq->status = NK_E_SIGMA_OVERFLOW;
        else if (err & kErrInternal) rq->status = NK_E_INTERNAL;
    }
    if (rq->status == NK_OK && rq->out) memcpy(rq->out, sl.staging, sizeof(double) * g.n);
    // a successful pair launch leaves its records all unreached
    if (rq->status == NK_OK && sl.plan.pair_rec) sl.scr->mark(sl.plan.pair_rec, pair_block_tag(sl.plan));
    sl.plan.pair_rec = nullptr;
    rq->t_done = now_s();
    delete sl.scr;
    sl.scr = nullptr;
    sl.req = nullptr;
    std::lock_guard<std::mutex> lk(sv->mu);
    sv->running_bytes -= rq->footprint;
    rq->done = true;
    if (rq->status == NK_OK) {
        sv->completed++;
        sv->latency.push_back(rq->t_done - rq->t_submit);
        sv->edge_work += (double)rq->work * (double)(g.m / 2);
        sv->last_done = rq->t_done;
    } else {
        sv->failed++;
    }
    sv->cv_done.notify_all();
}

// With fewer requests running than slots and none waiting, a request
// starting now takes a larger share of the GPU: 1/max(2, running + 1) of
// the resident-workgroup capacity (half the GPU when alone, so that a
// second arrival still finds room), if its scratch fits the budget;
// otherwise it keeps its submission-time share.
static void widen_grid(nk_server *sv, Request *rq, int busy) {
    const int div = std::max(2, busy + 1);
    if (div >= sv->n_share) return;
    const ServerGraph &g = *rq->g;
    const bool pair = rq->sources.empty();
    TuningOverride tuned(g.tuned && !pair ? &g.tuning : nullptr);
    LaunchPlan pl;
    if (plan_launch(pair ? kModePair : kModeBC, g.n, std::max<long long>(rq->tasks, 1), -div, &pl) != NK_OK) {
        clear_error();
        return;
    }
    if (pl.grid <= rq->grid) return;
    const size_t fp = request_footprint(g, rq->tasks, pl.grid, pair);
    if (sv->pool_bytes + sv->running_bytes + fp > sv->budget) return;
    rq->grid = pl.grid;
    rq->footprint = fp;
}

static void worker_main(nk_server *sv) {
    (void)hipSetDevice(sv->device);
    for (;;) {
        std::vector<std::pair<int, Request *>> to_start;
        {
            std::unique_lock<std::mutex> lk(sv->mu);
            int busy = 0;
            for (auto &sl : sv->slots) busy += sl.req != nullptr;
            if (sv->stop && busy == 0) return;
            if (busy == 0 && sv->pending.empty())
                sv->cv_work.wait_for(lk, std::chrono::milliseconds(50));
            // admit in arrival order while a slot is free and the footprint fits
            for (size_t i = 0; i < sv->slots.size() && !sv->pending.empty(); ++i) {
                if (sv->slots[i].req) continue;
                Request *rq = sv->pending.front();
                if (sv->pool_bytes + sv->running_bytes + rq->footprint > sv->budget && busy > 0) break;
                sv->pending.pop_front();
                // a wider grid only while nothing else waits: under load every
                // request keeps its fair share
                if (sv->pending.empty()) widen_grid(sv, rq, busy);
                sv->running_bytes += rq->footprint;
                sv->slots[i].req = rq;  // reserve
                to_start.push_back({(int)i, rq});
                busy++;
            }
            sv->max_inflight = std::max(sv->max_inflight, busy);
        }
        for (auto &ps : to_start) start_request(sv, sv->slots[ps.first], ps.second);
        bool any = false;
        for (auto &sl : sv->slots) {
            if (!sl.req) continue;
            any = true;
            const hipError_t q = hipEventQuery(sl.ev);
            if (q == hipSuccess) {
                finish_request(sv, sl);
            } else if (q != hipErrorNotReady) {
                (void)hipGetLastError();
                sl.req->status = NK_E_HIP;
                (void)hipStreamSynchronize(sl.stream);
                finish_request(sv, sl);
            }
        }
        if (any) std::this_thread::sleep_for(std::chrono::microseconds(50));
    }
}

}  // namespace nk

using namespace nk;

extern "C" {

nk_status nk_server_create(size_t hbm_budget_bytes, int32_t n_slots, nk_server **out) {
    clear_error();
    if (!out) return fail(NK_E_INVALID_ARG, "out is NULL");
    *out = nullptr;
    if (n_slots < 0 || n_slots > 16) return fail(NK_E_INVALID_ARG, "n_slots must lie in [0, 16]");
    if (n_slots == 0) n_slots = 4;
    DevInfo di;
    nk_status st = dev_info(&di);
    if (st != NK_OK) return st;
    nk_server *sv = new nk_server();
    sv->device = di.device;
    sv->budget = hbm_budget_bytes;
    sv->n_share = n_slots;
    sv->slots.resize(n_slots);
    for (auto &sl : sv->slots) {
        void *h = nullptr;
        if (hipStreamCreateWithFlags(&sl.stream, hipStreamNonBlocking) != hipSuccess ||
            hipEventCreateWithFlags(&sl.ev, hipEventDisableTiming) != hipSuccess ||
            hipMalloc((void **)&sl.dst, sizeof(DevStatus)) != hipSuccess ||
            hipHostMalloc(&h, sizeof(DevStatus), hipHostMallocDefault) != hipSuccess) {
            (void)hipGetLastError();
            nk_server_destroy(sv);
            return fail(NK_E_HIP, "could not create server streams");
        }
        sl.hst = (DevStatus *)h;
    }
    sv->worker = std::thread(worker_main, sv);
    *out = sv;
    return NK_OK;
}

nk_status nk_server_add_graph(nk_server *sv, const int32_t *rowptr, const int32_t *colidx, int32_t n, int64_t m,
                              int32_t *graph_id) {
    clear_error();
    if (!sv || !graph_id) return fail(NK_E_INVALID_ARG, "server or graph_id is NULL");
    nk_status st = check_graph_args(rowptr, colidx, n, m);
    if (st != NK_OK) return st;
    if (n < 1) return fail(NK_E_INVALID_ARG, "a served graph needs n >= 1");
    hipStream_t s = nullptr;
    NK_HIP(hipStreamCreateWithFlags(&s, hipStreamNonBlocking));
    ServerGraph g;
    g.n = n;
    g.m = m;
    const long long words = ((long long)n + 31) / 32;
    g.bytes = round256(((size_t)n + 1) * 4) + round256((size_t)std::max<int64_t>(m, 1) * 4) +
              2 * round256((size_t)n * 4) + round256((size_t)words * 4);
    {
        std::lock_guard<std::mutex> lk(sv->mu);
        if (sv->pool_bytes + g.bytes > sv->budget) {
            (void)hipStreamDestroy(s);
            return fail(NK_E_BUDGET, "graph of %zu bytes does not fit the HBM budget", g.bytes);
        }
    }
    Scratch scr;
    DevStatus *dst;
    if ((st = scr.get(1, &dst)) != NK_OK) return st;
    auto cleanup = [&](nk_status code) {
        (void)hipStreamSynchronize(s);
        (void)hipStreamDestroy(s);
        if (g.rowptr) (void)hipFree(g.rowptr);
        if (g.colidx) (void)hipFree(g.colidx);
        if (g.perm) (void)hipFree(g.perm);
        if (g.inv) (void)hipFree(g.inv);
        if (g.iso) (void)hipFree(g.iso);
        return code;
    };
    if (hipMalloc((void **)&g.rowptr, ((size_t)n + 1) * 4) != hipSuccess ||
        hipMalloc((void **)&g.colidx, (size_t)std::max<int64_t>(m, 1) * 4) != hipSuccess ||
        hipMalloc((void **)&g.perm, (size_t)n * 4) != hipSuccess ||
        hipMalloc((void **)&g.inv, (size_t)n * 4) != hipSuccess ||
        hipMalloc((void **)&g.iso, (size_t)words * 4) != hipSuccess) {
        (void)hipGetLastError();
        return cleanup(fail(NK_E_NO_MEMORY, "graph allocation failed"));
    }
    if (launch_status_init(dst, s) != hipSuccess || launch_validate(rowptr, colidx, n, m, 0, dst, s) != hipSuccess)
        return cleanup(fail(NK_E_HIP, "validation launch failed"));
    Relabeled rl;
    if ((st = relabel_graph(rowptr, colidx, n, m, dst, scr, s, &rl)) != NK_OK) return cleanup(st);
    if (hipMemcpyAsync(g.rowptr, rl.rowptr, ((size_t)n + 1) * 4, hipMemcpyDeviceToDevice, s) != hipSuccess ||
        (m > 0 && hipMemcpyAsync(g.colidx, rl.colidx, (size_t)m * 4, hipMemcpyDeviceToDevice, s) != hipSuccess) ||
        hipMemcpyAsync(g.perm, rl.perm, (size_t)n * 4, hipMemcpyDeviceToDevice, s) != hipSuccess ||
        hipMemcpyAsync(g.inv, rl.inv, (size_t)n * 4, hipMemcpyDeviceToDevice, s) != hipSuccess ||
        launch_iso_bitmap(g.rowptr, n, g.iso, s) != hipSuccess)
        return cleanup(fail(NK_E_HIP, "graph copy failed"));
    DevStatus *h = host_status();
    if (!h) return cleanup(fail(NK_E_NO_MEMORY, "pinned status buffer"));
    if ((st = finish(dst, h, s)) != NK_OK) return cleanup(st);
    int32_t info[8];
    if ((st = vd_bound_impl(rowptr, colidx, n, m, info, s)) != NK_OK) return cleanup(st);
    g.vd = info[4];
    // the autotuner cache's tuning for this graph's shape, if one is registered
    if (tuning_cache_active()) {
        int64_t dmax = 0;
        if ((st = graph_max_degree(g.rowptr, n, s, &dmax)) != NK_OK) return cleanup(st);
        g.tuned = cached_tuning(n, m, dmax, &g.tuning);
    }
    (void)hipStreamDestroy(s);
    std::lock_guard<std::mutex> lk(sv->mu);
    sv->pool_bytes += g.bytes;
    sv->graphs.push_back(g);
    *graph_id = (int32_t)sv->graphs.size() - 1;
    return NK_OK;
}

nk_status nk_server_submit(nk_server *sv, int32_t graph_id, const int32_t *sources, int32_t k, double eps,
                           double delta, uint64_t seed, double *bc_out, int64_t *ticket) {
    clear_error();
    if (!sv || !ticket) return fail(NK_E_INVALID_ARG, "server or ticket is NULL");
    std::unique_lock<std::mutex> lk(sv->mu);
    if (graph_id < 0 || graph_id >= (int32_t)sv->graphs.size()) return fail(NK_E_INVALID_ARG, "unknown graph %d", graph_id);
    const ServerGraph &g = sv->graphs[graph_id];
    if (k < 0 || (k > 0 && !sources)) return fail(NK_E_INVALID_ARG, "bad source list");
    if (k == 0 && (!(eps > 0.0 && eps < 1.0) || !(delta > 0.0 && delta < 1.0)))
        return fail(NK_E_INVALID_ARG, "eps and delta must lie in (0, 1)");
    Request *rq = new Request();
    rq->graph = graph_id;
    rq->g = &g;
    if (k > 0) {
        rq->sources.assign(sources, sources + k);
        for (int32_t v : rq->sources)
            if (v < 0 || v >= g.n) {
                delete rq;
                return fail(NK_E_INVALID_ARG, "source %d out of range", v);
            }
        rq->work = k;
    }
    rq->eps = eps;
    rq->delta = delta;
    rq->seed = seed;
    rq->out = bc_out;
    const long long tasks = k > 0 ? k : (g.n >= 2 ? nk_rk_sample_size(eps, delta, g.vd) : 0);
    // the kernel's grid: an equal share of the workgroups the GPU holds at
    // once for this kernel (block size and occupancy depend on the graph),
    // so that n_slots requests together fill the GPU
    {
        TuningOverride tuned(g.tuned && k > 0 ? &g.tuning : nullptr);
        LaunchPlan pl;
        const nk_status ps = plan_launch(k > 0 ? kModeBC : kModePair, g.n, std::max<long long>(tasks, 1),
                                         -sv->n_share, &pl);
        if (ps != NK_OK) {
            delete rq;
            return ps;
        }
        rq->grid = pl.grid;
    }
    // a smaller grid (slower, but admissible) when that share's scratch does
    // not fit the budget beside the resident graphs
    rq->tasks = tasks;
    rq->footprint = request_footprint(g, tasks, rq->grid, k == 0);
    while (rq->grid > 1 && sv->pool_bytes + rq->footprint > sv->budget) {
        rq->grid = (rq->grid + 1) / 2;
        rq->footprint = request_footprint(g, tasks, rq->grid, k == 0);
    }
    if (sv->pool_bytes + rq->footprint > sv->budget) {
        const size_t need = rq->footprint;
        delete rq;
        return fail(NK_E_BUDGET, "request needs %zu bytes beside the resident graphs; budget is %zu", need,
                    sv->budget);
    }
    rq->ticket = sv->next_ticket++;
    rq->t_submit = now_s();
    if (sv->first_submit == 0) sv->first_submit = rq->t_submit;
    sv->requests[rq->ticket] = rq;
    sv->pending.push_back(rq);
    *ticket = rq->ticket;
    sv->cv_work.notify_one();
    return NK_OK;
}

nk_status nk_server_poll(nk_server *sv, int64_t ticket, int32_t *done) {
    clear_error();
    if (!sv || !done) return fail(NK_E_INVALID_ARG, "server or done is NULL");
    std::lock_guard<std::mutex> lk(sv->mu);
    auto it = sv->requests.find(ticket);
    if (it == sv->requests.end()) return fail(NK_E_INVALID_ARG, "unknown ticket");
    *done = it->second->done ? 1 : 0;
    return NK_OK;
}

nk_status nk_server_wait(nk_server *sv, int64_t ticket, double timeout_s, double *latency_s) {
    clear_error();
    if (!sv) return fail(NK_E_INVALID_ARG, "server is NULL");
    std::unique_lock<std::mutex> lk(sv->mu);
    auto it = sv->requests.find(ticket);
    if (it == sv->requests.end()) return fail(NK_E_INVALID_ARG, "unknown ticket");
    Request *rq = it->second;
    const auto deadline = std::chrono::steady_clock::now() + std::chrono::duration<double>(timeout_s);
    while (!rq->done) {
        if (timeout_s >= 0 && sv->cv_done.wait_until(lk, deadline) == std::cv_status::timeout && !rq->done)
            return fail(NK_E_TIMEOUT, "request %lld not done", (long long)ticket);
        if (timeout_s < 0) sv->cv_done.wait(lk);
    }
    const nk_status st = rq->status;
    if (latency_s) *latency_s = rq->t_done - rq->t_submit;
    sv->requests.erase(it);
    delete rq;
    if (st != NK_OK) return fail(st, "request failed");
    return NK_OK;
}

nk_status nk_server_stats(nk_server *sv, double *out) {
    clear_error();
    if (!sv || !out) return fail(NK_E_INVALID_ARG, "server or out is NULL");
    std::lock_guard<std::mutex> lk(sv->mu);
    std::vector<double> lat = sv->latency;
    std::sort(lat.begin(), lat.end());
    auto pct = [&](double q) {
        if (lat.empty()) return 0.0;
        const size_t i = (size_t)std::min<double>((double)lat.size() - 1, std::ceil(q * lat.size()) - 1);
        return lat[i];
    };
    const double span = sv->last_done > sv->first_submit ? sv->last_done - sv->first_submit : 0.0;
    out[0] = (double)sv->completed;
    out[1] = (double)sv->failed;
    out[2] = pct(0.50) * 1e3;
    out[3] = pct(0.99) * 1e3;
    out[4] = lat.empty() ? 0.0 : lat.back() * 1e3;
    out[5] = span > 0 ? sv->edge_work / span / 1e9 : 0.0;
    out[6] = (double)sv->max_inflight;
    out[7] = (double)(sv->pool_bytes + sv->running_bytes);
    return NK_OK;
}

nk_status nk_server_reset_stats(nk_server *sv) {
    clear_error();
    if (!sv) return fail(NK_E_INVALID_ARG, "server is NULL");
    std::lock_guard<std::mutex> lk(sv->mu);
    sv->latency.clear();
    sv->first_submit = sv->last_done = 0;
    sv->completed = sv->failed = 0;
    sv->edge_work = 0;
    sv->max_inflight = 0;
    return NK_OK;
}

void nk_server_destroy(nk_server *sv) {
    if (!sv) return;
    {
        std::lock_guard<std::mutex> lk(sv->mu);
        sv->stop = true;
        // requests never started are dropped
        for (Request *rq : sv->pending) {
            rq->status = NK_E_INTERNAL;
            rq->done = true;
        }
        sv->pending.clear();
        sv->cv_work.notify_all();
    }
    if (sv->worker.joinable()) sv->worker.join();
    for (auto &kv : sv->requests) delete kv.second;
    for (auto &sl : sv->slots) {
        if (sl.stream) (void)hipStreamDestroy(sl.stream);
        if (sl.ev) (void)hipEventDestroy(sl.ev);
        if (sl.dst) (void)hipFree(sl.dst);
        if (sl.hst) (void)hipHostFree(sl.hst);
        if (sl.staging) (void)hipHostFree(sl.staging);
    }
    for (auto &g : sv->graphs) {
        (void)hipFree(g.rowptr);
        (void)hipFree(g.colidx);
        (void)hipFree(g.perm);
        (void)hipFree(g.inv);
        (void)hipFree(g.iso);
    }
    delete sv;
}

}  // extern "C"
