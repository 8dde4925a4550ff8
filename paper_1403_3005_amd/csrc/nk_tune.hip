// Autotuner for the source-set Brandes kernels.
//
// For a graph and a sample of its sources, times with the source-set entry
// point every setting of the workgroup size and the two direction
// thresholds (forward bottom-up switch, backward push switch) on the
// one-source kernel, then, from the fastest of those, the resident
// workgroups per compute unit, the sources per workgroup task (the
// multi-source kernel) and the workgroups per source (the group kernel),
// and keeps the fastest.  Winners are stored per graph-shape bucket -- (floor log2 n,
// round log2 mean degree, round log2 of max degree / mean degree) -- in a
// flat JSON object.  Once a cache file is registered (nk_set_tuning_cache),
// single-graph calls, batched plans and the server run every graph whose
// bucket has an entry under that entry's tuning.
#include <stdio.h>
#include <string.h>

#include <chrono>
#include <cmath>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "nk_runtime.h"

namespace nk {

static std::mutex g_cache_mu;

static std::string bucket_key(int32_t n, int64_t m, int64_t maxdeg) {
    const double mean = n > 0 ? (double)m / (double)n : 0.0;
    const int ln = n > 0 ? (int)std::floor(std::log2((double)n)) : 0;
    const int ld = mean > 0 ? (int)std::lround(std::log2(mean)) : -99;
    const int ls = (mean > 0 && maxdeg > 0) ? (int)std::lround(std::log2((double)maxdeg / mean)) : -99;
    char buf[64];
    snprintf(buf, sizeof(buf), "n%d_d%d_s%d", ln, ld, ls);
    return buf;
}

// The cache file is a flat JSON object:
// {"key": [block, bu_ratio, bw_ratio, wg_per_cu, batch, ms, kernel_flags,
// group], ...}, kernel_flags being the winner's tuning flag bits 3 and 4
// (group kernel forced or forbidden); entries of six values (no kernel
// choice: the flags stay the caller's, group 0) and of four values
// [block, bu_ratio, bw_ratio, ms] (also wg_per_cu = 0, batch = 0) are read
// too.
static std::map<std::string, std::vector<double>> read_cache(const char *path) {
    std::map<std::string, std::vector<double>> out;
    if (!path) return out;
    FILE *f = fopen(path, "r");
    if (!f) return out;
    std::string text;
    char buf[4096];
    size_t got;
    while ((got = fread(buf, 1, sizeof(buf), f)) > 0) text.append(buf, got);
    fclose(f);
    size_t i = 0;
    while ((i = text.find('"', i)) != std::string::npos) {
        const size_t j = text.find('"', i + 1);
        if (j == std::string::npos) break;
        const std::string key = text.substr(i + 1, j - i - 1);
        const size_t a = text.find('[', j), b = text.find(']', j);
        if (a == std::string::npos || b == std::string::npos || b < a) break;
        std::vector<double> vals;
        const char *p = text.c_str() + a + 1;
        const char *end = text.c_str() + b;
        while (p < end) {
            char *q = nullptr;
            const double v = strtod(p, &q);
            if (q == p) {
                ++p;
                continue;
            }
            vals.push_back(v);
            p = q;
        }
        if (vals.size() == 4) vals = {vals[0], vals[1], vals[2], 0.0, 0.0, vals[3]};
        if (vals.size() == 6) vals.insert(vals.end(), {-1.0, 0.0});
        if (vals.size() == 8) out[key] = vals;
        i = b + 1;
    }
    return out;
}

static bool write_cache(const char *path, const std::map<std::string, std::vector<double>> &c) {
    const std::string tmp = std::string(path) + ".tmp";
    FILE *f = fopen(tmp.c_str(), "w");
    if (!f) return false;
    fprintf(f, "{\n");
    size_t k = 0;
    for (const auto &kv : c) {
        fprintf(f, "  \"%s\": [%d, %.6g, %.6g, %d, %d, %.6g, %d, %d]%s\n", kv.first.c_str(), (int)kv.second[0],
                kv.second[1], kv.second[2], (int)kv.second[3], (int)kv.second[4], kv.second[5],
                (int)kv.second[6], (int)kv.second[7], ++k < c.size() ? "," : "");
    }
    fprintf(f, "}\n");
    fclose(f);
    return rename(tmp.c_str(), path) == 0;
}

nk_status graph_max_degree(const int32_t *rowptr, int32_t n, hipStream_t s, int64_t *out) {
    *out = 0;
    if (n <= 0) return NK_OK;
    Scratch scr;
    unsigned long long *key;
    nk_status st;
    if ((st = scr.get(1, &key)) != NK_OK) return st;
    NK_HIP(launch_fill_u64(key, 0ULL, 1, s));
    NK_HIP(launch_argmax_degree(rowptr, n, key, s));
    unsigned long long k = 0;
    NK_HIP(hipMemcpyAsync(&k, key, 8, hipMemcpyDeviceToHost, s));
    NK_HIP(hipStreamSynchronize(s));
    *out = (int64_t)(k >> 32);
    return NK_OK;
}

// The registered cache: its path and parsed entries (read once per
// registration, refreshed when the autotuner writes to the same file).
static std::string g_active_path;
static std::map<std::string, std::vector<double>> g_active;
// set while the autotuner times its candidates: they must run as given
static thread_local bool t_trials = false;

static void merge_entry(const std::vector<double> &e, nk_tuning *t) {
    t->block = (int32_t)e[0];
    t->bu_ratio = (float)e[1];
    t->bw_ratio = (float)e[2];
    t->wg_per_cu = (int32_t)e[3];
    t->batch = (int32_t)e[4];
    if (e[6] >= 0.0) {
        t->flags = (t->flags & ~24) | ((int32_t)e[6] & 24);
        t->group = (int32_t)e[7];
    }
}

bool tuning_cache_active() {
    if (t_trials) return false;
    std::lock_guard<std::mutex> lk(g_cache_mu);
    return !g_active_path.empty();
}

bool cached_tuning(int32_t n, int64_t m, int64_t max_deg, nk_tuning *out) {
    if (t_trials) return false;
    const nk_tuning base = tuning_get();
    std::lock_guard<std::mutex> lk(g_cache_mu);
    if (g_active_path.empty()) return false;
    auto it = g_active.find(bucket_key(n, m, max_deg));
    if (it == g_active.end()) return false;
    *out = base;
    merge_entry(it->second, out);
    return true;
}

}  // namespace nk

using namespace nk;

extern "C" {

nk_status nk_tuning_lookup(const char *cache_path, int32_t n, int64_t m, int64_t max_deg, nk_tuning *out) {
    clear_error();
    if (!cache_path || !out) return fail(NK_E_INVALID_ARG, "cache_path or out is NULL");
    std::lock_guard<std::mutex> lk(g_cache_mu);
    auto c = read_cache(cache_path);
    auto it = c.find(bucket_key(n, m, max_deg));
    if (it == c.end()) return fail(NK_E_INVALID_ARG, "no cached tuning for this graph shape");
    nk_tuning t = tuning_get();
    merge_entry(it->second, &t);
    *out = t;
    return NK_OK;
}

nk_status nk_set_tuning_cache(const char *cache_path) {
    clear_error();
    std::lock_guard<std::mutex> lk(g_cache_mu);
    if (!cache_path || !cache_path[0]) {
        g_active_path.clear();
        g_active.clear();
        return NK_OK;
    }
    FILE *f = fopen(cache_path, "r");
    if (!f) return fail(NK_E_INVALID_ARG, "cannot read %s", cache_path);
    fclose(f);
    g_active_path = cache_path;
    g_active = read_cache(cache_path);
    return NK_OK;
}

nk_status nk_autotune(const int32_t *rowptr, const int32_t *colidx, int32_t n, int64_t m, const int32_t *sources,
                      int32_t k, const char *cache_path, nk_tuning *best, void *stream) {
    clear_error();
    nk_status st = check_graph_args(rowptr, colidx, n, m);
    if (st != NK_OK) return st;
    if (n == 0 || k <= 0 || !sources || !best) return fail(NK_E_INVALID_ARG, "need n > 0, k > 0, sources, best");
    hipStream_t s = (hipStream_t)stream;
    int64_t dmax = 0;
    if ((st = graph_max_degree(rowptr, n, s, &dmax)) != NK_OK) return st;
    double *bc = nullptr;
    NK_HIP(hipMalloc((void **)&bc, sizeof(double) * (size_t)n));
    const nk_tuning saved = tuning_get();
    nk_tuning win = saved;
    double best_ms = 1e300;
    nk_status result = NK_OK;
    struct TrialScope {
        TrialScope() { t_trials = true; }
        ~TrialScope() { t_trials = false; }
    } trials;
    // times one setting: an untimed run (allocation, caches), then the timed one
    auto trial = [&](const nk_tuning &t) -> bool {
        tuning_set(t);
        st = nk_bc_sources(rowptr, colidx, n, m, sources, k, 1.0, bc, stream);
        if (st != NK_OK) {
            result = st;
            return false;
        }
        const auto t0 = std::chrono::steady_clock::now();
        st = nk_bc_sources(rowptr, colidx, n, m, sources, k, 1.0, bc, stream);
        const double ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
        if (st != NK_OK) {
            result = st;
            return false;
        }
        if (ms < best_ms) {
            best_ms = ms;
            win = t;
        }
        return true;
    };
    // stage 1: block size x the two direction thresholds, one source per task
    const int blocks[] = {256, 512, 1024};
    const float bus[] = {0.0f, 2.0f, 8.0f, 16.0f, 64.0f};
    const float bws[] = {0.0f, 0.1f, 0.25f, 1.0f};
    for (int b : blocks)
        for (float bu : bus)
            for (float bw : bws) {
                nk_tuning t = saved;
                t.block = b;
                t.bu_ratio = bu;
                t.bw_ratio = bw;
                t.wg_per_cu = 0;
                t.batch = 1;
                t.flags = (saved.flags & ~24) | 16;   // the one-source kernel
                t.group = 0;
                if (result == NK_OK) trial(t);
            }
    // stage 2: from the stage-1 winner, one resident workgroup per compute
    // unit, then the multi-source kernel with 4, 8 and 16 sources per task
    if (result == NK_OK) {
        const nk_tuning base = win;
        nk_tuning t = base;
        t.wg_per_cu = 1;
        trial(t);
        for (int b : {4, 8, 16}) {
            t = base;
            t.batch = b;
            t.block = 1024;
            if (result == NK_OK) trial(t);
        }
        // the group kernel with 2, 4 and 8 workgroups per source, where its
        // visited bitmap fits LDS
        for (int g : {2, 4, 8}) {
            t = base;
            t.flags = (saved.flags & ~24) | 8;
            t.group = g;
            t.block = 1024;
            t.wg_per_cu = 0;
            tuning_set(t);
            const bool fits = group_wanted(n, m);
            if (fits && result == NK_OK) trial(t);
        }
    }
    tuning_set(saved);
    (void)hipFree(bc);
    if (result != NK_OK) return result;
    *best = win;
    if (cache_path) {
        std::lock_guard<std::mutex> lk(g_cache_mu);
        auto c = read_cache(cache_path);
        c[bucket_key(n, m, dmax)] = {(double)win.block, (double)win.bu_ratio, (double)win.bw_ratio,
                                     (double)win.wg_per_cu, (double)win.batch, best_ms,
                                     (double)(win.flags & 24), (double)win.group};
        if (!write_cache(cache_path, c)) return fail(NK_E_INVALID_ARG, "cannot write %s", cache_path);
        if (g_active_path == cache_path) g_active = c;
    }
    clear_error();
    return NK_OK;
}

}  // extern "C"
