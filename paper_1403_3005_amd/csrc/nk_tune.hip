// Autotuner for the per-source Brandes kernel.
//
// For a graph and a sample of its sources, times every candidate setting of
// the workgroup size and the two direction thresholds (forward bottom-up
// switch, backward push switch) with the source-set entry point, and keeps
// the fastest.  Winners are stored per graph-shape bucket -- (floor log2 n,
// round log2 mean degree, round log2 of max degree / mean degree) -- in a
// flat JSON object, so later runs on graphs of the same shape can reuse
// them without timing.
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

// The cache file is a flat JSON object: {"key": [block, bu_ratio, bw_ratio, ms], ...}.
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
        if (vals.size() == 4) out[key] = vals;
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
        fprintf(f, "  \"%s\": [%d, %.6g, %.6g, %.6g]%s\n", kv.first.c_str(), (int)kv.second[0], kv.second[1],
                kv.second[2], kv.second[3], ++k < c.size() ? "," : "");
    }
    fprintf(f, "}\n");
    fclose(f);
    return rename(tmp.c_str(), path) == 0;
}

static nk_status max_degree(const int32_t *rowptr, int32_t n, hipStream_t s, int64_t *out) {
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
    t.block = (int32_t)it->second[0];
    t.bu_ratio = (float)it->second[1];
    t.bw_ratio = (float)it->second[2];
    *out = t;
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
    if ((st = max_degree(rowptr, n, s, &dmax)) != NK_OK) return st;
    double *bc = nullptr;
    NK_HIP(hipMalloc((void **)&bc, sizeof(double) * (size_t)n));
    const nk_tuning saved = tuning_get();
    const int blocks[] = {256, 512, 1024};
    const float bus[] = {0.0f, 2.0f, 8.0f, 16.0f, 64.0f};
    const float bws[] = {0.0f, 0.1f, 0.25f, 1.0f};
    nk_tuning win = saved;
    double best_ms = 1e300;
    nk_status result = NK_OK;
    for (int b : blocks) {
        for (float bu : bus) {
            for (float bw : bws) {
                nk_tuning t = saved;
                t.block = b;
                t.bu_ratio = bu;
                t.bw_ratio = bw;
                tuning_set(t);
                // one untimed run (allocation, caches), then the timed one
                st = nk_bc_sources(rowptr, colidx, n, m, sources, k, 1.0, bc, stream);
                if (st != NK_OK) {
                    result = st;
                    break;
                }
                const auto t0 = std::chrono::steady_clock::now();
                st = nk_bc_sources(rowptr, colidx, n, m, sources, k, 1.0, bc, stream);
                const double ms =
                    std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
                if (st != NK_OK) {
                    result = st;
                    break;
                }
                if (ms < best_ms) {
                    best_ms = ms;
                    win = t;
                }
            }
            if (result != NK_OK) break;
        }
        if (result != NK_OK) break;
    }
    tuning_set(saved);
    (void)hipFree(bc);
    if (result != NK_OK) return result;
    *best = win;
    if (cache_path) {
        std::lock_guard<std::mutex> lk(g_cache_mu);
        auto c = read_cache(cache_path);
        c[bucket_key(n, m, dmax)] = {(double)win.block, (double)win.bu_ratio, (double)win.bw_ratio, best_ms};
        if (!write_cache(cache_path, c)) return fail(NK_E_INVALID_ARG, "cannot write %s", cache_path);
    }
    clear_error();
    return NK_OK;
}

}  // extern "C"
