// Source-set betweenness that allocates nothing (nk_bc_sources_noalloc).
//
// The same kernels as nk_bc_sources, on the graph under the caller's own
// vertex ids (the degree relabelling needs sort buffers), with every piece
// of device scratch -- the status block, the isolated-vertex bitmap and the
// per-workgroup-slot state of the persistent kernel -- carved from one
// fixed array in device memory, and the status read back into host stack
// memory.  No device or pinned allocation, no event, no library routine
// that allocates.  The grid shrinks until the slots' state fits the array.
#include <string.h>

#include <mutex>

#include "nk_runtime.h"

namespace nk {

constexpr size_t kNoAllocBytes = (size_t)128 << 20;

// One copy per device, held until the process ends.  Host code never uses
// this name as an address: it takes the device address once per device
// (scratch_base) and passes that to kernels.
static __device__ __align__(256) unsigned char scratch[kNoAllocBytes];

static std::mutex g_base_mu;
static void *g_base[64];

// Device address of `scratch` on the current device, looked up on the first
// call on that device.
static nk_status scratch_base(void **out) {
    int dev = 0;
    NK_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= 64) return fail(NK_E_HIP, "device index %d out of range", dev);
    std::lock_guard<std::mutex> lk(g_base_mu);
    if (!g_base[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            (void)hipGetLastError();
            return fail(NK_E_HIP, "hipGetSymbolAddress(scratch) failed: %s", hipGetErrorString(e));
        }
        g_base[dev] = p;
    }
    *out = g_base[dev];
    return NK_OK;
}

// Bump carving of the array in 256-byte aligned pieces.
struct Carve {
    unsigned char *base;
    size_t used;
    template <typename T>
    T *take(long long count) {
        const size_t bytes = ((size_t)(count > 0 ? count : 1) * sizeof(T) + 255) & ~(size_t)255;
        if (used + bytes > kNoAllocBytes) return nullptr;
        T *p = reinterpret_cast<T *>(base + used);
        used += bytes;
        return p;
    }
};

static size_t round256(size_t b) { return (b + 255) & ~(size_t)255; }

static nk_status read_status(DevStatus *dst, DevStatus *host, hipStream_t s) {
    NK_HIP(hipMemcpyAsync(host, dst, sizeof(DevStatus), hipMemcpyDeviceToHost, s));
    NK_HIP(hipStreamSynchronize(s));
    return map_err(host->err);
}

}  // namespace nk

using namespace nk;

extern "C" {

nk_status nk_bc_sources_noalloc(const int32_t *rowptr, const int32_t *colidx, int32_t n, int64_t m,
                                const int32_t *sources, int32_t k, double scale, double *bc, void *stream) {
    clear_error();
    stats_clear();
    nk_status st = check_graph_args(rowptr, colidx, n, m);
    if (st != NK_OK) return st;
    if (n == 0) return NK_OK;
    if (!bc) return fail(NK_E_INVALID_ARG, "bc is NULL");
    if (k < 0) return fail(NK_E_INVALID_ARG, "k is negative");
    if (k > 0 && !sources) return fail(NK_E_INVALID_ARG, "sources is NULL");
    hipStream_t s = (hipStream_t)stream;
    void *base = nullptr;
    if ((st = scratch_base(&base)) != NK_OK) return st;
    Carve cv = {reinterpret_cast<unsigned char *>(base), 0};
    const long long words = ((long long)n + 31) / 32;
    DevStatus *dst = cv.take<DevStatus>(1);
    uint32_t *iso = cv.take<uint32_t>(words);
    if (!dst || !iso)
        return fail(NK_E_BUDGET, "n = %d needs %zu bytes of fixed scratch; the no-allocation scratch holds %zu", n,
                    round256(sizeof(DevStatus)) + round256((size_t)words * 4), kNoAllocBytes);
    LaunchPlan plan = {};
    int where = 2;
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
    // the whole plan, and the scratch it needs, before anything is launched
    const bool persistent = k > 0 && !plan_lds(lds_graph_bytes(n, m), n, k, &plan);
    long long cells = 0;
    if (persistent) {
        DevInfo di;
        if ((st = dev_info(&di)) != NK_OK) return st;
        const nk_tuning t = tuning_get();
        int block = t.block;
        if (block != 256 && block != 512 && block != 1024) block = auto_block(n);
        const size_t bm_bytes = (size_t)words * 4;
        hipFuncAttributes attr;
        NK_HIP(hipFuncGetAttributes(&attr, brandes_kernel(kModeBC, block, true).fn));
        const bool lds = attr.sharedSizeBytes + bm_bytes <= di.lds_per_block && !(t.flags & 1);
        KernelRef kr = brandes_kernel(kModeBC, block, lds);
        const size_t dyn = lds ? bm_bytes : 0;
        if (dyn > 0) NK_HIP(hipFuncSetAttribute(kr.fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)dyn));
        int occ = 0;
        NK_HIP(hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, kr.fn, block, dyn));
        if (occ < 1) return fail(NK_E_INTERNAL, "kernel does not fit a compute unit (block %d, lds %zu)", block, dyn);
        if (t.wg_per_cu > 0 && t.wg_per_cu < occ) occ = t.wg_per_cu;
        long long grid = std::min<long long>((long long)di.cus * occ, k);
        const long long stride = (((long long)n + 2) + 63) / 64 * 64;
        const long long bm_words = (words + 63) / 64 * 64;
        // per slot: sigma u64, push accumulator f64, seven int32 arrays
        // (level degree sums, d, level offsets, three level-list arrays,
        // bottom-up candidates), and the visited bitmap unless it is in LDS;
        // each array is one 256-byte aligned piece over all slots
        auto need = [&](long long g) {
            const long long c = g * stride;
            size_t b = round256((size_t)c * 8) * 2 + round256((size_t)c * 4) * 7;
            if (!lds) b += round256((size_t)(g * bm_words) * 4);
            return b;
        };
        const size_t room = kNoAllocBytes - cv.used;
        if (need(1) > room)
            return fail(NK_E_BUDGET,
                        "n = %d needs %zu bytes of scratch for one workgroup slot; the no-allocation scratch holds "
                        "%zu beside %zu fixed bytes",
                        n, need(1), kNoAllocBytes, cv.used);
        while (grid > 1 && need(grid) > room) grid = grid > di.cus ? (grid - 1) / di.cus * di.cus : grid - 1;
        cells = grid * stride;
        p.sigma = cv.take<unsigned long long>(cells);
        p.dacc = cv.take<double>(cells);
        p.ldeg = cv.take<int32_t>(cells);
        p.d = cv.take<int32_t>(cells);
        p.lvl = cv.take<int32_t>(cells);
        p.lv = cv.take<int32_t>(cells);
        p.la = cv.take<int32_t>(cells);
        p.ld = cv.take<int32_t>(cells);
        p.cand = cv.take<int32_t>(cells);
        p.bmg = lds ? nullptr : cv.take<uint32_t>(grid * bm_words);
        if (!p.sigma || !p.dacc || !p.ldeg || !p.d || !p.lvl || !p.lv || !p.la || !p.ld || !p.cand ||
            (!lds && !p.bmg))
            return fail(NK_E_INTERNAL, "scratch carving overflowed");
        p.iso = iso;
        p.stride = stride;
        p.bm_words = bm_words;
        p.bu_ratio = t.bu_ratio;
        p.bw_ratio = t.bw_ratio;
        plan.block = block;
        plan.grid = (int)grid;
        plan.dyn_lds = dyn;
        plan.lds = lds;
        plan.kernel = kr;
        where = lds ? 1 : 0;
    }
    DevStatus h;
    memset(&h, 0, sizeof(h));
    NK_HIP(launch_status_init(dst, s));
    NK_HIP(launch_validate(rowptr, colidx, n, m, 0, dst, s));
    NK_HIP(launch_fill_f64(bc, 0.0, n, s));
    if (k == 0) {
        st = read_status(dst, &h, s);
        stats_record(h, 0, 0, 0, 0.0f);
        return st;
    }
    if (persistent) {
        // the array keeps the previous call's contents: clear what the
        // kernel expects clear
        NK_HIP(launch_fill_u64(p.sigma, 0ULL, cells, s));
        NK_HIP(launch_fill_f64(p.dacc, 0.0, cells, s));
        NK_HIP(launch_iso_bitmap(rowptr, n, iso, s));
    }
    plan.kernel.launch(dim3(plan.grid), dim3(plan.block), plan.dyn_lds, s, p);
    NK_HIP(hipGetLastError());
    if (scale != 1.0) NK_HIP(launch_scale_f64(bc, scale, n, s));
    st = read_status(dst, &h, s);
    stats_record(h, plan.grid, plan.block, where, 0.0f);
    return st;
}

}  // extern "C"
