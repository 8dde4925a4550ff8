// Grid-wide breadth-first search and restricted component labelling for the
// vertex-diameter bound of pair sampling.
//
// The bound (double sweep from the highest-degree vertex plus the largest
// other component; used for the Riondato-Kornaropoulos sample size the
// paper cites for its epsilon guarantee) needs two plain BFS distances and
// component sizes, once per call.  Each BFS level here is one launch over
// the whole GPU: one wave per frontier vertex scans its arcs 64 at a time,
// claims unreached neighbours with a compare-and-swap on the distance and
// appends them with one atomic per wave.  The host reads the new level's
// size after each launch to stop.  Components are labelled only among the
// vertices the first sweep did not reach, so the giant component never
// becomes a contended label.
#include "nk_runtime.h"

namespace nk {

namespace {

__global__ void k_gbfs_init(int32_t *d, int32_t n, int32_t src, int32_t *front, int32_t *cnt) {
    const long long stride = (long long)gridDim.x * blockDim.x;
    for (long long v = (long long)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += stride)
        d[v] = (v == src) ? 0 : -1;
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        front[0] = src;
        cnt[0] = 0;
    }
}

// Expands level `level` (front[0, nf)) into next[]; cnt[0] counts the new
// vertices.
__global__ void k_gbfs_level(const int32_t *rowptr, const int32_t *colidx, int32_t *d, const int32_t *front,
                             int32_t nf, int32_t level, int32_t *next, int32_t *cnt, unsigned long long *arcs) {
    const int lane = lane_id();
    const long long waves = (long long)gridDim.x * (blockDim.x / kWave);
    for (long long i = (long long)blockIdx.x * (blockDim.x / kWave) + wave_id(); i < nf; i += waves) {
        const int32_t v = front[i];
        const int32_t a1 = rowptr[v + 1];
        for (int32_t base = rowptr[v]; base < a1; base += kWave) {
            const int32_t e = base + lane;
            bool fresh = false;
            int32_t z = 0;
            if (e < a1) {
                z = colidx[e];
                if (d[z] < 0) fresh = atomicCAS(&d[z], -1, level + 1) == -1;
            }
            const unsigned long long mask = __ballot(fresh);
            if (mask) {
                const int leader = __ffsll((long long)mask) - 1;
                int32_t pos = 0;
                if (lane == leader) pos = atomicAdd(cnt, (int32_t)__popcll(mask));
                pos = __shfl(pos, leader, kWave);
                if (fresh) next[pos + (int32_t)__popcll(mask & ((1ULL << lane) - 1ULL))] = z;
                unsigned long long dg = fresh ? (unsigned long long)(rowptr[z + 1] - rowptr[z]) : 0ULL;
                dg = wave_sum<unsigned long long>(dg);
                if (lane == 0) atomicAdd(arcs, dg);
            }
        }
    }
}

// Appends `take` (one flag per lane) to list with one atomic per wave.
__device__ __forceinline__ void wave_push(bool take, int32_t x, int32_t *list, int32_t *count) {
    const unsigned long long mask = __ballot(take);
    if (!mask) return;
    const int lane = lane_id();
    const int leader = __ffsll((long long)mask) - 1;
    int32_t pos = 0;
    if (lane == leader) pos = atomicAdd(count, (int32_t)__popcll(mask));
    pos = __shfl(pos, leader, kWave);
    if (take) list[pos + (int32_t)__popcll(mask & ((1ULL << lane) - 1ULL))] = x;
}

constexpr int32_t kBuCap = 256;  // arcs a thread scans before handing a vertex to a wave

// Bottom-up step: every unreached vertex looks for a neighbour on `level`
// among its first kBuCap arcs and stops at the first; vertices with more
// arcs that found none yet go to `defer` for k_gbfs_bu_wide.
__global__ void k_gbfs_bu(const int32_t *rowptr, const int32_t *colidx, int32_t *d, int32_t n, int32_t level,
                          int32_t *next, int32_t *cnt, unsigned long long *arcs, int32_t *defer, int32_t *ndefer) {
    const long long stride = (long long)gridDim.x * blockDim.x;
    const long long start = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const long long rounds = ((long long)n + stride - 1) / stride;
    for (long long r = 0; r < rounds; ++r) {
        const long long v = start + r * stride;
        bool found = false, later = false;
        unsigned long long dg = 0;
        if (v < n && d[v] < 0) {
            const int32_t a0 = rowptr[v], a1 = rowptr[v + 1];
            const int32_t stop = a1 - a0 > kBuCap ? a0 + kBuCap : a1;
            for (int32_t e = a0; e < stop; ++e)
                if (d[colidx[e]] == level) {
                    found = true;
                    break;
                }
            if (found) {
                d[v] = level + 1;
                dg = (unsigned long long)(a1 - a0);
            } else {
                later = stop < a1;
            }
        }
        wave_push(found, (int32_t)v, next, cnt);
        wave_push(later, (int32_t)v, defer, ndefer);
        dg = wave_sum<unsigned long long>(dg);
        if (lane_id() == 0 && dg) atomicAdd(arcs, dg);
    }
}

// The rest of the arcs of deferred vertices, one wave per vertex.
__global__ void k_gbfs_bu_wide(const int32_t *rowptr, const int32_t *colidx, int32_t *d, const int32_t *defer,
                               const int32_t *ndefer, int32_t level, int32_t *next, int32_t *cnt,
                               unsigned long long *arcs) {
    const int lane = lane_id();
    const int32_t nd = *ndefer;
    const long long waves = (long long)gridDim.x * (blockDim.x / kWave);
    for (long long i = (long long)blockIdx.x * (blockDim.x / kWave) + wave_id(); i < nd; i += waves) {
        const int32_t v = defer[i];
        const int32_t a1 = rowptr[v + 1];
        bool found = false;
        for (int32_t base = rowptr[v] + kBuCap; base < a1 && !found; base += kWave) {
            const int32_t e = base + lane;
            found = __ballot(e < a1 && d[colidx[e]] == level) != 0ULL;
        }
        if (found && lane == 0) {
            d[v] = level + 1;
            const int32_t pos = atomicAdd(cnt, 1);
            next[pos] = v;
            atomicAdd(arcs, (unsigned long long)(a1 - rowptr[v]));
        }
    }
}

__global__ void k_min_i32(const int32_t *x, int32_t count, int32_t *out) {
    const long long stride = (long long)gridDim.x * blockDim.x;
    int32_t best = 0x7fffffff;
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += stride) best = min(best, x[i]);
    best = wave_min(best);
    if (lane_id() == 0) atomicMin(out, best);
}

// Component labelling among vertices with skip[v] >= 0 left out (the first
// sweep's distances): minimum-label hooking with pointer jumping.
__global__ void k_rcc_init(const int32_t *skip, int32_t *label, int32_t n) {
    const long long stride = (long long)gridDim.x * blockDim.x;
    for (long long v = (long long)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += stride)
        label[v] = skip[v] >= 0 ? -1 : (int32_t)v;
}

__global__ void k_rcc_hook(const int32_t *rowptr, const int32_t *colidx, const int32_t *skip, int32_t n,
                           int32_t *label, int32_t *changed) {
    const long long stride = (long long)gridDim.x * blockDim.x;
    int ch = 0;
    for (long long u = (long long)blockIdx.x * blockDim.x + threadIdx.x; u < n; u += stride) {
        if (skip[u] >= 0) continue;
        const int32_t lu = label[u];
        for (int32_t e = rowptr[u]; e < rowptr[u + 1]; ++e) {
            const int32_t lv = label[colidx[e]];   // a neighbour of an unreached vertex is unreached
            if (lu < lv) {
                atomicMin(&label[lv], lu);
                ch = 1;
            }
        }
    }
    if (ch) atomicOr(changed, 1);
}

__global__ void k_rcc_compress(int32_t *label, int32_t n) {
    const long long stride = (long long)gridDim.x * blockDim.x;
    for (long long v = (long long)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += stride) {
        int32_t l = label[v];
        if (l < 0) continue;
        while (label[l] != l) l = label[l];
        label[v] = l;
    }
}

// size[root] = vertices per component; lanes sharing lane 0's label add once.
__global__ void k_rcc_sizes(const int32_t *label, int32_t n, int32_t *size) {
    const long long stride = (long long)gridDim.x * blockDim.x;
    const long long start = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const long long rounds = ((long long)n + stride - 1) / stride;
    for (long long r = 0; r < rounds; ++r) {
        const long long v = start + r * stride;
        const int32_t l = v < n ? label[v] : -1;
        const int32_t l0 = __shfl(l, 0, kWave);
        const unsigned long long same = __ballot(l >= 0 && l == l0);
        if (lane_id() == 0 && same) atomicAdd(&size[l0], (int32_t)__popcll(same));
        if (l >= 0 && l != l0) atomicAdd(&size[l], 1);
    }
}

__global__ void k_rcc_max(const int32_t *label, const int32_t *size, int32_t n, int32_t *out) {
    const long long stride = (long long)gridDim.x * blockDim.x;
    int32_t best = 0;
    for (long long v = (long long)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += stride)
        if (label[v] == (int32_t)v) best = max(best, size[v]);
    if (best) atomicMax(out, best);
}

unsigned grid_of(long long count, int block) {
    long long g = (count + block - 1) / block;
    if (g < 1) g = 1;
    if (g > 65536) g = 65536;
    return (unsigned)g;
}

}  // namespace

nk_status grid_bfs(const int32_t *rowptr, const int32_t *colidx, int32_t n, int64_t m, int32_t src, int32_t *d,
                   int32_t *f0, int32_t *f1, int32_t *f2, long long *cnt, hipStream_t s, int32_t out[3]) {
    // cnt: [0] new-vertex count (int), [1] arcs of the new vertices (u64),
    //      [2] deferred count (int), [3] lowest id (int)
    int32_t *newc = reinterpret_cast<int32_t *>(cnt);
    unsigned long long *arcs = reinterpret_cast<unsigned long long *>(cnt + 1);
    int32_t *ndef = reinterpret_cast<int32_t *>(cnt + 2);
    int32_t *low = reinterpret_cast<int32_t *>(cnt + 3);
    hipLaunchKernelGGL(k_gbfs_init, dim3(grid_of(n, 256)), dim3(256), 0, s, d, n, src, f0, newc);
    NK_HIP(hipGetLastError());
    int32_t nf = 1, level = 0, reached = 1;
    int32_t *front = f0, *next = f1;
    int32_t src_deg = 0;
    {
        int32_t rp2[2];
        NK_HIP(hipMemcpyAsync(rp2, rowptr + src, 8, hipMemcpyDeviceToHost, s));
        NK_HIP(hipStreamSynchronize(s));
        src_deg = rp2[1] - rp2[0];
    }
    // Direction rule (Beamer et al.): bottom-up while the frontier's arcs
    // exceed 1/14 of the unreached vertices' arcs and the frontier holds more
    // than n/24 vertices; top-down otherwise.
    long long mf = src_deg, mu = m - src_deg;
    bool bu = false;
    struct {
        int32_t newc, pad;
        unsigned long long arcs;
    } h;
    for (;;) {
        NK_HIP(launch_fill_u64(reinterpret_cast<unsigned long long *>(cnt), 0ULL, 3, s));
        if (!bu && (double)mf * 14.0 > (double)mu) bu = true;
        else if (bu && (long long)nf * 24 < n) bu = false;
        if (bu) {
            hipLaunchKernelGGL(k_gbfs_bu, dim3(grid_of(n, 256)), dim3(256), 0, s, rowptr, colidx, d, n, level, next,
                               newc, arcs, f2, ndef);
            NK_HIP(hipGetLastError());
            hipLaunchKernelGGL(k_gbfs_bu_wide, dim3(1024), dim3(256), 0, s, rowptr, colidx, d, f2, ndef, level, next,
                               newc, arcs);
            NK_HIP(hipGetLastError());
        } else {
            // one wave per frontier vertex, 4 waves per workgroup
            hipLaunchKernelGGL(k_gbfs_level, dim3(grid_of((long long)nf * kWave, 256)), dim3(256), 0, s, rowptr,
                               colidx, d, front, nf, level, next, newc, arcs);
            NK_HIP(hipGetLastError());
        }
        NK_HIP(hipMemcpyAsync(&h, cnt, 16, hipMemcpyDeviceToHost, s));
        NK_HIP(hipStreamSynchronize(s));
        if (h.newc <= 0 || h.newc > n) break;
        reached += h.newc;
        mf = (long long)h.arcs;
        mu -= mf;
        int32_t *t = front;
        front = next;
        next = t;
        nf = h.newc;
        ++level;
    }
    if (h.newc > n) return fail(NK_E_INTERNAL, "breadth-first search overran its frontier");
    // lowest id on the deepest level (front[0, nf))
    NK_HIP(launch_fill_i32(low, 0x7fffffff, 1, s));
    hipLaunchKernelGGL(k_min_i32, dim3(grid_of(nf, 256)), dim3(256), 0, s, front, nf, low);
    NK_HIP(hipGetLastError());
    int32_t lowest = 0;
    NK_HIP(hipMemcpyAsync(&lowest, low, 4, hipMemcpyDeviceToHost, s));
    NK_HIP(hipStreamSynchronize(s));
    out[0] = level;
    out[1] = lowest;
    out[2] = reached;
    return NK_OK;
}

nk_status largest_unreached_component(const int32_t *rowptr, const int32_t *colidx, int32_t n, const int32_t *skip,
                                      int32_t *label, int32_t *size, int32_t *flag, hipStream_t s, int32_t *out) {
    hipLaunchKernelGGL(k_rcc_init, dim3(grid_of(n, 256)), dim3(256), 0, s, skip, label, n);
    NK_HIP(hipGetLastError());
    int32_t h = 1;
    for (int it = 0; h && it < 100000; ++it) {
        NK_HIP(launch_fill_i32(flag, 0, 1, s));
        hipLaunchKernelGGL(k_rcc_hook, dim3(grid_of(n, 256)), dim3(256), 0, s, rowptr, colidx, skip, n, label, flag);
        NK_HIP(hipGetLastError());
        hipLaunchKernelGGL(k_rcc_compress, dim3(grid_of(n, 256)), dim3(256), 0, s, label, n);
        NK_HIP(hipGetLastError());
        NK_HIP(hipMemcpyAsync(&h, flag, 4, hipMemcpyDeviceToHost, s));
        NK_HIP(hipStreamSynchronize(s));
    }
    if (h) return fail(NK_E_INTERNAL, "component labelling did not converge");
    NK_HIP(launch_fill_i32(size, 0, n, s));
    hipLaunchKernelGGL(k_rcc_sizes, dim3(grid_of(n, 256)), dim3(256), 0, s, label, n, size);
    NK_HIP(hipGetLastError());
    NK_HIP(launch_fill_i32(flag, 0, 1, s));
    hipLaunchKernelGGL(k_rcc_max, dim3(grid_of(n, 256)), dim3(256), 0, s, label, size, n, flag);
    NK_HIP(hipGetLastError());
    NK_HIP(hipMemcpyAsync(out, flag, 4, hipMemcpyDeviceToHost, s));
    NK_HIP(hipStreamSynchronize(s));
    return NK_OK;
}

}  // namespace nk
