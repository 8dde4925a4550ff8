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
                             int32_t nf, int32_t level, int32_t *next, int32_t *cnt) {
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
            }
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

nk_status grid_bfs(const int32_t *rowptr, const int32_t *colidx, int32_t n, int32_t src, int32_t *d,
                   int32_t *f0, int32_t *f1, int32_t *cnt, hipStream_t s, int32_t out[3]) {
    hipLaunchKernelGGL(k_gbfs_init, dim3(grid_of(n, 256)), dim3(256), 0, s, d, n, src, f0, cnt);
    NK_HIP(hipGetLastError());
    int32_t nf = 1, level = 0, reached = 1;
    int32_t *front = f0, *next = f1;
    int32_t h = 0;
    for (;;) {
        // one wave per frontier vertex, 4 waves per workgroup
        hipLaunchKernelGGL(k_gbfs_level, dim3(grid_of((long long)nf * kWave, 256)), dim3(256), 0, s, rowptr, colidx,
                           d, front, nf, level, next, cnt);
        NK_HIP(hipGetLastError());
        NK_HIP(hipMemcpyAsync(&h, cnt, 4, hipMemcpyDeviceToHost, s));
        NK_HIP(hipStreamSynchronize(s));
        if (h <= 0 || h > n) break;
        reached += h;
        NK_HIP(launch_fill_i32(cnt, 0, 1, s));
        int32_t *t = front;
        front = next;
        next = t;
        nf = h;
        ++level;
    }
    if (h > n) return fail(NK_E_INTERNAL, "breadth-first search overran its frontier");
    // lowest id on the deepest level (front[0, nf))
    NK_HIP(launch_fill_i32(cnt + 1, 0x7fffffff, 1, s));
    hipLaunchKernelGGL(k_min_i32, dim3(grid_of(nf, 256)), dim3(256), 0, s, front, nf, cnt + 1);
    NK_HIP(hipGetLastError());
    int32_t lowest = 0;
    NK_HIP(hipMemcpyAsync(&lowest, cnt + 1, 4, hipMemcpyDeviceToHost, s));
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
