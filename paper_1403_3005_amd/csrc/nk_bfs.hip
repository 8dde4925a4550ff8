// Grid-wide breadth-first search and restricted component labelling for the
// vertex-diameter bound of pair sampling.
//
// The bound (double sweep from the highest-degree vertex plus the largest
// other component; used for the Riondato-Kornaropoulos sample size the
// paper cites for its epsilon guarantee) needs two plain BFS distances and
// component sizes, once per call.  Each BFS level here runs over the whole
// GPU, top-down balanced over the frontier's arcs (so a hub's arcs spread
// over every workgroup) or bottom-up over the unreached vertices; new
// vertices are staged in LDS and leave with one global atomic per
// workgroup tile, since same-address atomics serialise.  The host reads the
// new level's size after each level to pick the direction and to stop.  Components are labelled only among the
// vertices the first sweep did not reach, so the giant component never
// becomes a contended label.
#include <hipcub/hipcub.hpp>

#include "nk_runtime.h"

namespace nk {

namespace {

constexpr int kBfsBlock = 256;
constexpr int kTdPer = 8;                        // arcs per thread per top-down tile
constexpr int kTdTile = kBfsBlock * kTdPer;      // arcs per top-down tile
constexpr int kBuStage = 4 * kBfsBlock;          // LDS staging of bottom-up appends
constexpr int32_t kBuCap = 256;                  // arcs a thread scans before handing a vertex to a wave

// Counter set of one level (four 8-byte words): new-vertex count (int),
// arcs of the new vertices (u64), deferred count (int), spare.  Level L
// uses set L & 1 and clears the other set for level L + 1, so no level
// needs a separate clearing launch.
struct LevelCounters {
    int32_t *newc;
    unsigned long long *arcs;
    int32_t *ndef;
};
__device__ __forceinline__ LevelCounters counters(long long *set) {
    return {reinterpret_cast<int32_t *>(set), reinterpret_cast<unsigned long long *>(set + 1),
            reinterpret_cast<int32_t *>(set + 2)};
}

__global__ void k_gbfs_init(int32_t *d, int32_t n, int32_t src, int32_t *front, long long *set0) {
    const long long stride = (long long)gridDim.x * blockDim.x;
    for (long long v = (long long)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += stride)
        d[v] = (v == src) ? 0 : -1;
    if (blockIdx.x == 0 && threadIdx.x < 4) set0[threadIdx.x] = 0;
    if (blockIdx.x == 0 && threadIdx.x == 0) front[0] = src;
}

// Appends `val` of every lane with `pred` to an LDS list, one LDS atomic
// per wave.
__device__ __forceinline__ void lds_push(bool pred, int32_t val, int32_t *buf, int32_t *count) {
    const unsigned long long mask = __ballot(pred);
    if (!mask) return;
    const int lane = lane_id();
    const int leader = __ffsll((long long)mask) - 1;
    int32_t pos = 0;
    if (lane == leader) pos = atomicAdd(count, (int32_t)__popcll(mask));
    pos = __shfl(pos, leader, kWave);
    if (pred) buf[pos + (int32_t)__popcll(mask & ((1ULL << lane) - 1ULL))] = val;
}

// Adds the block's sum of v to *out with one global atomic; all threads
// must call it (it holds two barriers).
__device__ __forceinline__ void block_add(unsigned long long v, unsigned long long *part, unsigned long long *out) {
    v = wave_sum<unsigned long long>(v);
    if (lane_id() == 0) part[wave_id()] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long t = 0;
        for (int w = 0; w < kBfsBlock / kWave; ++w) t += part[w];
        if (t) atomicAdd(out, t);
    }
    __syncthreads();
}

// Largest i in [0, count) with off[i] <= x (off[0] = 0 <= x).
__device__ __forceinline__ int32_t last_le(const int32_t *off, int32_t count, int32_t x) {
    int32_t lo = 0, hi = count - 1;
    while (lo < hi) {
        const int32_t mid = (lo + hi + 1) >> 1;
        if (off[mid] <= x) lo = mid; else hi = mid - 1;
    }
    return lo;
}

// Degrees of the frontier, deg[nf] = 0, for the arc offsets of a top-down
// level.
__global__ void k_front_deg(const int32_t *rowptr, const int32_t *front, int32_t nf, int32_t *deg) {
    const long long stride = (long long)gridDim.x * blockDim.x;
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i <= nf; i += stride)
        deg[i] = i < nf ? rowptr[front[i] + 1] - rowptr[front[i]] : 0;
}

// Top-down level, balanced over arcs: the frontier's arcs are numbered
// 0 .. total-1 by the offsets off[] (exclusive prefix sums of the frontier
// degrees) and every workgroup takes tiles of kTdTile consecutive arcs, so
// a hub's arcs spread over the grid.  A thread finds its arc's frontier
// vertex by binary search over the tile's offsets (staged in LDS), claims
// an unreached head with a compare-and-swap on its distance and stages it
// in LDS; the tile's new vertices go out with one global atomic.
__global__ __launch_bounds__(kBfsBlock) void k_gbfs_td(const int32_t *rowptr, const int32_t *colidx, int32_t *d,
                                                       const int32_t *front, const int32_t *off, int32_t nf,
                                                       int32_t level, int32_t *next, long long *set,
                                                       long long *other) {
    __shared__ int32_t s_off[kTdTile + 1];
    __shared__ int32_t s_arc[kTdTile + 1];
    __shared__ int32_t s_buf[kTdTile];
    __shared__ int32_t s_i0, s_n, s_cnt, s_base;
    __shared__ unsigned long long s_part[kBfsBlock / kWave];
    const LevelCounters c = counters(set);
    const int tid = threadIdx.x;
    if (blockIdx.x == 0 && tid < 4) other[tid] = 0;
    const int32_t total = off[nf];   // the frontier's arcs
    for (long long t0 = (long long)blockIdx.x * kTdTile; t0 < total; t0 += (long long)gridDim.x * kTdTile) {
        const int32_t e0 = (int32_t)t0;
        const int32_t e1 = (int32_t)(t0 + kTdTile < total ? t0 + kTdTile : total);
        if (tid == 0) {
            const int32_t i0 = last_le(off, nf, e0);
            s_i0 = i0;
            s_n = last_le(off, nf, e1 - 1) - i0 + 1;
            s_cnt = 0;
        }
        __syncthreads();
        const int32_t i0 = s_i0, ns = s_n;
        // zero-degree frontier vertices (possible only in an asymmetric
        // graph) can make the covered range longer than the tile: then the
        // search runs on global memory
        const bool fits = ns <= kTdTile + 1;
        if (fits)
            for (int k = tid; k < ns; k += kBfsBlock) {
                s_off[k] = off[i0 + k];
                s_arc[k] = rowptr[front[i0 + k]];
            }
        __syncthreads();
        for (int q = 0; q < kTdPer; ++q) {
            const int32_t e = e0 + q * kBfsBlock + tid;
            bool fresh = false;
            int32_t z = 0;
            if (e < e1) {
                int32_t lo = 0, hi = ns - 1;
                while (lo < hi) {
                    const int32_t mid = (lo + hi + 1) >> 1;
                    if ((fits ? s_off[mid] : off[i0 + mid]) <= e) lo = mid; else hi = mid - 1;
                }
                const int32_t first = fits ? s_arc[lo] : rowptr[front[i0 + lo]];
                z = colidx[first + (e - (fits ? s_off[lo] : off[i0 + lo]))];
                if (d[z] < 0) fresh = atomicCAS(&d[z], -1, level + 1) == -1;
            }
            lds_push(fresh, z, s_buf, &s_cnt);
        }
        __syncthreads();
        const int32_t nb = s_cnt;
        if (tid == 0 && nb > 0) s_base = atomicAdd(c.newc, nb);
        __syncthreads();
        unsigned long long dg = 0;
        for (int k = tid; k < nb; k += kBfsBlock) {
            const int32_t z = s_buf[k];
            next[s_base + k] = z;
            dg += (unsigned long long)(rowptr[z + 1] - rowptr[z]);
        }
        block_add(dg, s_part, c.arcs);
    }
}

// Writes the staged bottom-up appends with one global atomic per list.
__device__ __forceinline__ void bu_flush(int32_t *s_next, int32_t *s_def, int32_t &s_nn, int32_t &s_nd,
                                         int32_t &s_bn, int32_t &s_bd, int32_t *next, int32_t *defer,
                                         const LevelCounters &c) {
    const int tid = threadIdx.x;
    const int32_t nn = s_nn, nd = s_nd;
    if (tid == 0) {
        s_bn = nn > 0 ? atomicAdd(c.newc, nn) : 0;
        s_bd = nd > 0 ? atomicAdd(c.ndef, nd) : 0;
    }
    __syncthreads();
    for (int k = tid; k < nn; k += kBfsBlock) next[s_bn + k] = s_next[k];
    for (int k = tid; k < nd; k += kBfsBlock) defer[s_bd + k] = s_def[k];
    __syncthreads();
    if (tid == 0) {
        s_nn = 0;
        s_nd = 0;
    }
    __syncthreads();
}

// Bottom-up step: every unreached vertex looks for a neighbour on `level`
// among its first kBuCap arcs and stops at the first; vertices with more
// arcs that found none yet go to `defer` for k_gbfs_bu_wide.  Workgroups
// stride over the vertices 256 at a time and stage both lists in LDS.
__global__ __launch_bounds__(kBfsBlock) void k_gbfs_bu(const int32_t *rowptr, const int32_t *colidx, int32_t *d,
                                                       int32_t n, int32_t level, int32_t *next, int32_t *defer,
                                                       long long *set, long long *other) {
    __shared__ int32_t s_next[kBuStage], s_def[kBuStage];
    __shared__ int32_t s_nn, s_nd, s_bn, s_bd;
    __shared__ unsigned long long s_part[kBfsBlock / kWave];
    const LevelCounters c = counters(set);
    const int tid = threadIdx.x;
    if (blockIdx.x == 0 && tid < 4) other[tid] = 0;
    if (tid == 0) {
        s_nn = 0;
        s_nd = 0;
    }
    __syncthreads();
    unsigned long long dsum = 0;
    for (long long v0 = (long long)blockIdx.x * kBfsBlock; v0 < n; v0 += (long long)gridDim.x * kBfsBlock) {
        const long long v = v0 + tid;
        bool found = false, later = false;
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
                dsum += (unsigned long long)(a1 - a0);
            } else {
                later = stop < a1;
            }
        }
        lds_push(found, (int32_t)v, s_next, &s_nn);
        lds_push(later, (int32_t)v, s_def, &s_nd);
        __syncthreads();
        if (s_nn > kBuStage - kBfsBlock || s_nd > kBuStage - kBfsBlock)
            bu_flush(s_next, s_def, s_nn, s_nd, s_bn, s_bd, next, defer, c);
    }
    bu_flush(s_next, s_def, s_nn, s_nd, s_bn, s_bd, next, defer, c);
    block_add(dsum, s_part, c.arcs);
}

// The rest of the arcs of deferred vertices, one wave per vertex.
__global__ void k_gbfs_bu_wide(const int32_t *rowptr, const int32_t *colidx, int32_t *d, const int32_t *defer,
                               int32_t level, int32_t *next, long long *set) {
    const LevelCounters c = counters(set);
    const int lane = lane_id();
    const int32_t nd = *c.ndef;
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
            const int32_t pos = atomicAdd(c.newc, 1);
            next[pos] = v;
            atomicAdd(c.arcs, (unsigned long long)(a1 - rowptr[v]));
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

nk_status bfs_work_get(Scratch &scr, int32_t n, hipStream_t s, BfsWork *w) {
    nk_status st;
    if ((st = scr.get(n, &w->d)) != NK_OK) return st;
    if ((st = scr.get(n, &w->f0)) != NK_OK) return st;
    if ((st = scr.get(n, &w->f1)) != NK_OK) return st;
    if ((st = scr.get((long long)n + 1, &w->f2)) != NK_OK) return st;
    if ((st = scr.get((long long)n + 1, &w->off)) != NK_OK) return st;
    if ((st = scr.get(9, &w->cnt)) != NK_OK) return st;
    w->tmp_bytes = 0;
    NK_HIP(hipcub::DeviceScan::ExclusiveSum(nullptr, w->tmp_bytes, w->f2, w->off, n + 1, s));
    if ((st = scr.get(w->tmp_bytes > 0 ? w->tmp_bytes : 1, &w->tmp)) != NK_OK) return st;
    return NK_OK;
}

nk_status grid_bfs(const int32_t *rowptr, const int32_t *colidx, int32_t n, int64_t m, int32_t src,
                   const BfsWork &w, hipStream_t s, int32_t out[3], int32_t src_deg, bool want_lowest) {
    int32_t *d = w.d;
    int32_t *low = reinterpret_cast<int32_t *>(w.cnt + 8);
    hipLaunchKernelGGL(k_gbfs_init, dim3(grid_of(n, 256)), dim3(256), 0, s, d, n, src, w.f0, w.cnt);
    NK_HIP(hipGetLastError());
    int32_t nf = 1, level = 0, reached = 1;
    int32_t *front = w.f0, *next = w.f1;
    if (src_deg < 0) {
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
    const unsigned bu_grid = grid_of(n, kBfsBlock) < 2048 ? grid_of(n, kBfsBlock) : 2048;
    for (;;) {
        long long *set = w.cnt + 4 * (level & 1), *other = w.cnt + 4 * ((level + 1) & 1);
        if (!bu && (double)mf * 14.0 > (double)mu) bu = true;
        else if (bu && (long long)nf * 24 < n) bu = false;
        if (bu) {
            hipLaunchKernelGGL(k_gbfs_bu, dim3(bu_grid), dim3(kBfsBlock), 0, s, rowptr, colidx, d, n, level, next,
                               w.f2, set, other);
            NK_HIP(hipGetLastError());
            hipLaunchKernelGGL(k_gbfs_bu_wide, dim3(1024), dim3(256), 0, s, rowptr, colidx, d, w.f2, level, next,
                               set);
            NK_HIP(hipGetLastError());
        } else if (mf > 0) {
            // arc offsets of the frontier, then the arc-balanced level
            hipLaunchKernelGGL(k_front_deg, dim3(grid_of((long long)nf + 1, 256)), dim3(256), 0, s, rowptr, front, nf,
                               w.f2);
            NK_HIP(hipGetLastError());
            size_t tb = 0;
            NK_HIP(hipcub::DeviceScan::ExclusiveSum(nullptr, tb, w.f2, w.off, nf + 1, s));
            if (tb > w.tmp_bytes) return fail(NK_E_INTERNAL, "prefix-sum storage too small");
            NK_HIP(hipcub::DeviceScan::ExclusiveSum(w.tmp, tb, w.f2, w.off, nf + 1, s));
            const long long tiles = (mf + kTdTile - 1) / kTdTile;
            hipLaunchKernelGGL(k_gbfs_td, dim3((unsigned)(tiles < 8192 ? tiles : 8192)), dim3(kBfsBlock), 0, s,
                               rowptr, colidx, d, front, w.off, nf, level, next, set, other);
            NK_HIP(hipGetLastError());
        }
        // (a top-down level without arcs finds nothing: its set is still clear)
        NK_HIP(hipMemcpyAsync(&h, set, 16, hipMemcpyDeviceToHost, s));
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
    out[0] = level;
    out[1] = -1;
    out[2] = reached;
    if (!want_lowest) return NK_OK;
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
