// All-in-LDS Brandes kernel for small graphs.
//
// When a graph's CSR and one source's state fit in a workgroup's 160 KB of
// LDS, a persistent workgroup copies the graph into LDS once and then runs
// whole sources out of LDS: the forward path-counting search and the
// backward dependency sweep of Brandes' algorithm (the betweenness method
// the paper relies on, "Heuristics and Approximation Algorithms" and
// Table 1) touch global memory only to add each vertex's dependency into
// bc.  A level costs a few LDS round trips instead of a few HBM round
// trips, which is what bounds the global kernel on graphs of a few
// thousand vertices.
//
// Tasks are (graph, source) pairs, drawn from one dynamic counter, for a
// single graph or for a batch of concatenated graphs; a workgroup reloads
// the CSR only when its next task belongs to another graph.
//
// LDS layout (dynamic part, bytes, n vertices, m arcs):
//   sig  u64[n]     sigma during the forward phase, coef = (1 + delta) /
//                   sigma (FP64 bits) once a vertex's level is swept
//   rp   i32[n+1]   row pointers
//   ci   i32[m]     column indices
//   lv   i32[n]     concatenated level lists (visit order)
//   lvl  i32[n+2]   level offsets into lv
//   bm   u32[ceil(n/32)] visited bitmap
// Both phases run level-synchronously over LDS tiles of up to BLOCK listed
// vertices with an exclusive prefix of degrees, exactly as in the global
// kernel: the forward phase is always top-down (an LDS 64-bit atomic add
// into sigma of unmarked neighbours; the first adder appends the vertex),
// the backward phase is a pull over unmarked neighbours (levels are
// unmarked from the deepest up).
#include "nk_kernels.h"

namespace nk {

namespace {

constexpr int kLdsChunk = 4;

struct LdsGraph {
    unsigned long long *sig;
    int32_t *rp;
    int32_t *ci;
    int32_t *lv;
    int32_t *lvl;
    uint32_t *bm;
};

__device__ __forceinline__ LdsGraph lds_carve(unsigned long long *base, int32_t n, int32_t m) {
    LdsGraph L;
    char *p = reinterpret_cast<char *>(base);
    L.sig = reinterpret_cast<unsigned long long *>(p);
    p += 8 * (size_t)n;
    L.rp = reinterpret_cast<int32_t *>(p);
    p += 4 * ((size_t)n + 1);
    L.ci = reinterpret_cast<int32_t *>(p);
    p += 4 * (size_t)m;
    L.lv = reinterpret_cast<int32_t *>(p);
    p += 4 * (size_t)n;
    L.lvl = reinterpret_cast<int32_t *>(p);
    p += 4 * ((size_t)n + 2);
    L.bm = reinterpret_cast<uint32_t *>(p);
    return L;
}

__device__ __forceinline__ bool lbit(const uint32_t *bm, int32_t v) { return (bm[v >> 5] >> (v & 31)) & 1u; }
__device__ __forceinline__ double lf64(unsigned long long x) { return __longlong_as_double((long long)x); }
__device__ __forceinline__ unsigned long long lu64(double x) { return (unsigned long long)__double_as_longlong(x); }

struct LdsCounters {
    unsigned long long arcs_fwd, arcs_bwd, dag, reached, tasks, levels, arcs_reached;
};

// Stages list entries lv[tb, tb+cnt) into the tile (vertex, first arc,
// degree prefix) and returns the tile's arc count.  Contains barriers.
template <int BLOCK>
__device__ __forceinline__ int32_t lds_stage(Tile<BLOCK> &sm, const LdsGraph &L, int32_t tb, int32_t cnt) {
    const int tid = threadIdx.x;
    int32_t dg = 0;
    if (tid < cnt) {
        const int32_t v = L.lv[tb + tid];
        const int32_t a0 = L.rp[v];
        dg = L.rp[v + 1] - a0;
        sm.v[tid] = v;
        sm.a0[tid] = a0;
    }
    int32_t total;
    const int32_t ex = block_excl_scan<BLOCK>(dg, sm, total);
    if (tid < cnt) sm.pre[tid] = ex;
    if (tid == 0) sm.pre[cnt] = total;
    __syncthreads();
    return total;
}

// Column indices of the thread's chunk [i0, i0 + kLdsChunk) of the tile's
// arcs; kk[j] = tile row of arc j, or -1 past the end.
template <int BLOCK>
__device__ __forceinline__ void lds_chunk(const Tile<BLOCK> &sm, const LdsGraph &L, int32_t cnt, int32_t total,
                                          int32_t i0, int32_t (&kk)[kLdsChunk], int32_t (&w)[kLdsChunk]) {
    int32_t k = (i0 < total) ? tile_search(sm.pre, cnt, i0) : 0;
#pragma unroll
    for (int j = 0; j < kLdsChunk; ++j) {
        const int32_t i = i0 + j;
        kk[j] = -1;
        w[j] = 0;
        if (i < total) {
            while (sm.pre[k + 1] <= i) ++k;
            kk[j] = k;
        }
    }
#pragma unroll
    for (int j = 0; j < kLdsChunk; ++j)
        if (kk[j] >= 0) w[j] = L.ci[sm.a0[kk[j]] + (i0 + j - sm.pre[kk[j]])];
}

// One source: forward (top-down, LDS atomics) then the backward pull.
template <int BLOCK>
__device__ void lds_source(const Params &p, Tile<BLOCK> &sm, const LdsGraph &L, int32_t n, int32_t src,
                           double *bcg, LdsCounters &c) {
    const int tid = threadIdx.x;
    const int32_t nw = (n + 31) >> 5;
    for (int32_t v = tid; v < n; v += BLOCK) L.sig[v] = 0ULL;
    for (int32_t wi = tid; wi < nw; wi += BLOCK) {
        const int32_t hi = (wi + 1) * 32;
        L.bm[wi] = hi > n ? (~0u << (32 - (hi - n))) : 0u;  // padding bits beyond n stay marked
    }
    __syncthreads();
    if (tid == 0) {
        L.sig[src] = 1ULL;
        L.bm[src >> 5] |= 1u << (src & 31);
        L.lv[0] = src;
        L.lvl[0] = 0;
        L.lvl[1] = 1;
        c.arcs_reached += (unsigned long long)(L.rp[src + 1] - L.rp[src]);
    }
    __syncthreads();

    // ---- forward
    int32_t lvl = 0, f0 = 0, f1 = 1;
    for (;;) {
        if (tid == 0) sm.count = 0;
        __syncthreads();
        for (int32_t tb = f0; tb < f1; tb += BLOCK) {
            const int32_t cnt = min(BLOCK, f1 - tb);
            if (tid < cnt) sm.val.u[tid] = L.sig[L.lv[tb + tid]];
            const int32_t total = lds_stage<BLOCK>(sm, L, tb, cnt);
            if (tid == 0) c.arcs_fwd += (unsigned long long)total;
            for (int32_t rb = 0; rb < total; rb += BLOCK * kLdsChunk) {
                int32_t kk[kLdsChunk], w[kLdsChunk];
                lds_chunk<BLOCK>(sm, L, cnt, total, rb + tid * kLdsChunk, kk, w);
                // independent steps across the chunk so their LDS accesses overlap
                bool act[kLdsChunk];
                unsigned long long add[kLdsChunk], old[kLdsChunk];
#pragma unroll
                for (int j = 0; j < kLdsChunk; ++j) {
                    act[j] = kk[j] >= 0 && !lbit(L.bm, w[j]);
                    add[j] = act[j] ? sm.val.u[kk[j]] : 0ULL;
                }
#pragma unroll
                for (int j = 0; j < kLdsChunk; ++j) old[j] = act[j] ? atomicAdd(&L.sig[w[j]], add[j]) : 1ULL;
                unsigned long long fresh = 0;
#pragma unroll
                for (int j = 0; j < kLdsChunk; ++j) {
                    if (act[j]) {
                        c.dag++;
                        if (old[j] + add[j] < old[j]) atomicOr(&p.st->err, kErrOverflow);
                    }
                    fresh |= __ballot(act[j] && old[j] == 0ULL) != 0ULL ? (1ULL << j) : 0ULL;
                }
                if (fresh) {
#pragma unroll
                    for (int j = 0; j < kLdsChunk; ++j)
                        if (fresh & (1ULL << j))
                            wave_append(act[j] && old[j] == 0ULL, w[j], L.lv + f1, &sm.count, n - f1, &p.st->err);
                }
            }
            __syncthreads();
        }
        const int32_t nnew = sm.count < n - f1 ? sm.count : n - f1;
        long long dsum = 0;
        for (int32_t i = f1 + tid; i < f1 + nnew; i += BLOCK) {
            const int32_t w = L.lv[i];
            atomicOr(&L.bm[w >> 5], 1u << (w & 31));
            dsum += L.rp[w + 1] - L.rp[w];
        }
        dsum = wave_sum<long long>(dsum);
        if (lane_id() == 0) c.arcs_reached += (unsigned long long)dsum;
        if (tid == 0) {
            L.lvl[lvl + 2] = f1 + nnew;
            c.levels++;
        }
        __syncthreads();
        if (nnew == 0) break;
        f0 = f1;
        f1 += nnew;
        ++lvl;
    }
    if (tid == 0) {
        c.reached += (unsigned long long)f1;
        c.tasks++;
        atomicAdd(&p.st->stat[kStDone], 1ULL);
    }
    const int32_t Ld = lvl;
    if (Ld == 0) return;

    // ---- backward
    for (int32_t i = L.lvl[Ld] + tid; i < L.lvl[Ld + 1]; i += BLOCK) {
        const int32_t v = L.lv[i];
        L.sig[v] = lu64(1.0 / (double)L.sig[v]);
        atomicAnd(&L.bm[v >> 5], ~(1u << (v & 31)));
    }
    __syncthreads();
    for (int32_t l = Ld - 1; l >= 1; --l) {
        const int32_t lo = L.lvl[l], hi = L.lvl[l + 1];
        // linear scaling: pair weights d(s,v)/d(s,t) factor as l/(l+1) per DAG step
        const double wfac = p.linear ? (double)l / (double)(l + 1) : 1.0;
        for (int32_t tb = lo; tb < hi; tb += BLOCK) {
            const int32_t cnt = min(BLOCK, hi - tb);
            if (tid < cnt) sm.val.f[tid] = 0.0;
            const int32_t total = lds_stage<BLOCK>(sm, L, tb, cnt);
            if (tid == 0) c.arcs_bwd += (unsigned long long)total;
            for (int32_t rb = 0; rb < total; rb += BLOCK * kLdsChunk) {
                int32_t kk[kLdsChunk], w[kLdsChunk];
                lds_chunk<BLOCK>(sm, L, cnt, total, rb + tid * kLdsChunk, kk, w);
                double cf[kLdsChunk];
#pragma unroll
                for (int j = 0; j < kLdsChunk; ++j) cf[j] = (kk[j] >= 0 && !lbit(L.bm, w[j])) ? lf64(L.sig[w[j]]) : 0.0;
                int32_t kcur = kk[0];
                double acc = 0.0;
#pragma unroll
                for (int j = 0; j < kLdsChunk; ++j) {
                    if (kk[j] < 0) continue;
                    if (kk[j] != kcur) {
                        if (acc != 0.0) atomicAdd(&sm.val.f[kcur], acc);
                        kcur = kk[j];
                        acc = 0.0;
                    }
                    acc += cf[j];
                }
                if (acc != 0.0) atomicAdd(&sm.val.f[kcur], acc);
            }
            __syncthreads();
            if (tid < cnt) {
                const int32_t v = sm.v[tid];
                const double sg = (double)L.sig[v];
                const double delta = sg * sm.val.f[tid] * wfac;
                L.sig[v] = lu64((1.0 + delta) / sg);
                if (delta != 0.0) atomicAdd(bcg + v, delta);
            }
            __syncthreads();
        }
        for (int32_t i = lo + tid; i < hi; i += BLOCK) {
            const int32_t v = L.lv[i];
            atomicAnd(&L.bm[v >> 5], ~(1u << (v & 31)));
        }
        __syncthreads();
    }
}

template <int BLOCK>
__global__ __launch_bounds__(BLOCK) void k_brandes_lds(Params p) {
    extern __shared__ unsigned long long lds_dyn[];
    __shared__ Tile<BLOCK> sm;
    __shared__ int32_t loaded;  // graph id whose CSR is in LDS, -1 = none
    const int tid = threadIdx.x;
    if (tid == 0) {
        sm.flag = p.st->err & kErrGraph;
        loaded = -1;
    }
    __syncthreads();
    if (sm.flag) return;
    LdsCounters c = {0, 0, 0, 0, 0, 0, 0};
    for (;;) {
        if (tid == 0) sm.task = (long long)atomicAdd(&p.st->head, 1ULL);
        __syncthreads();
        const long long task = sm.task;
        __syncthreads();
        if (task >= p.ntasks) break;

        int32_t gid = 0, src = 0, n = p.n, m = p.m;
        const int32_t *rpg = p.rowptr, *cig = p.colidx;
        long long vbase = 0;
        if (p.G > 0) {
            int32_t lo = 0, hi = p.G - 1;
            while (lo < hi) {
                const int32_t mid = (lo + hi + 1) >> 1;
                if (p.g_task[mid] <= task) lo = mid; else hi = mid - 1;
            }
            gid = p.g_order[lo];
            vbase = p.g_vtx[gid];
            rpg = p.rowptr + vbase + gid;
            cig = p.colidx + p.g_arc[gid];
            n = (int32_t)(p.g_vtx[gid + 1] - vbase);
            m = (int32_t)(p.g_arc[gid + 1] - p.g_arc[gid]);
            src = (int32_t)(task - p.g_task[lo]);
        } else {
            src = p.sources ? p.sources[task] : (int32_t)task;
        }
        if (src < 0 || src >= n) {
            if (tid == 0) atomicOr(&p.st->err, kErrArg);
            continue;
        }
        const LdsGraph L = lds_carve(lds_dyn, n, m);
        if (gid != loaded) {
            for (int32_t i = tid; i <= n; i += BLOCK) L.rp[i] = rpg[i];
            for (int32_t i = tid; i < m; i += BLOCK) L.ci[i] = cig[i];
            __syncthreads();
            if (tid == 0) loaded = gid;
        }
        __syncthreads();
        lds_source<BLOCK>(p, sm, L, n, src, p.bc + vbase, c);
        __syncthreads();
    }
    const unsigned long long dag = wave_sum<unsigned long long>(c.dag);
    if (lane_id() == 0 && dag) atomicAdd(&p.st->stat[kStDag], dag);
    const unsigned long long ar = wave_sum<unsigned long long>(c.arcs_reached);
    if (lane_id() == 0 && ar) atomicAdd(&p.st->stat[kStArcsReached], ar);
    if (tid == 0) {
        atomicAdd(&p.st->stat[kStSources], c.tasks);
        atomicAdd(&p.st->stat[kStReached], c.reached);
        atomicAdd(&p.st->stat[kStArcsFwd], c.arcs_fwd);
        atomicAdd(&p.st->stat[kStArcsBwd], c.arcs_bwd);
        atomicAdd(&p.st->stat[kStTd], c.levels);
    }
}

template <int BLOCK>
void launch_lds(dim3 grid, dim3 block, size_t lds, hipStream_t s, const Params &p) {
    hipLaunchKernelGGL(k_brandes_lds<BLOCK>, grid, block, lds, s, p);
}

template <int BLOCK>
KernelRef lds_ref() {
    return KernelRef{(const void *)&k_brandes_lds<BLOCK>, &launch_lds<BLOCK>};
}

// One workgroup column per graph: the structural CSR checks of k_validate
// for every graph of a batch in one launch.
__global__ void k_validate_batched(const int32_t *rowptr_cat, const int32_t *colidx_cat, const long long *g_vtx,
                                   const long long *g_arc, DevStatus *st) {
    const int32_t g = blockIdx.x;
    const long long v0 = g_vtx[g];
    const int32_t n = (int32_t)(g_vtx[g + 1] - v0);
    const long long m = g_arc[g + 1] - g_arc[g];
    if (n == 0) return;
    const int32_t *rowptr = rowptr_cat + v0 + g;
    const int32_t *colidx = colidx_cat + g_arc[g];
    const long long tid = (long long)blockIdx.y * blockDim.x + threadIdx.x;
    const long long stride = (long long)gridDim.y * blockDim.x;
    int bad = 0;
    if (tid == 0 && (rowptr[0] != 0 || (long long)rowptr[n] != m)) bad = 1;
    for (long long i = tid; i < n; i += stride)
        if (rowptr[i + 1] < rowptr[i]) bad = 1;
    for (long long e = tid; e < m; e += stride) {
        const int32_t x = colidx[e];
        if (x < 0 || x >= n) bad = 1;
    }
    if (bad) atomicOr(&st->err, kErrGraph);
}

// One thread per arc e = u -> v with u < v: finds the reverse arc by binary
// search in v's ascending adjacency and writes the scaled sum to both.
__global__ void k_edge_symmetrize(const int32_t *rowptr, const int32_t *colidx, int32_t n, double *ebc, double scale,
                                  DevStatus *st) {
    if (st->err & kErrGraph) return;
    const long long stride = (long long)gridDim.x * blockDim.x;
    const long long m = rowptr[n];
    for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < m; e += stride) {
        // tail u of arc e: the last u with rowptr[u] <= e
        int32_t lo = 0, hi = n - 1;
        while (lo < hi) {
            const int32_t mid = (lo + hi + 1) >> 1;
            if (rowptr[mid] <= e) lo = mid; else hi = mid - 1;
        }
        const int32_t u = lo, v = colidx[e];
        if (v <= u) continue;
        int32_t a = rowptr[v], b = rowptr[v + 1] - 1;
        int32_t r = -1;
        while (a <= b) {
            const int32_t mid = (a + b) >> 1;
            const int32_t x = colidx[mid];
            if (x == u) { r = mid; break; }
            if (x < u) a = mid + 1; else b = mid - 1;
        }
        if (r < 0) {
            atomicOr(&st->err, kErrGraph);
            continue;
        }
        const double tot = (ebc[e] + ebc[r]) * scale;
        ebc[e] = tot;
        ebc[r] = tot;
    }
}

__global__ void k_reset_head(DevStatus *st) {
    if (threadIdx.x == 0) st->head = 0ULL;
}

}  // namespace

size_t lds_graph_bytes(int32_t n, int64_t m) {
    return 8 * (size_t)n + 4 * ((size_t)n + 1) + 4 * (size_t)m + 4 * (size_t)n + 4 * ((size_t)n + 2) +
           4 * (((size_t)n + 31) / 32);
}

KernelRef brandes_lds_kernel(int block) {
    switch (block) {
        case 256: return lds_ref<256>();
        case 512: return lds_ref<512>();
        default: return lds_ref<1024>();
    }
}

hipError_t launch_validate_batched(const int32_t *rowptr_cat, const int32_t *colidx_cat, const long long *g_vtx,
                                   const long long *g_arc, int32_t G, DevStatus *st, hipStream_t s) {
    if (G <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_validate_batched, dim3(G, 16), dim3(256), 0, s, rowptr_cat, colidx_cat, g_vtx, g_arc, st);
    return hipGetLastError();
}

hipError_t launch_edge_symmetrize(const int32_t *rowptr, const int32_t *colidx, int32_t n, double *ebc,
                                  double scale, DevStatus *st, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_edge_symmetrize, dim3(1024), dim3(256), 0, s, rowptr, colidx, n, ebc, scale, st);
    return hipGetLastError();
}

hipError_t launch_reset_head(DevStatus *st, hipStream_t s) {
    hipLaunchKernelGGL(k_reset_head, dim3(1), dim3(64), 0, s, st);
    return hipGetLastError();
}

}  // namespace nk
