// HIP kernels for Brandes betweenness on gfx950.
//
// One persistent kernel runs whole tasks per workgroup: a task is one
// source (exact / source-set / batched multi-graph forms), one sampled pair
// (pair sampling) or one inspection source.  Per task the workgroup runs
// Brandes' two phases (Brandes 2001, the algorithm the paper cites for
// betweenness in "Heuristics and Approximation Algorithms" and Table 1):
//
//   forward   level-synchronous breadth-first search that counts shortest
//             paths: sigma[w] = sum of sigma[v] over neighbours v one level
//             closer to the source.  Each level runs either top-down (scan
//             the arcs of the frontier list, 64-bit atomic adds into sigma
//             of unvisited neighbours, the first adder appends the vertex)
//             or bottom-up (scan all arcs of every unvisited vertex and sum
//             sigma over neighbours in the frontier, no atomics, no early
//             exit because every frontier neighbour contributes).  New
//             vertices are compacted into the next level list with a wave
//             ballot and one LDS atomic per wave.  The concatenated level
//             lists are the visit order S of Brandes' algorithm; each entry
//             carries the vertex, its first arc and its degree so later
//             passes read adjacency bounds sequentially.
//
//   backward  for levels from deepest to 1, every vertex v of the level
//             pulls over its neighbours w one level deeper:
//                 delta_v = sigma_v * sum_w (1 + delta_w) / sigma_w,
//             and replaces sigma_v in place by coef_v = (1 + delta_v) /
//             sigma_v (the only value the level above reads), then adds
//             delta_v to bc[v] (FP64 atomic add).  This is the dependency
//             recursion of Brandes' algorithm rearranged as a pull, so no
//             vertex is written by two threads.  A level whose successor
//             level has far fewer arcs is done the other way round: the
//             successor level pushes its coefficients into an accumulator
//             of its marked neighbours, which are exactly level l.
//
// The other modes (pair sampling, closeness, the bisection estimator,
// weighted graphs) reuse the same tiles and bitmap; each has its own
// section below.
//
// Visited state lives in one bitmap (LDS when it fits, else a per-slot
// global bitmap).  Isolated vertices start marked.  During the forward phase
// a neighbour of a level-l vertex that is unmarked must be at level l+1,
// and a marked neighbour of an unvisited vertex must be at level l; during
// the backward phase levels are unmarked from the deepest up, so an
// unmarked neighbour of a level-l vertex is at level l+1.  No distance
// array is read on the hot path.
//
// Work inside a level is balanced over arcs, not vertices: a tile of up to
// BLOCK listed vertices is staged in LDS with an exclusive prefix sum of
// degrees, and each thread takes kChunk consecutive arcs of the tile (one
// binary search, then a forward walk), so hubs with 10^5 arcs and leaves
// share the same loop.  Each thread first issues the column loads of its
// whole chunk, then the bitmap tests, then the path-count atomics or loads,
// so several global accesses per lane are in flight at once.
#include "nk_kernels.h"

namespace nk {

constexpr int kChunk = 4;

struct GView {
    const int32_t *rp;
    const int32_t *ci;
    int32_t n;
    int32_t m;
    long long vbase;   // offset of vertex 0 in concatenated outputs
    // arcs a bottom-up level scans: the in-arcs (the same arrays as rp/ci
    // for an undirected graph)
    const int32_t *trp;
    const int32_t *tci;
};

struct Scr {
    unsigned long long *dist;   // weighted mode: distances (all-ones = unreached)
    int32_t *mark;              // weighted mode: round that last queued the vertex
    int32_t *wl0, *wl1;         // weighted mode: worklists of the distance rounds
    int32_t *wl2;               // weighted mode: far pile
    uint32_t *dagm;             // weighted mode: DAG-arc bitmap over the arcs
    double *bvec;               // bisection: kBisK cutoff coefficients per vertex
    unsigned long long *sigma;  // path counts; coef bits during the backward phase
    double *dacc;               // push-mode dependency sums (kept at zero between uses)
    int32_t *ldeg;              // degree sum of each level
    int32_t *d;
    int32_t *lv;                // level lists: vertex
    int32_t *la;                // first arc
    int32_t *ld;                // degree
    int32_t *lvl;               // level offsets
    int32_t *cand;
    int32_t *ls;                // hashed pair records: table slot of each listed vertex
};

struct Counters {
    unsigned long long arcs_fwd, arcs_bwd, dag, reached, tasks, td, bu, arcs_reached, bw_push;
};

// Phase timing by thread 0 into LDS: phases end at block barriers, so
// thread 0's clock brackets the workgroup's time in the phase.
template <int BLOCK>
__device__ __forceinline__ void phase_start(Tile<BLOCK> &sm) {
    if (threadIdx.x == 0) sm.t0 = clock64();
}
template <int BLOCK>
__device__ __forceinline__ void phase_end(Tile<BLOCK> &sm, int ph) {
    if (threadIdx.x == 0) sm.cyc[ph] += (unsigned long long)(clock64() - sm.t0);
}
template <int BLOCK>
__device__ __forceinline__ void sub_mark(Tile<BLOCK> &sm, int sb) {
    if (threadIdx.x == 0) {
        const long long now = clock64();
        sm.sub[sb] += (unsigned long long)(now - sm.ts);
        sm.ts = now;
    }
}
template <int BLOCK>
__device__ __forceinline__ void sub_start(Tile<BLOCK> &sm) {
    if (threadIdx.x == 0) sm.ts = clock64();
}

__device__ __forceinline__ bool bit_test(const uint32_t *bm, int32_t v) {
    return (bm[v >> 5] >> (v & 31)) & 1u;
}
__device__ __forceinline__ void bit_set(uint32_t *bm, int32_t v) { atomicOr(&bm[v >> 5], 1u << (v & 31)); }
__device__ __forceinline__ void bit_clear(uint32_t *bm, int32_t v) { atomicAnd(&bm[v >> 5], ~(1u << (v & 31))); }

__device__ __forceinline__ double as_f64(unsigned long long x) { return __longlong_as_double((long long)x); }
__device__ __forceinline__ unsigned long long as_u64(double x) { return (unsigned long long)__double_as_longlong(x); }

// Stages list entries [tb, tb+cnt) into the tile and returns the tile's arc
// count.  Contains barriers.
template <int BLOCK>
__device__ __forceinline__ int32_t stage_list(Tile<BLOCK> &sm, const Scr &s, int32_t tb, int32_t cnt) {
    const int tid = threadIdx.x;
    int32_t dg = 0;
    if (tid < cnt) {
        sm.v[tid] = s.lv[tb + tid];
        sm.a0[tid] = s.la[tb + tid];
        dg = s.ld[tb + tid];
    }
    int32_t total;
    const int32_t ex = block_excl_scan<BLOCK>(dg, sm, total);
    if (tid < cnt) sm.pre[tid] = ex;
    if (tid == 0) sm.pre[cnt] = total;
    return total;
}

// Stages list[tb, tb+cnt) (vertex ids) with their arc ranges in g.
template <int BLOCK>
__device__ __forceinline__ int32_t stage_ids(Tile<BLOCK> &sm, const int32_t *list, const GView &g, int32_t tb,
                                             int32_t cnt) {
    const int tid = threadIdx.x;
    int32_t dg = 0;
    if (tid < cnt) {
        const int32_t v = list[tb + tid];
        const int32_t a0 = g.rp[v];
        sm.v[tid] = v;
        sm.a0[tid] = a0;
        dg = g.rp[v + 1] - a0;
    }
    int32_t total;
    const int32_t ex = block_excl_scan<BLOCK>(dg, sm, total);
    if (tid < cnt) sm.pre[tid] = ex;
    if (tid == 0) sm.pre[cnt] = total;
    return total;
}

// Column indices of the thread's chunk [i0, i0 + kChunk) of the tile's arcs;
// kk[j] = tile row of arc j, or -1 past the end.
template <int BLOCK>
__device__ __forceinline__ void load_chunk(const Tile<BLOCK> &sm, const GView &g, int32_t cnt, int32_t total,
                                           int32_t i0, int32_t (&kk)[kChunk], int32_t (&w)[kChunk]) {
    int32_t k = (i0 < total) ? tile_search(sm.pre, cnt, i0) : 0;
#pragma unroll
    for (int j = 0; j < kChunk; ++j) {
        const int32_t i = i0 + j;
        kk[j] = -1;
        w[j] = 0;
        if (i < total) {
            while (sm.pre[k + 1] <= i) ++k;
            kk[j] = k;
            w[j] = g.ci[sm.a0[k] + (i - sm.pre[k])];
        }
    }
}

// Word-granular staging of the level list [tb, tb + cnt): row k's arc range
// is [sm.a0[k], ends[k]), and sm.pre holds the exclusive prefix of the
// 32-arc bitmap words each range touches (sm.pre[cnt] = total words, the
// return value).  deg: the thread's row length (0 past cnt).  Callers that
// need the vertex ids stage them themselves.
template <int BLOCK>
__device__ __forceinline__ int32_t stage_words(Tile<BLOCK> &sm, const Scr &s, int32_t tb, int32_t cnt, int32_t *ends,
                                               int32_t &deg) {
    const int tid = threadIdx.x;
    int32_t wc = 0;
    deg = 0;
    if (tid < cnt) {
        const int32_t a0 = s.la[tb + tid];
        deg = s.ld[tb + tid];
        sm.a0[tid] = a0;
        ends[tid] = a0 + deg;
        wc = deg > 0 ? ((a0 + deg - 1) >> 5) - (a0 >> 5) + 1 : 0;
    }
    int32_t total;
    const int32_t ex = block_excl_scan<BLOCK>(wc, sm, total);
    if (tid < cnt) sm.pre[tid] = ex;
    if (tid == 0) sm.pre[cnt] = total;
    return total;
}

// As stage_words, for the vertex list list[tb, tb + cnt) (arc ranges from
// g.rp).
template <int BLOCK>
__device__ __forceinline__ int32_t stage_words_ids(Tile<BLOCK> &sm, const int32_t *list, const GView &g, int32_t tb,
                                                   int32_t cnt, int32_t *ends) {
    const int tid = threadIdx.x;
    int32_t wc = 0;
    if (tid < cnt) {
        const int32_t v = list[tb + tid];
        const int32_t a0 = g.rp[v], a1 = g.rp[v + 1];
        sm.a0[tid] = a0;
        ends[tid] = a1;
        wc = a1 > a0 ? ((a1 - 1) >> 5) - (a0 >> 5) + 1 : 0;
    }
    int32_t total;
    const int32_t ex = block_excl_scan<BLOCK>(wc, sm, total);
    if (tid < cnt) sm.pre[tid] = ex;
    if (tid == 0) sm.pre[cnt] = total;
    return total;
}

// Word wi of a word-staged tile: its row k, the word's index W in the arc
// bitmap, and the mask of the bits that belong to row k's arcs.
template <int BLOCK>
__device__ __forceinline__ void tile_word(const Tile<BLOCK> &sm, const int32_t *ends, int32_t cnt, int32_t wi,
                                          int32_t &k, long long &W, uint32_t &range) {
    k = tile_search(sm.pre, cnt, wi);
    const int32_t a0 = sm.a0[k], a1 = ends[k];
    W = (long long)(a0 >> 5) + (wi - sm.pre[k]);
    const long long base = W * 32;
    const int32_t blo = a0 > base ? (int32_t)(a0 - base) : 0;
    const int32_t bhi = (long long)a1 - base < 32 ? (int32_t)(a1 - base) : 32;
    range = (bhi >= 32 ? ~0u : ((1u << bhi) - 1u)) & ~((1u << blo) - 1u);
}

// ---------------------------------------------------------------- forward --

// Top-down expansion of level `lvl` (list[f0, f1)) into list[f1, ...).
template <int BLOCK, int MODE>
__device__ void td_level(const Params &p, Tile<BLOCK> &sm, uint32_t *bm, const Scr &s, const GView &g,
                         int32_t f0, int32_t f1, int32_t lvl, Counters &c) {
    const int tid = threadIdx.x;
    for (int32_t tb = f0; tb < f1; tb += BLOCK) {
        const int32_t cnt = min(BLOCK, f1 - tb);
        // closeness needs distances only: unit counts keep them from wrapping
        if (tid < cnt) sm.val.u[tid] = (MODE == kModeClose) ? 1ULL : s.sigma[s.lv[tb + tid]];
        const int32_t total = stage_list<BLOCK>(sm, s, tb, cnt);
        __syncthreads();
        if (tid == 0) c.arcs_fwd += (unsigned long long)total;
        for (int32_t rb = 0; rb < total; rb += BLOCK * kChunk) {
            int32_t kk[kChunk], w[kChunk];
            load_chunk<BLOCK>(sm, g, cnt, total, rb + tid * kChunk, kk, w);
            bool act[kChunk];
            unsigned long long add[kChunk], old[kChunk];
#pragma unroll
            for (int j = 0; j < kChunk; ++j) {
                act[j] = kk[j] >= 0 && !bit_test(bm, w[j]);
                add[j] = act[j] ? sm.val.u[kk[j]] : 0ULL;
            }
#pragma unroll
            for (int j = 0; j < kChunk; ++j) old[j] = act[j] ? atomicAdd(&s.sigma[w[j]], add[j]) : 1ULL;
#pragma unroll
            for (int j = 0; j < kChunk; ++j) {
                if (act[j]) {
                    c.dag++;
                    if (old[j] + add[j] < old[j]) atomicOr(&p.st->err, kErrOverflow);
                    if ((MODE == kModeSSSP) && old[j] == 0ULL) s.d[w[j]] = lvl + 1;
                }
                wave_append(act[j] && old[j] == 0ULL, w[j], s.lv + f1, &sm.count, g.n - f1, &p.st->err);
            }
        }
        __syncthreads();
    }
}

// Bottom-up expansion: every unvisited vertex sums sigma over its marked
// (= frontier) neighbours.
template <int BLOCK, int MODE>
__device__ void bu_level(const Params &p, Tile<BLOCK> &sm, uint32_t *bm, const Scr &s, const GView &go,
                         int32_t f1, int32_t lvl, Counters &c) {
    const int tid = threadIdx.x;
    const int lane = lane_id();
    // an unreached vertex looks for visited in-neighbours
    GView g = go;
    g.rp = go.trp;
    g.ci = go.tci;
    const bool sym = go.trp == go.rp;
    const int32_t nw = (g.n + 31) >> 5;
    if (tid == 0) sm.redmin = 0;  // candidate counter
    __syncthreads();
    for (int32_t wb = 0; wb < nw; wb += BLOCK) {
        const int32_t wi = wb + tid;
        uint32_t bits = (wi < nw) ? ~bm[wi] : 0u;
        const int32_t cnt = __popc(bits);
        const int32_t incl = wave_incl_scan<int32_t>(cnt);
        const int32_t wtot = __shfl(incl, kWave - 1, kWave);
        int32_t base = 0;
        if (lane == kWave - 1 && wtot > 0) base = atomicAdd(&sm.redmin, wtot);
        base = __shfl(base, kWave - 1, kWave);
        int32_t pos = base + incl - cnt;
        while (bits) {
            const int b = __ffs(bits) - 1;
            bits &= bits - 1u;
            s.cand[pos++] = wi * 32 + b;
        }
    }
    __syncthreads();
    const int32_t nc = sm.redmin;
    sub_start<BLOCK>(sm);
    for (int32_t tb = 0; tb < nc; tb += BLOCK) {
        const int32_t cnt = min(BLOCK, nc - tb);
        int32_t dg = 0;
        if (tid < cnt) {
            const int32_t w = s.cand[tb + tid];
            const int32_t a0 = g.rp[w];
            dg = g.rp[w + 1] - a0;
            sm.v[tid] = w;
            sm.a0[tid] = a0;
            sm.val.u[tid] = 0ULL;
        }
        int32_t total;
        const int32_t ex = block_excl_scan<BLOCK>(dg, sm, total);
        if (tid < cnt) sm.pre[tid] = ex;
        if (tid == 0) sm.pre[cnt] = total;
        __syncthreads();
        sub_mark<BLOCK>(sm, kSbBuStage);
        if (tid == 0) c.arcs_fwd += (unsigned long long)total;
        for (int32_t rb = 0; rb < total; rb += BLOCK * kChunk) {
            int32_t kk[kChunk], v[kChunk];
            load_chunk<BLOCK>(sm, g, cnt, total, rb + tid * kChunk, kk, v);
            unsigned long long sv[kChunk];
#pragma unroll
            for (int j = 0; j < kChunk; ++j) {
                const bool act = kk[j] >= 0 && bit_test(bm, v[j]);
                sv[j] = act ? ((MODE == kModeClose) ? 1ULL : s.sigma[v[j]]) : 0ULL;
            }
            int32_t kcur = kk[0];
            unsigned long long acc = 0ULL;
#pragma unroll
            for (int j = 0; j < kChunk; ++j) {
                if (kk[j] < 0) continue;
                if (kk[j] != kcur) {
                    if (acc) {
                        const unsigned long long o = atomicAdd(&sm.val.u[kcur], acc);
                        if (o + acc < o) atomicOr(&p.st->err, kErrOverflow);
                    }
                    kcur = kk[j];
                    acc = 0ULL;
                }
                if (sv[j]) {
                    const unsigned long long nacc = acc + sv[j];
                    if (nacc < acc) atomicOr(&p.st->err, kErrOverflow);
                    acc = nacc;
                    c.dag++;
                }
            }
            if (acc) {
                const unsigned long long o = atomicAdd(&sm.val.u[kcur], acc);
                if (o + acc < o) atomicOr(&p.st->err, kErrOverflow);
            }
        }
        __syncthreads();
        sub_mark<BLOCK>(sm, kSbBuArcs);
        bool fresh = false;
        int32_t w = 0;
        int32_t wa = 0, wd = 0;   // first out-arc and out-degree of the new vertex
        if (tid < cnt) {
            const unsigned long long sum = sm.val.u[tid];
            if (sum != 0ULL) {
                w = sm.v[tid];
                if (sym) {
                    wa = sm.a0[tid];
                    wd = dg;
                } else {
                    wa = go.rp[w];
                    wd = go.rp[w + 1] - wa;
                }
                s.sigma[w] = sum;
                if (MODE == kModeSSSP) s.d[w] = lvl + 1;
                fresh = true;
            }
        }
        // block-ordered append: candidates are in id order, so the new level
        // list comes out sorted and later per-vertex passes touch memory in
        // increasing address order
        int32_t nfresh;
        const int32_t rank = block_excl_scan<BLOCK>(fresh ? 1 : 0, sm, nfresh);
        const int32_t base = sm.count;
        if (fresh) {
            const int32_t pos = base + rank;
            if (pos < g.n - f1) {
                s.lv[f1 + pos] = w;
                s.la[f1 + pos] = wa;
                s.ld[f1 + pos] = wd;
            } else {
                atomicOr(&p.st->err, kErrInternal);
            }
        }
        __syncthreads();
        if (tid == 0) sm.count = base + nfresh;
        __syncthreads();
        sub_mark<BLOCK>(sm, kSbBuFin);
    }
}

// Forward phase from `src`.  Returns the deepest non-empty level Ld; the
// list holds levels 0..Ld at s.lvl[l] .. s.lvl[l+1].
template <int BLOCK, int MODE>
__device__ int32_t forward(const Params &p, Tile<BLOCK> &sm, uint32_t *bm, const Scr &s, const GView &g,
                           const uint32_t *iso, int32_t src, Counters &c) {
    const int tid = threadIdx.x;
    const int32_t nw = (g.n + 31) >> 5;
    phase_start<BLOCK>(sm);
    for (int32_t wi = tid; wi < nw; wi += BLOCK) {
        uint32_t x = iso ? iso[wi] : 0u;
        const int32_t hi = (wi + 1) * 32;
        if (hi > g.n) x |= ~0u << (32 - (hi - g.n));   // padding bits beyond n stay marked
        bm[wi] = x;
    }
    __syncthreads();
    if (tid == 0) {
        bm[src >> 5] |= 1u << (src & 31);
        s.sigma[src] = 1ULL;
        if (MODE == kModeSSSP) s.d[src] = 0;
        const int32_t a0 = g.rp[src];
        const int32_t dsrc = g.rp[src + 1] - a0;
        s.lv[0] = src;
        s.la[0] = a0;
        s.ld[0] = dsrc;
        s.lvl[0] = 0;
        s.lvl[1] = 1;
        s.ldeg[0] = dsrc;
        sm.mf = dsrc;
        sm.mu = (long long)g.m - dsrc;
        c.arcs_reached += (unsigned long long)dsrc;
        sm.lvl_lo[0] = 0;
        sm.lvl_lo[1] = 1;
    }
    __syncthreads();
    phase_end<BLOCK>(sm, kPhInit);
    int32_t lvl = 0;
    for (;;) {
        const int32_t f0 = sm.lvl_lo[0], f1 = sm.lvl_lo[1];
        const bool bu = (p.bu_ratio > 0.0f) && ((double)sm.mu < (double)p.bu_ratio * (double)sm.mf);
        __syncthreads();
        if (tid == 0) {
            sm.count = 0;
            sm.acc_mf = 0;
            if (bu) c.bu++; else c.td++;
        }
        __syncthreads();
        phase_start<BLOCK>(sm);
        if (bu)
            bu_level<BLOCK, MODE>(p, sm, bm, s, g, f1, lvl, c);
        else
            td_level<BLOCK, MODE>(p, sm, bm, s, g, f0, f1, lvl, c);
        __syncthreads();
        if (bu) phase_end<BLOCK>(sm, kPhBu); else phase_end<BLOCK>(sm, kPhTd);
        phase_start<BLOCK>(sm);
        const int32_t nnew = sm.count < g.n - f1 ? sm.count : g.n - f1;
        // mark the new level; a top-down level also records first arc and
        // degree of each new vertex (the bottom-up append already did)
        long long dsum = 0;
        for (int32_t i = f1 + tid; i < f1 + nnew; i += BLOCK) {
            const int32_t w = s.lv[i];
            bit_set(bm, w);
            int32_t dg;
            if (bu) {
                dg = s.ld[i];
            } else {
                const int32_t a0 = g.rp[w];
                dg = g.rp[w + 1] - a0;
                s.la[i] = a0;
                s.ld[i] = dg;
            }
            dsum += dg;
        }
        dsum = wave_sum<long long>(dsum);
        if (lane_id() == 0 && dsum) atomicAdd((unsigned long long *)&sm.acc_mf, (unsigned long long)dsum);
        __syncthreads();
        if (tid == 0) {
            s.lvl[lvl + 2] = f1 + nnew;
            s.ldeg[lvl + 1] = (int32_t)sm.acc_mf;
            sm.lvl_lo[0] = f1;
            sm.lvl_lo[1] = f1 + nnew;
            sm.mu -= sm.acc_mf;
            sm.mf = sm.acc_mf;
            c.arcs_reached += (unsigned long long)sm.acc_mf;
        }
        __syncthreads();
        phase_end<BLOCK>(sm, kPhMark);
        if (nnew == 0) break;
        ++lvl;
    }
    return lvl;
}

// --------------------------------------------------------------- backward --

// Level l by pull: every vertex v of level l sums coef over its unmarked
// (= level l+1) neighbours.
template <int BLOCK>
__device__ void bw_pull(Tile<BLOCK> &sm, const uint32_t *bm, const Scr &s, const GView &g, int32_t lo, int32_t hi,
                        double *bcg, double wfac, double owt, double *ebc, bool add_bc, Counters &c) {
    const int tid = threadIdx.x;
    sub_start<BLOCK>(sm);
    for (int32_t tb = lo; tb < hi; tb += BLOCK) {
        const int32_t cnt = min(BLOCK, hi - tb);
        if (tid < cnt) sm.val.f[tid] = 0.0;
        const int32_t total = stage_list<BLOCK>(sm, s, tb, cnt);
        __syncthreads();
        sub_mark<BLOCK>(sm, kSbPlStage);
        if (tid == 0) c.arcs_bwd += (unsigned long long)total;
        for (int32_t rb = 0; rb < total; rb += BLOCK * kChunk) {
            int32_t kk[kChunk], w[kChunk];
            load_chunk<BLOCK>(sm, g, cnt, total, rb + tid * kChunk, kk, w);
            double cf[kChunk];
#pragma unroll
            for (int j = 0; j < kChunk; ++j)
                cf[j] = (kk[j] >= 0 && !bit_test(bm, w[j])) ? as_f64(s.sigma[w[j]]) : 0.0;
            if (ebc) {
                // edge term of the DAG arc v -> w: sigma_v * (1 + delta_w) / sigma_w
#pragma unroll
                for (int j = 0; j < kChunk; ++j) {
                    if (cf[j] != 0.0) {
                        const int32_t k = kk[j];
                        const double sv = (double)s.sigma[sm.v[k]];
                        atomicAdd(ebc + sm.a0[k] + (rb + tid * kChunk + j - sm.pre[k]), sv * cf[j]);
                    }
                }
            }
            int32_t kcur = kk[0];
            double acc = 0.0;
#pragma unroll
            for (int j = 0; j < kChunk; ++j) {
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
        sub_mark<BLOCK>(sm, kSbPlArcs);
        if (tid < cnt) {
            const int32_t v = sm.v[tid];
            const double sg = (double)s.sigma[v];
            const double delta = sg * sm.val.f[tid] * wfac;
            s.sigma[v] = as_u64((1.0 + delta) / sg);
            if (add_bc && delta != 0.0 && owt != 0.0) atomicAdd(bcg + v, delta * owt);
        }
        __syncthreads();
        sub_mark<BLOCK>(sm, kSbPlFin);
    }
}

// Level l by push: every vertex w of level l+1 (list[lo1, hi1)) adds its
// coef to dacc of its marked (= level l) neighbours; then each vertex v of
// level l (list[lo, hi)) takes delta_v = sigma_v * dacc[v] and clears dacc.
// A directed graph pushes over the in-arcs (g is then the in-arc view: an
// in-neighbour of level l+1 is on level l or deeper, so a marked one is on
// level l) and skips the vertices no search reaches (`iso`, in-degree 0),
// which stay marked.  Edge scores (undirected): the DAG arc v -> w adds
// sigma_v * coef_w to the slot of its reverse arc w -> v, the one this
// scan holds (the two arcs of an edge are summed at the end).  add_bc:
// level l's dependencies are scores (not for the source's level).
template <int BLOCK>
__device__ void bw_push(Tile<BLOCK> &sm, const uint32_t *bm, const Scr &s, const GView &g, int32_t lo, int32_t hi,
                        int32_t lo1, int32_t hi1, double *bcg, double wfac, double owt, bool in_arcs,
                        const uint32_t *iso, double *ebc, bool add_bc, Counters &c) {
    const int tid = threadIdx.x;
    for (int32_t tb = lo1; tb < hi1; tb += BLOCK) {
        const int32_t cnt = min(BLOCK, hi1 - tb);
        if (tid < cnt) sm.val.f[tid] = as_f64(s.sigma[s.lv[tb + tid]]);
        const int32_t total = in_arcs ? stage_ids<BLOCK>(sm, s.lv, g, tb, cnt) : stage_list<BLOCK>(sm, s, tb, cnt);
        __syncthreads();
        if (tid == 0) c.arcs_bwd += (unsigned long long)total;
        for (int32_t rb = 0; rb < total; rb += BLOCK * kChunk) {
            int32_t kk[kChunk], v[kChunk];
            load_chunk<BLOCK>(sm, g, cnt, total, rb + tid * kChunk, kk, v);
#pragma unroll
            for (int j = 0; j < kChunk; ++j)
                if (kk[j] >= 0 && bit_test(bm, v[j]) && !(iso && bit_test(iso, v[j]))) {
                    const double cw = sm.val.f[kk[j]];
                    atomicAdd(s.dacc + v[j], cw);
                    if (ebc)
                        atomicAdd(ebc + sm.a0[kk[j]] + (rb + tid * kChunk + j - sm.pre[kk[j]]),
                                  (double)s.sigma[v[j]] * cw);
                }
        }
        __syncthreads();
    }
    for (int32_t i = lo + tid; i < hi; i += BLOCK) {
        const int32_t v = s.lv[i];
        const double sg = (double)s.sigma[v];
        const double delta = sg * s.dacc[v] * wfac;
        s.dacc[v] = 0.0;
        s.sigma[v] = as_u64((1.0 + delta) / sg);
        if (add_bc && delta != 0.0 && owt != 0.0) atomicAdd(bcg + v, delta * owt);
    }
    __syncthreads();
}

// Bisection estimator, truncated dependencies: delta^T (2 <= T < Ld)
// counts only targets at depth <= T, and a vertex on level l takes half of
// delta^(2l-1) and half of delta^(2l).  Cutoff T therefore needs the levels
// T-1 down to lmin(T) = ceil(T/2) only.  One pass serves a group of up to
// kBisK consecutive cutoffs T0..T1: every vertex keeps a vector of kBisK
// coefficients (one 32-byte line, slot T - T0) in s.bvec -- 1/sigma when
// it sits on level T itself (the targets), (1 + delta^T)/sigma above it --
// and level l is scanned once for all cutoffs active there (l < T <= 2l).
// A vertex on level lmin(T) adds delta^T / 2 to its score instead.
// As in the full sweep, the visited bitmap tells the level below: on entry
// every reached level is marked; levels T1.. are cleared first and each
// processed level after its pass, so an unmarked neighbour of level l is on
// level l+1 and a marked neighbour of level l+1 is on level l.  A level
// whose successor level has far fewer arcs is done by push from that level
// (its sums built in the same vector slots, cleared first).  Every slot a
// pass reads was written earlier in the same pass.  On exit every level is
// marked again.

template <int BLOCK>
__device__ void bis_group(Tile<BLOCK> &sm, uint32_t *bm, const Scr &s, const GView &g, int32_t T0, int32_t T1,
                          int32_t Ld, double *bcg, float bw_ratio, Counters &c) {
    constexpr int TV = BLOCK / kBisK;   // vertices per tile: their sums fill sm.val.f
    const int tid = threadIdx.x;
    const int32_t lmin0 = (T0 + 1) / 2;
    double *vec = s.bvec;
    for (int32_t i = s.lvl[T1] + tid; i < s.lvl[Ld + 1]; i += BLOCK) bit_clear(bm, s.lv[i]);
    for (int32_t i = s.lvl[T1] + tid; i < s.lvl[T1 + 1]; i += BLOCK) {
        const int32_t w = s.lv[i];
        vec[(long long)w * kBisK + (T1 - T0)] = 1.0 / (double)s.sigma[w];
    }
    __syncthreads();
    for (int32_t l = T1 - 1; l >= lmin0; --l) {
        const int32_t lo = s.lvl[l], hi = s.lvl[l + 1];
        // active cutoffs at level l: slots qa..qb
        const int qa = max(T0, l + 1) - T0, qb = min(T1, 2 * l) - T0;
        const bool seed = l >= T0;   // level l holds the targets of cutoff T = l
        const bool push = (double)s.ldeg[l + 1] < (double)bw_ratio * (double)s.ldeg[l];
        if (push) {
            if (tid == 0) c.bw_push++;
            for (int32_t i = lo + tid; i < hi; i += BLOCK) {
                double *x = vec + (long long)s.lv[i] * kBisK;
                for (int q = qa; q <= qb; ++q) x[q] = 0.0;
            }
            __syncthreads();
            const int32_t hi1 = s.lvl[l + 2];
            for (int32_t tb = hi; tb < hi1; tb += TV) {
                const int32_t cnt = min(TV, hi1 - tb);
                if (tid < cnt * kBisK) {
                    const int32_t r = tid / kBisK, q = tid % kBisK;
                    sm.val.f[tid] = (q >= qa && q <= qb) ? vec[(long long)s.lv[tb + r] * kBisK + q] : 0.0;
                }
                const int32_t total = stage_list<BLOCK>(sm, s, tb, cnt);
                __syncthreads();
                if (tid == 0) c.arcs_bwd += (unsigned long long)total;
                for (int32_t rb = 0; rb < total; rb += BLOCK * kChunk) {
                    int32_t kk[kChunk], v[kChunk];
                    load_chunk<BLOCK>(sm, g, cnt, total, rb + tid * kChunk, kk, v);
#pragma unroll
                    for (int j = 0; j < kChunk; ++j)
                        if (kk[j] >= 0 && bit_test(bm, v[j]))
                            for (int q = qa; q <= qb; ++q)
                                atomicAdd(vec + (long long)v[j] * kBisK + q, sm.val.f[kk[j] * kBisK + q]);
                }
                __syncthreads();
            }
            for (int32_t i = lo + tid; i < hi; i += BLOCK) {
                const int32_t v = s.lv[i];
                double *x = vec + (long long)v * kBisK;
                const double sg = (double)s.sigma[v];
                double add = 0.0;
                for (int q = qa; q <= qb; ++q) {
                    const double delta = sg * x[q];
                    if (l > (T0 + q + 1) / 2)
                        x[q] = (1.0 + delta) / sg;
                    else
                        add += 0.5 * delta;
                }
                if (seed) x[l - T0] = 1.0 / sg;
                if (add != 0.0) atomicAdd(bcg + v, add);
            }
            __syncthreads();
        } else {
            for (int32_t tb = lo; tb < hi; tb += TV) {
                const int32_t cnt = min(TV, hi - tb);
                if (tid < cnt * kBisK) sm.val.f[tid] = 0.0;
                const int32_t total = stage_list<BLOCK>(sm, s, tb, cnt);
                __syncthreads();
                if (tid == 0) c.arcs_bwd += (unsigned long long)total;
                for (int32_t rb = 0; rb < total; rb += BLOCK * kChunk) {
                    int32_t kk[kChunk], w[kChunk];
                    load_chunk<BLOCK>(sm, g, cnt, total, rb + tid * kChunk, kk, w);
                    int32_t kcur = kk[0];
                    double acc[kBisK] = {};
#pragma unroll
                    for (int j = 0; j < kChunk; ++j) {
                        if (kk[j] < 0) continue;
                        if (kk[j] != kcur) {
#pragma unroll
                            for (int q = 0; q < kBisK; ++q)
                                if (acc[q] != 0.0) atomicAdd(&sm.val.f[kcur * kBisK + q], acc[q]);
                            kcur = kk[j];
#pragma unroll
                            for (int q = 0; q < kBisK; ++q) acc[q] = 0.0;
                        }
                        if (!bit_test(bm, w[j])) {
                            // the vector is one aligned line: 16-byte loads
                            const double2 *x = reinterpret_cast<const double2 *>(vec + (long long)w[j] * kBisK);
#pragma unroll
                            for (int h = 0; h < kBisK / 2; ++h) {
                                const double2 y = x[h];
                                if (2 * h >= qa && 2 * h <= qb) acc[2 * h] += y.x;
                                if (2 * h + 1 >= qa && 2 * h + 1 <= qb) acc[2 * h + 1] += y.y;
                            }
                        }
                    }
                    if (kcur >= 0)
#pragma unroll
                        for (int q = 0; q < kBisK; ++q)
                            if (acc[q] != 0.0) atomicAdd(&sm.val.f[kcur * kBisK + q], acc[q]);
                }
                __syncthreads();
                if (tid < cnt) {
                    const int32_t v = sm.v[tid];
                    double *x = vec + (long long)v * kBisK;
                    const double sg = (double)s.sigma[v];
                    double add = 0.0;
                    for (int q = qa; q <= qb; ++q) {
                        const double delta = sg * sm.val.f[tid * kBisK + q];
                        if (l > (T0 + q + 1) / 2)
                            x[q] = (1.0 + delta) / sg;
                        else
                            add += 0.5 * delta;
                    }
                    if (seed) x[l - T0] = 1.0 / sg;
                    if (add != 0.0) atomicAdd(bcg + v, add);
                }
                __syncthreads();
            }
        }
        for (int32_t i = lo + tid; i < hi; i += BLOCK) bit_clear(bm, s.lv[i]);
        __syncthreads();
    }
    for (int32_t i = s.lvl[lmin0] + tid; i < s.lvl[Ld + 1]; i += BLOCK) bit_set(bm, s.lv[i]);
    __syncthreads();
}

template <int BLOCK, bool BIS>
__device__ void backward(const Params &p, Tile<BLOCK> &sm, uint32_t *bm, const Scr &s, const GView &g,
                         int32_t Ld, double *bcg, Counters &c) {
    const int tid = threadIdx.x;
    if (Ld == 0) return;
    // bisection: the truncated sweeps need the path counts, which the full
    // sweep below overwrites with coefficients, so they run first
    if constexpr (BIS) {
        phase_start<BLOCK>(sm);
        for (int32_t T0 = 2; T0 < Ld; T0 += kBisK)
            bis_group<BLOCK>(sm, bm, s, g, T0, min(T0 + kBisK - 1, Ld - 1), Ld, bcg, p.bw_ratio, c);
        phase_end<BLOCK>(sm, kPhPull);
    }
    {
        const int32_t lo = s.lvl[Ld], hi = s.lvl[Ld + 1];
        for (int32_t i = lo + tid; i < hi; i += BLOCK) {
            const int32_t v = s.lv[i];
            s.sigma[v] = as_u64(1.0 / (double)s.sigma[v]);
            bit_clear(bm, v);
        }
    }
    __syncthreads();
    // edge scores need the source's own arcs too: sweep down to level 0
    // (the source's dependency is not a score and is not added)
    const int32_t lmin = p.ebc ? 0 : 1;
    for (int32_t l = Ld - 1; l >= lmin; --l) {
        const int32_t lo = s.lvl[l], hi = s.lvl[l + 1], hi1 = s.lvl[l + 2];
        // linear scaling: the pair weights d(s,v)/d(s,t) factor as l/(l+1)
        // per DAG step from level l+1 to level l
        const double wfac = p.linear ? (double)l / (double)(l + 1) : 1.0;
        // bisection: level l takes the full dependency once for each of the
        // depths 2l-1, 2l that reach the deepest level Ld
        const double owt = BIS ? 0.5 * ((2 * l - 1 >= Ld ? 1.0 : 0.0) + (2 * l >= Ld ? 1.0 : 0.0)) : 1.0;
        // scan whichever side of the level pair has fewer arcs (a push
        // scans in-arcs, which a directed run has only with the in-arc CSR;
        // its level degree sums count out-arcs, the proxy used there too)
        const bool push = (!p.directed || p.trowptr) &&
                          (double)s.ldeg[l + 1] < (double)p.bw_ratio * (double)s.ldeg[l];
        phase_start<BLOCK>(sm);
        if (push) {
            if (tid == 0) c.bw_push++;
            if (p.directed) {
                GView gin = g;
                gin.rp = g.trp;
                gin.ci = g.tci;
                bw_push<BLOCK>(sm, bm, s, gin, lo, hi, hi, hi1, bcg, wfac, owt, true, p.iso, nullptr, l >= 1, c);
            } else {
                bw_push<BLOCK>(sm, bm, s, g, lo, hi, hi, hi1, bcg, wfac, owt, false, nullptr, p.ebc, l >= 1, c);
            }
        } else {
            bw_pull<BLOCK>(sm, bm, s, g, lo, hi, bcg, wfac, owt, p.ebc, l >= 1, c);
        }
        if (push) phase_end<BLOCK>(sm, kPhPush); else phase_end<BLOCK>(sm, kPhPull);
        for (int32_t i = lo + tid; i < hi; i += BLOCK) bit_clear(bm, s.lv[i]);
        __syncthreads();
    }
}

// --------------------------------------------------------------- weighted --
//
// Positive integer arc weights.  Per source: (1) distances by label-
// correcting rounds: each round relaxes the out-arcs of the vertices whose
// distance dropped in the previous round (64-bit atomicMin), queueing each
// improved vertex once per round, and marks every arc that ties or improves
// its head's distance as a DAG candidate in the per-slot arc bitmap; (2) the
// shortest-path DAG (arcs with dist_v + w = dist_x, tested on candidates
// only, the others' bits dropped) in layers -- one per distance value, or
// Kahn layers after an in-degree pass -- with each layer pushing its path
// counts to its DAG successors, so every DAG arc goes from a layer to a
// later one; (3) the dependency pull over the layers in reverse over the
// arcs whose bits are set, clearing them.

constexpr unsigned long long kInf = ~0ULL;

// Distances from src; returns the number of reached vertices, listed in
// s.cand.  ep: the workgroup's round counter (never repeats in a launch).
// Near-far ordering (a two-bucket form of delta-stepping): a round relaxes
// the queued vertices whose distance is below the threshold; an improved
// vertex joins the next round if its new distance is below the threshold,
// else a "far" pile (once: s.d flags membership).  When no near vertex is
// left the threshold rises by p.wdelta and the far vertices now below it
// move to the next round.  Vertices are then settled roughly in distance
// order, so fewer of them are relaxed more than once.
template <int BLOCK>
__device__ int32_t w_distances(const Params &p, Tile<BLOCK> &sm, uint32_t *bm, const Scr &s, const GView &g,
                               int32_t src, int32_t &ep, unsigned long long *sd, Counters &c) {
    const int tid = threadIdx.x;
    __shared__ int32_t s_reach, s_next, s_far, s_keep;
    const unsigned long long step = p.wdelta > 0 ? (unsigned long long)p.wdelta : kInf;
    unsigned long long thr = step;
    // bm: settled vertices.  When no near vertex is left below the
    // threshold, every vertex whose distance is below it is final; those
    // processed since the last rise (listed in s.lv, the pending list) are
    // marked then, and later rounds skip arcs into them: with weights >= 1
    // such an arc can neither improve nor tie their distance.
    const int32_t nw = (g.n + 31) >> 5;
    for (int32_t wi = tid; wi < nw; wi += BLOCK) bm[wi] = 0u;
    if (tid == 0) {
        s.dist[src] = 0ULL;
        s.cand[0] = src;
        s.wl0[0] = src;
        s_reach = 1;
        s_far = 0;
    }
    __syncthreads();
    int32_t cur = 0, ncur = 1;
    long long npend = 0;   // pending list length (uniform across the workgroup)
    for (;;) {
        ++ep;
        const int32_t *in = cur == 0 ? s.wl0 : s.wl1;
        int32_t *out = cur == 0 ? s.wl1 : s.wl0;
        if (tid == 0) {
            s_next = 0;
            c.td++;
        }
        // this round's vertices join the pending list while it has room (a
        // vertex left out is only not skipped later)
        if (npend + ncur <= p.stride) {
            for (int32_t i = tid; i < ncur; i += BLOCK) s.lv[npend + i] = in[i];
            npend += ncur;
        }
        __syncthreads();
        for (int32_t tb = 0; tb < ncur; tb += BLOCK) {
            const int32_t cnt = min(BLOCK, ncur - tb);
            const int32_t total = stage_ids<BLOCK>(sm, in, g, tb, cnt);
            if (tid < cnt) sd[tid] = s.dist[sm.v[tid]];
            __syncthreads();
            if (tid == 0) c.arcs_fwd += (unsigned long long)total;
            for (int32_t rb = 0; rb < total; rb += BLOCK * kChunk) {
                int32_t kk[kChunk], w[kChunk];
                load_chunk<BLOCK>(sm, g, cnt, total, rb + tid * kChunk, kk, w);
                int32_t word = -1;
                uint32_t bits = 0u;
#pragma unroll
                for (int j = 0; j < kChunk; ++j) {
                    bool first = false, queue = false, far = false;
                    if (kk[j] >= 0 && !bit_test(bm, w[j])) {
                        const int32_t k = kk[j];
                        const int32_t arc = sm.a0[k] + (rb + tid * kChunk + j - sm.pre[k]);
                        const unsigned long long nd = sd[k] + (unsigned long long)p.wts[arc];
                        const unsigned long long cur = s.dist[w[j]];
                        // an arc that ties or improves its head's distance may
                        // end in the shortest-path DAG: every DAG arc does so
                        // when its tail is relaxed at its final distance
                        if (nd <= cur) {
                            if ((arc >> 5) != word) {
                                if (bits) atomicOr(&s.dagm[word], bits);
                                word = arc >> 5;
                                bits = 0u;
                            }
                            bits |= 1u << (arc & 31);
                        }
                        if (nd < cur) {
                            const unsigned long long old = atomicMin(&s.dist[w[j]], nd);
                            if (nd < old) {
                                first = old == kInf;
                                if (nd < thr) {
                                    queue = atomicExch(&s.mark[w[j]], ep) != ep;
                                    s.d[w[j]] = 0;   // a far-pile entry of w is stale now
                                } else {
                                    far = atomicExch(&s.d[w[j]], 1) == 0;
                                }
                            }
                        }
                    }
                    wave_append(first, w[j], s.cand, &s_reach, g.n, &p.st->err);
                    wave_append(queue, w[j], out, &s_next, g.n, &p.st->err);
                    wave_append(far, w[j], s.wl2, &s_far, g.n, &p.st->err);
                }
                if (bits) atomicOr(&s.dagm[word], bits);
            }
            __syncthreads();
        }
        int32_t nn = s_next;
        __syncthreads();
        if (nn == 0 && s_far > 0) {
            // the threshold rises: the pending vertices are final
            for (long long i = tid; i < npend; i += BLOCK) bit_set(bm, s.lv[i]);
            npend = 0;
            __syncthreads();
        }
        // no near vertex left: raise the threshold until some far vertex is
        // below it, and move those to the next round
        while (nn == 0 && s_far > 0) {
            thr = thr > kInf - step ? kInf : thr + step;
            const int32_t nf = s_far;
            if (tid == 0) s_keep = 0;
            __syncthreads();
            // far vertices are kept in place (their order matters not);
            // each pass rewrites the pile's prefix with the ones that stay
            for (int32_t tb = 0; tb < nf; tb += BLOCK) {
                const int32_t i = tb + tid;
                const int32_t v = i < nf ? s.wl2[i] : 0;
                // an entry whose vertex was queued near since is dropped
                const bool live = i < nf && s.d[v] != 0;
                const bool near = live && s.dist[v] < thr;
                __syncthreads();   // every thread has read its entry before any is rewritten
                wave_append(near, v, out, &s_next, g.n, &p.st->err);
                wave_append(live && !near, v, s.wl2, &s_keep, g.n, &p.st->err);
                if (near) s.d[v] = 0;
                __syncthreads();
            }
            if (tid == 0) s_far = s_keep;
            __syncthreads();
            nn = s_next;
            __syncthreads();
        }
        if (nn == 0) break;
        cur ^= 1;
        ncur = nn;
    }
    return s_reach;
}

// Shortest-path DAG layers from src over the reached vertices (s.cand[0,
// nreach)): path counts into s.sigma, layers into s.lv/la/ld with offsets
// s.lvl, DAG arcs into the bitmap s.dagm; s.d holds DAG in-degrees.
// Returns the deepest layer.
template <int BLOCK>
__device__ int32_t w_layers_kahn(const Params &p, Tile<BLOCK> &sm, const Scr &s, const GView &g, int32_t src,
                                 int32_t nreach, unsigned long long *sd, Counters &c) {
    const int tid = threadIdx.x;
    for (int32_t i = tid; i < nreach; i += BLOCK) s.d[s.cand[i]] = 0;
    __syncthreads();
    // DAG in-degrees, a thread per arc-bitmap word (candidate arcs only;
    // the rows' ends take the place of the vertex ids)
    for (int32_t tb = 0; tb < nreach; tb += BLOCK) {
        const int32_t cnt = min(BLOCK, nreach - tb);
        if (tid < cnt) sd[tid] = s.dist[s.cand[tb + tid]];
        const int32_t total = stage_words_ids<BLOCK>(sm, s.cand, g, tb, cnt, sm.v);
        __syncthreads();
        for (int32_t wi = tid; wi < total; wi += BLOCK) {
            int32_t k;
            long long W;
            uint32_t bits;
            tile_word<BLOCK>(sm, sm.v, cnt, wi, k, W, bits);
            bits &= s.dagm[W];
            uint32_t drop = 0u;
            while (bits) {
                const int b = __builtin_ctz(bits);
                bits &= bits - 1u;
                const int32_t arc = (int32_t)(W * 32 + b);
                const int32_t x = g.ci[arc];
                if (sd[k] + (unsigned long long)p.wts[arc] == s.dist[x]) {
                    atomicAdd(&s.d[x], 1);
                    c.dag++;
                } else {
                    drop |= 1u << b;
                }
            }
            if (drop) atomicAnd(&s.dagm[W], ~drop);
        }
        __syncthreads();
    }
    if (tid == 0) {
        const int32_t a0 = g.rp[src];
        s.sigma[src] = 1ULL;
        s.lv[0] = src;
        s.la[0] = a0;
        s.ld[0] = g.rp[src + 1] - a0;
        s.lvl[0] = 0;
        s.lvl[1] = 1;
    }
    __syncthreads();
    int32_t lo = 0, hi = 1, L = 0;
    for (;;) {
        if (tid == 0) {
            sm.count = 0;
            c.bu++;
        }
        __syncthreads();
        for (int32_t tb = lo; tb < hi; tb += BLOCK) {
            const int32_t cnt = min(BLOCK, hi - tb);
            if (tid < cnt) sm.val.u[tid] = s.sigma[s.lv[tb + tid]];
            // a thread per arc-bitmap word, DAG arcs only (the rows' ends
            // take the place of the vertex ids); a head whose last DAG
            // in-arc this is joins the next layer by an LDS counter
            int32_t deg;
            const int32_t total = stage_words<BLOCK>(sm, s, tb, cnt, sm.v, deg);
            __syncthreads();
            for (int32_t wi = tid; wi < total; wi += BLOCK) {
                int32_t k;
                long long W;
                uint32_t bits;
                tile_word<BLOCK>(sm, sm.v, cnt, wi, k, W, bits);
                bits &= s.dagm[W];
                while (bits) {
                    const int b = __builtin_ctz(bits);
                    bits &= bits - 1u;
                    const int32_t x = g.ci[(int32_t)(W * 32 + b)];
                    const unsigned long long add = sm.val.u[k];
                    const unsigned long long o = atomicAdd(&s.sigma[x], add);
                    if (o + add < o) atomicOr(&p.st->err, kErrOverflow);
                    if (atomicSub(&s.d[x], 1) == 1) {
                        const int32_t pos = atomicAdd(&sm.count, 1);
                        if (pos < g.n - hi) {
                            const int32_t a0 = g.rp[x];
                            s.lv[hi + pos] = x;
                            s.la[hi + pos] = a0;
                            s.ld[hi + pos] = g.rp[x + 1] - a0;
                        } else {
                            atomicOr(&p.st->err, kErrInternal);
                        }
                    }
                }
            }
            __syncthreads();
        }
        const int32_t nnew = sm.count < g.n - hi ? sm.count : g.n - hi;
        if (tid == 0) s.lvl[L + 2] = hi + nnew;
        __syncthreads();
        if (nnew == 0) break;
        lo = hi;
        hi += nnew;
        ++L;
    }
    return L;
}


// The same layers when every reached distance is below kDistBuckets (and
// below the per-slot stride): one layer per distance value, found by a
// counting sort in LDS -- a DAG arc always goes to a larger distance, so
// the layers are a topological order and no in-degree pass is needed.
// Layer l holds the vertices at distance l (often none).  Returns the
// deepest layer.
template <int BLOCK>
__device__ int32_t w_layers_buckets(const Params &p, Tile<BLOCK> &sm, const Scr &s, const GView &g, int32_t src,
                                    int32_t nreach, int32_t D, int32_t *hist, unsigned long long *sd,
                                    Counters &c) {
    const int tid = threadIdx.x;
    for (int32_t b = tid; b < D; b += BLOCK) hist[b] = 0;
    __syncthreads();
    for (int32_t i = tid; i < nreach; i += BLOCK) atomicAdd(&hist[(int32_t)s.dist[s.cand[i]]], 1);
    __syncthreads();
    // exclusive prefix of the histogram into s.lvl and into hist (cursors)
    int32_t carry = 0;
    for (int32_t b0 = 0; b0 < D; b0 += BLOCK) {
        const int32_t b = b0 + tid;
        const int32_t x = b < D ? hist[b] : 0;
        int32_t total;
        const int32_t ex = block_excl_scan<BLOCK>(x, sm, total);
        if (b < D) {
            s.lvl[b] = carry + ex;
            hist[b] = carry + ex;
        }
        carry += total;
    }
    if (tid == 0) s.lvl[D] = carry;
    __syncthreads();
    for (int32_t i = tid; i < nreach; i += BLOCK) {
        const int32_t v = s.cand[i];
        const int32_t pos = atomicAdd(&hist[(int32_t)s.dist[v]], 1);
        const int32_t a0 = g.rp[v];
        s.lv[pos] = v;
        s.la[pos] = a0;
        s.ld[pos] = g.rp[v + 1] - a0;
    }
    if (tid == 0) s.sigma[src] = 1ULL;
    __syncthreads();
    // path counts: each layer pushes to its DAG successors, all in later layers
    for (int32_t l = 0; l < D; ++l) {
        const int32_t lo = s.lvl[l], hi = s.lvl[l + 1];
        if (lo == hi) continue;
        if (tid == 0) c.bu++;
        for (int32_t tb = lo; tb < hi; tb += BLOCK) {
            const int32_t cnt = min(BLOCK, hi - tb);
            if (tid < cnt) {
                const int32_t v = s.lv[tb + tid];
                sd[tid] = s.dist[v];
                sm.val.u[tid] = s.sigma[v];
            }
            // the rows' ends take the place of the vertex ids
            int32_t deg;
            const int32_t total = stage_words<BLOCK>(sm, s, tb, cnt, sm.v, deg);
            __syncthreads();
            // a thread per bitmap word: only candidate arcs are looked at
            for (int32_t wi = tid; wi < total; wi += BLOCK) {
                int32_t k;
                long long W;
                uint32_t bits;
                tile_word<BLOCK>(sm, sm.v, cnt, wi, k, W, bits);
                bits &= s.dagm[W];
                uint32_t drop = 0u;
                while (bits) {
                    const int b = __builtin_ctz(bits);
                    bits &= bits - 1u;
                    const int32_t arc = (int32_t)(W * 32 + b);
                    const int32_t x = g.ci[arc];
                    if (sd[k] + (unsigned long long)p.wts[arc] == s.dist[x]) {
                        const unsigned long long add = sm.val.u[k];
                        const unsigned long long o = atomicAdd(&s.sigma[x], add);
                        if (o + add < o) atomicOr(&p.st->err, kErrOverflow);
                        c.dag++;
                    } else {
                        drop |= 1u << b;
                    }
                }
                if (drop) atomicAnd(&s.dagm[W], ~drop);
            }
            __syncthreads();
        }
    }
    return D - 1;
}

// Layers of the shortest-path DAG (see w_layers_kahn / w_layers_buckets):
// by distance buckets when the reached distances span few values, else by
// Kahn layering.
template <int BLOCK>
__device__ int32_t w_layers(const Params &p, Tile<BLOCK> &sm, const Scr &s, const GView &g, int32_t src,
                            int32_t nreach, int32_t *hist, unsigned long long *sd, Counters &c) {
    __shared__ unsigned long long s_maxd;
    const int tid = threadIdx.x;
    if (tid == 0) s_maxd = 0ULL;
    __syncthreads();
    unsigned long long mx = 0ULL;
    for (int32_t i = tid; i < nreach; i += BLOCK) {
        const unsigned long long d = s.dist[s.cand[i]];
        mx = d > mx ? d : mx;
    }
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) {
        const unsigned long long y = __shfl_xor(mx, off, kWave);
        mx = y > mx ? y : mx;
    }
    if (lane_id() == 0) atomicMax(&s_maxd, mx);
    __syncthreads();
    const unsigned long long maxd = s_maxd;
    __syncthreads();
    if (maxd + 1 <= (unsigned long long)kDistBuckets && (long long)maxd + 2 <= p.stride)
        return w_layers_buckets<BLOCK>(p, sm, s, g, src, nreach, (int32_t)maxd + 1, hist, sd, c);
    return w_layers_kahn<BLOCK>(p, sm, s, g, src, nreach, sd, c);
}

// Dependencies over the layers in reverse: delta_v = sigma_v * sum over DAG
// successors x of (1 + delta_x) / sigma_x, kept as coefficients in place
// of sigma; bc[v] += delta_v for every layer but the source's.  The DAG
// arcs are the bits the path-count pass set in s.dagm (a few percent of the
// arcs on weighted graphs, whose shortest paths are mostly unique), so
// the sweep reads no distances and no weights.
template <int BLOCK>
__device__ void w_backward(Tile<BLOCK> &sm, const Scr &s, const GView &g, int32_t Ld, double *bcg, int32_t *ends,
                           Counters &c) {
    const int tid = threadIdx.x;
    if (Ld == 0) return;
    for (int32_t i = s.lvl[Ld] + tid; i < s.lvl[Ld + 1]; i += BLOCK) {
        const int32_t v = s.lv[i];
        s.sigma[v] = as_u64(1.0 / (double)s.sigma[v]);
    }
    __syncthreads();
    for (int32_t l = Ld - 1; l >= 1; --l) {
        const int32_t lo = s.lvl[l], hi = s.lvl[l + 1];
        for (int32_t tb = lo; tb < hi; tb += BLOCK) {
            const int32_t cnt = min(BLOCK, hi - tb);
            if (tid < cnt) {
                sm.val.f[tid] = 0.0;
                sm.v[tid] = s.lv[tb + tid];
            }
            int32_t deg;
            const int32_t total = stage_words<BLOCK>(sm, s, tb, cnt, ends, deg);
            __syncthreads();
            c.arcs_bwd += (unsigned long long)deg;
            // a thread per bitmap word: the DAG arcs load their head's
            // coefficient; their bits are cleared on the way
            for (int32_t wi = tid; wi < total; wi += BLOCK) {
                int32_t k;
                long long W;
                uint32_t bits;
                tile_word<BLOCK>(sm, ends, cnt, wi, k, W, bits);
                bits &= s.dagm[W];
                if (bits == 0u) continue;
                atomicAnd(&s.dagm[W], ~bits);
                double acc = 0.0;
                while (bits) {
                    const int b = __builtin_ctz(bits);
                    bits &= bits - 1u;
                    acc += as_f64(s.sigma[g.ci[(int32_t)(W * 32 + b)]]);
                }
                atomicAdd(&sm.val.f[k], acc);
            }
            __syncthreads();
            if (tid < cnt) {
                const int32_t v = sm.v[tid];
                const double sg = (double)s.sigma[v];
                const double delta = sg * sm.val.f[tid];
                s.sigma[v] = as_u64((1.0 + delta) / sg);
                if (delta != 0.0) atomicAdd(bcg + v, delta);
            }
            __syncthreads();
        }
    }
}

// --------------------------------------------------------------- path walk --

// Block-scope state of one bidirectional search (side 0 grows from u,
// side 1 from v).
struct BiState {
    int32_t lo[2], hi[2], depth[2];  // deepest level of each side: list[lo, hi)
    long long cost[2];               // arcs leaving that level
    long long newcost;
    int32_t nm;                      // meeting vertices collected
    int32_t z;                       // chosen meeting vertex
    int32_t result;                  // 0 searching, 1 met, -1 unreachable, -3 overflow
    int32_t pad;
    int32_t pickw, pickv;            // block walk: first crossing wave, chosen vertex
    int32_t full;                    // hashed records: a claim found the table full
    int32_t small[2];                // the path counts of each side's deepest level sum below 2^64
    long long dsum[2];               // arcs of all the vertices each side has listed
    int32_t tover;                   // the level being built: its path counts' sum reached 2^64
    unsigned long long tsum;         // ... and that sum modulo 2^64
    unsigned long long part_lo[16], part_hi[16];
    unsigned long long total, r0;
};

// Block-wide 128-bit sum of one u64 per thread: (hi, lo) words.  Contains
// barriers.
template <int BLOCK>
__device__ void block_sum_u128(unsigned long long x, BiState &bs, unsigned long long &lo,
                               unsigned long long &hi) {
    unsigned long long l = x, h = 0;
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) {
        const unsigned long long ol = __shfl_xor(l, off, kWave), oh = __shfl_xor(h, off, kWave);
        const unsigned long long nl = l + ol;
        h = h + oh + (nl < l ? 1ULL : 0ULL);
        l = nl;
    }
    if (lane_id() == 0) {
        bs.part_lo[wave_id()] = l;
        bs.part_hi[wave_id()] = h;
    }
    __syncthreads();
    lo = 0;
    hi = 0;
#pragma unroll
    for (int w = 0; w < BLOCK / kWave; ++w) {
        const unsigned long long nl = lo + bs.part_lo[w];
        hi += bs.part_hi[w] + (nl < lo ? 1ULL : 0ULL);
        lo = nl;
    }
    __syncthreads();
}

// Pair mode keeps both search sides' state of a vertex in one 32-byte
// record, so the visited test, the path-count update, the meeting test, the
// side-choice cost and the walk's predecessor test each touch one cache
// line.  d = -1 is unreached; a sample resets the path counts and distances
// of the records it touched.
struct PairRec {
    unsigned long long sig[2];   // path counts from u (side 0) and from v (side 1)
    int32_t d[2];                // distances from u and from v
    int32_t key;                 // one record per vertex: the vertex's degree;
                                 // hashed records: vertex + 1 (0 = free entry)
    int32_t pad;
};

// Record access: one record per vertex (DirectRecs), or a per-slot table of
// 2^ph_log2 entries keyed by vertex with linear probing (HashRecs), whose
// free entries hold the unreached state, so a claimed entry needs no set-up.
// A sample claims an entry the first time a search side reaches its vertex,
// lists the vertex with the entry's slot, and frees every listed slot at
// the end.  Within a sample keys are only added, so a probe that meets a
// free entry has seen all of the vertex's chain.  The table stays at most
// half full (a level that could pass that is not run), and a probe gives
// up after kPairHashProbes entries (the sample is then deferred as well).
struct DirectRecs {
    static constexpr bool kHashed = false;
    PairRec *R;
    __device__ PairRec *find(int32_t v) const { return R + v; }
    __device__ PairRec *claim(int32_t v) const { return R + v; }
    __device__ int32_t slot(const PairRec *e) const { return (int32_t)(e - R); }
    __device__ PairRec *listed(const Scr &s, int32_t i) const { return R + s.lv[i]; }
    __device__ PairRec *lookup(int32_t v, int32_t *) const { return R + v; }
};

struct HashRecs {
    static constexpr bool kHashed = true;
    PairRec *T;
    uint32_t mask;     // entries - 1
    int32_t shift;     // 32 - log2 entries
    __device__ uint32_t home(int32_t v) const { return ((uint32_t)v * 0x9E3779B1u) >> shift; }
    // the entry of v, or NULL when no side has reached v (or, past the
    // probe limit, when the sample is being deferred anyway)
    __device__ PairRec *find(int32_t v) const {
        uint32_t h = home(v);
        for (int i = 0; i < kPairHashProbes; ++i) {
            const int32_t k = T[h].key;
            if (k == v + 1) return T + h;
            if (k == 0) return nullptr;
            h = (h + 1u) & mask;
        }
        return nullptr;
    }
    // the entry of v, claimed if v has none; NULL past the probe limit
    __device__ PairRec *claim(int32_t v) const {
        uint32_t h = home(v);
        for (int i = 0; i < kPairHashProbes; ++i) {
            int32_t k = T[h].key;
            // the compare-and-swap's old value settles a stale read
            if (k == 0) k = atomicCAS(&T[h].key, 0, v + 1);
            if (k == 0 || k == v + 1) return T + h;
            h = (h + 1u) & mask;
        }
        return nullptr;
    }
    __device__ int32_t slot(const PairRec *e) const { return (int32_t)(e - T); }
    __device__ PairRec *listed(const Scr &s, int32_t i) const { return T + s.ls[i]; }
    // the entry of v, or NULL when no side has reached v; a probe that gives
    // up raises *full (the sample is then deferred)
    __device__ PairRec *lookup(int32_t v, int32_t *full) const {
        uint32_t h = home(v);
        for (int i = 0; i < kPairHashProbes; ++i) {
            const int32_t k = T[h].key;
            if (k == v + 1) return T + h;
            if (k == 0) return nullptr;
            h = (h + 1u) & mask;
        }
        *full = 1;
        return nullptr;
    }
};

// Per-side filters in LDS: one bit per hashed vertex id for every vertex a
// search side has listed (2^kPairFilterLog2 bits a side).  A clear bit
// means the side has not reached the vertex, so its record need not be
// read; a set bit may be a collision.  Vertices written by a probe that
// ends the search are not added (nothing tests them afterwards: every
// later test looks for levels below the meeting level).
constexpr int kPairFilterLog2 = 17;
constexpr int kProbeChunks = 4;
// A level is probed first when at least this many of its arcs are expected
// to meet the other side (Chung-Lu 4M, 300 samples on the CPU: 87% of the
// levels that do not end the search go unprobed, 3 of 300 last levels run
// in full).
constexpr double kProbeMeets = 0.05;
constexpr int kPairFilterWords = 1 << (kPairFilterLog2 - 5);
__device__ __forceinline__ uint32_t filter_bit(int32_t v) {
    return ((uint32_t)v * 0x85EBCA6Bu) >> (32 - kPairFilterLog2);
}
__device__ __forceinline__ void filter_add(uint32_t *f, int32_t v) {
    const uint32_t b = filter_bit(v);
    atomicOr(&f[b >> 5], 1u << (b & 31));
}
__device__ __forceinline__ bool filter_has(const uint32_t *f, int32_t v) {
    const uint32_t b = filter_bit(v);
    return (f[b >> 5] >> (b & 31)) & 1u;
}

// Top-down growth of side X by one level (list[f0, f1) at distance dep)
// into list[f1, ...): every arc y -> z with z not reached by X before this
// level adds sigma_X(y) to sigma_X(z).  The first adder appends z with its
// degree, adds the degree to *newcost, and, when the other side has reached
// z, appends z to the meeting list (meet, *nm).  One record per vertex
// holds the degree, so a reached vertex costs its record's line only; its
// arc range is read when (if ever) its level is expanded.  Hash-table
// entries hold no degree: the row pointers give it, and the arc range is
// listed with the vertex.  Side 1 - X does not change during the level, so its
// distance is read with side X's.
template <int BLOCK, class Recs>
__device__ void pair_level(const Params &p, Tile<BLOCK> &sm, BiState &bs, const Recs &R, int X, const Scr &s,
                           const GView &g, int32_t f0, int32_t f1, int32_t dep, int32_t *meet, int32_t *nm,
                           unsigned long long *newcost, int32_t lcap, int32_t *full, bool count_arcs,
                           uint32_t *filt, Counters &c) {
    const int tid = threadIdx.x;
    unsigned long long dsum = 0;
    // sum of the path counts the level adds (= of its vertices' counts)
    unsigned long long tsum = 0;
    bool tover = false;
    for (int32_t tb = f0; tb < f1; tb += BLOCK) {
        const int32_t cnt = min(BLOCK, f1 - tb);
        if (tid < cnt) sm.val.u[tid] = R.listed(s, tb + tid)->sig[X];
        const int32_t total =
            Recs::kHashed ? stage_list<BLOCK>(sm, s, tb, cnt) : stage_ids<BLOCK>(sm, s.lv, g, tb, cnt);
        __syncthreads();
        if (tid == 0 && count_arcs) c.arcs_fwd += (unsigned long long)total;
        for (int32_t rb = 0; rb < total; rb += BLOCK * kChunk) {
            int32_t kk[kChunk], w[kChunk];
            load_chunk<BLOCK>(sm, g, cnt, total, rb + tid * kChunk, kk, w);
            bool act[kChunk];
            unsigned long long add[kChunk], old[kChunk];
            PairRec *e[kChunk];
            int32_t dother[kChunk], deg[kChunk];
#pragma unroll
            for (int j = 0; j < kChunk; ++j) {
                e[j] = kk[j] >= 0 ? R.claim(w[j]) : nullptr;
                if (Recs::kHashed && kk[j] >= 0 && !e[j]) *full = 1;
                // d[0], d[1] and the degree (one record per vertex) in one load
                const int4 q = e[j] ? *reinterpret_cast<const int4 *>(e[j]->d) : make_int4(0, 0, 0, 0);
                const int32_t dz = X == 0 ? q.x : q.y;
                dother[j] = X == 0 ? q.y : q.x;
                deg[j] = q.z;
                // unreached, or reached on this very level by another adder
                act[j] = e[j] != nullptr && (dz < 0 || dz == dep + 1);
                add[j] = act[j] ? sm.val.u[kk[j]] : 0ULL;
            }
#pragma unroll
            for (int j = 0; j < kChunk; ++j) old[j] = act[j] ? atomicAdd(&e[j]->sig[X], add[j]) : 1ULL;
#pragma unroll
            for (int j = 0; j < kChunk; ++j) {
                const bool fresh = act[j] && old[j] == 0ULL;
                int32_t a0 = 0, dg = 0;
                bool met = false;
                if (act[j]) {
                    c.dag++;
                    if (old[j] + add[j] < old[j]) atomicOr(&p.st->err, kErrOverflow);
                    tsum += add[j];
                    if (tsum < add[j]) tover = true;
                }
                if (fresh) {
                    e[j]->d[X] = dep + 1;
                    filter_add(filt, w[j]);
                    if (Recs::kHashed) {
                        a0 = g.rp[w[j]];
                        dg = g.rp[w[j] + 1] - a0;
                    } else {
                        dg = deg[j];
                    }
                    met = dother[j] >= 0;
                    dsum += (unsigned long long)dg;
                }
                const int32_t pos = wave_append_pos(fresh, w[j], s.lv + f1, &sm.count, lcap - f1, &p.st->err);
                if (Recs::kHashed && pos >= 0) {
                    s.la[f1 + pos] = a0;
                    s.ld[f1 + pos] = dg;
                    s.ls[f1 + pos] = R.slot(e[j]);
                }
                // meeting vertices: new on side X and already reached by the other side
                wave_append(met, w[j], meet, nm, lcap, &p.st->err);
            }
        }
        __syncthreads();
    }
    dsum = wave_sum<unsigned long long>(dsum);
    if (lane_id() == 0 && dsum) atomicAdd(newcost, dsum);
    if (tsum) {
        const unsigned long long o = atomicAdd(&bs.tsum, tsum);
        if (o + tsum < o) tover = true;
    }
    if (tover) bs.tover = 1;
}

// The arcs leaving side X's deepest level (list[f0, f1) at distance dep)
// when the next level may be the last: only vertices the other side has
// already reached (the meeting set M) are written -- path count, distance,
// appended to meet -- exactly as the full level would write them; every
// other vertex of that level is left untouched, and only targets the other
// side's filter lets through have their records read.  If M comes out
// empty nothing was written and the full level runs.  Almost all of a
// sample's reached vertices sit in its last level (Chung-Lu 4M: 95%,
// against about 30 in M), so that level costs little beyond its column
// indices.  The full level's overflow
// check is kept by running this only while the deepest level's counts sum
// below 2^64: on a simple graph no count of the next level can then reach
// it.
template <int BLOCK, class Recs>
__device__ void pair_probe(const Params &p, Tile<BLOCK> &sm, const Recs &R, int X, const Scr &s, const GView &g,
                           int32_t f0, int32_t f1, int32_t dep, int32_t *meet, int32_t *nm, int32_t lcap,
                           int32_t *full, const uint32_t *other, Counters &c) {
    const int tid = threadIdx.x;
    for (int32_t tb = f0; tb < f1; tb += BLOCK) {
        const int32_t cnt = min(BLOCK, f1 - tb);
        if (tid < cnt) sm.val.u[tid] = R.listed(s, tb + tid)->sig[X];
        const int32_t total =
            Recs::kHashed ? stage_list<BLOCK>(sm, s, tb, cnt) : stage_ids<BLOCK>(sm, s.lv, g, tb, cnt);
        __syncthreads();
        if (tid == 0) c.arcs_fwd += (unsigned long long)total;
        // most arcs end at a clear filter bit: U chunks of column indices
        // are loaded at once, then each chunk is settled (hash tables: one,
        // their probe loops need the registers)
        constexpr int U = Recs::kHashed ? 1 : kProbeChunks;
        for (int32_t rb = 0; rb < total; rb += BLOCK * kChunk * U) {
            int32_t kkq[U][kChunk], wq[U][kChunk];
#pragma unroll
            for (int u = 0; u < U; ++u)
                load_chunk<BLOCK>(sm, g, cnt, total, rb + (u * BLOCK + tid) * kChunk, kkq[u], wq[u]);
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int32_t(&kk)[kChunk] = kkq[u];
                const int32_t(&w)[kChunk] = wq[u];
                bool hit[kChunk];
                unsigned long long add[kChunk], old[kChunk];
                PairRec *e[kChunk];
#pragma unroll
                for (int j = 0; j < kChunk; ++j) {
                    // only vertices the other side may have reached are looked up
                    e[j] = kk[j] >= 0 && filter_has(other, w[j]) ? R.lookup(w[j], full) : nullptr;
                    const int4 q = e[j] ? *reinterpret_cast<const int4 *>(e[j]->d) : make_int4(-1, -1, 0, 0);
                    const int32_t dz = X == 0 ? q.x : q.y, dy = X == 0 ? q.y : q.x;
                    // reached by the other side, and by X not before this level
                    hit[j] = e[j] != nullptr && dy >= 0 && (dz < 0 || dz == dep + 1);
                    add[j] = hit[j] ? sm.val.u[kk[j]] : 0ULL;
                }
#pragma unroll
                for (int j = 0; j < kChunk; ++j) old[j] = hit[j] ? atomicAdd(&e[j]->sig[X], add[j]) : 1ULL;
#pragma unroll
                for (int j = 0; j < kChunk; ++j) {
                    const bool fresh = hit[j] && old[j] == 0ULL;
                    if (hit[j]) {
                        c.dag++;
                        if (old[j] + add[j] < old[j]) atomicOr(&p.st->err, kErrOverflow);
                    }
                    if (fresh) e[j]->d[X] = dep + 1;
                    wave_append(fresh, w[j], meet, nm, lcap, &p.st->err);
                }
            }
        }
        __syncthreads();
    }
}

// Walk from `from` to the root `rootv` of search side X, all threads of
// the block together (the same choice as the oracle's walk: at w, step t,
// r = bounded(draw(seed, stream, j, t), sigma[w]) and the first neighbour
// in adjacency order one level closer to the root whose running sigma sum
// exceeds r).  Each iteration covers kWalkArcs * BLOCK consecutive arcs of
// w, kWalkArcs per thread in order: per-thread sums, a wave scan, the wave
// totals in LDS; the first thread whose running sum crosses r finds the
// arc among its own.  A vertex one level from the root has the root as its
// only predecessor.  Thread 0 calls emit(i, vertex) for step i = 1, 2, ...,
// the root included.  Returns false if no predecessor is found (only after
// a reported overflow).
constexpr int kWalkArcs = 4;

template <int BLOCK, class Recs, typename Emit>
__device__ bool walk_block(const Params &p, BiState &bs, const Recs &R, int X, const uint32_t *filt, const GView &g,
                           int32_t from, int32_t rootv, unsigned long long stream, long long j, Emit emit) {
    constexpr int NW = BLOCK / kWave;
    const int tid = threadIdx.x, lane = lane_id(), wid = wave_id();
    int32_t x = from;
    for (unsigned long long tt = 0;; ++tt) {
        // x's arc range is read together with its record
        const int32_t a0 = g.rp[x], a1 = g.rp[x + 1];
        const PairRec *ex = R.find(x);
        if (!ex) return false;
        const int32_t dx = ex->d[X];
        if (dx <= 0) return true;
        if (dx == 1) {
            if (tid == 0) emit((int32_t)tt + 1, rootv);
            return true;
        }
        const unsigned long long r = bounded(draw(p.seed, stream, (unsigned long long)j, tt), ex->sig[X]);
        unsigned long long carry = 0ULL;
        int32_t pick = -1;
        for (int32_t base = a0; base < a1; base += BLOCK * kWalkArcs) {
            const int32_t e0 = base + tid * kWalkArcs;
            int32_t pp[kWalkArcs];
            unsigned long long sp[kWalkArcs];
#pragma unroll
            for (int q = 0; q < kWalkArcs; ++q) pp[q] = e0 + q < a1 ? g.ci[e0 + q] : -1;
#pragma unroll
            for (int q = 0; q < kWalkArcs; ++q) {
                sp[q] = 0ULL;
                // a predecessor is listed on side X: its filter bit is set
                if (pp[q] >= 0 && filter_has(filt, pp[q])) {
                    const PairRec *ep = R.find(pp[q]);
                    if (ep && ep->d[X] == dx - 1) sp[q] = ep->sig[X];
                }
            }
            unsigned long long tsum = 0ULL;
#pragma unroll
            for (int q = 0; q < kWalkArcs; ++q) tsum += sp[q];
            const unsigned long long incl = wave_incl_scan<unsigned long long>(tsum);
            if (lane == kWave - 1) bs.part_lo[wid] = incl;
            if (tid == 0) bs.pickw = NW;
            __syncthreads();
            unsigned long long before = carry, total = carry;
#pragma unroll
            for (int w = 0; w < NW; ++w) {
                const unsigned long long ws = bs.part_lo[w];
                if (w < wid) before += ws;
                total += ws;
            }
            // running sums are non-decreasing: the first thread whose
            // inclusive sum passes r holds the chosen arc
            const unsigned long long mask = __ballot(before + incl > r);
            if (lane == 0 && mask) atomicMin(&bs.pickw, wid);
            __syncthreads();
            const int pw = bs.pickw;
            if (pw < NW) {
                if (wid == pw && lane == __ffsll((long long)mask) - 1) {
                    unsigned long long run = before + incl - tsum;
                    int32_t chosen = -1;
#pragma unroll
                    for (int q = 0; q < kWalkArcs; ++q) {
                        run += sp[q];
                        if (chosen < 0 && run > r) chosen = pp[q];
                    }
                    bs.pickv = chosen;
                }
                __syncthreads();
                pick = bs.pickv;
                break;
            }
            carry = total;
        }
        if (pick < 0) return false;
        if (tid == 0) emit((int32_t)tt + 1, pick);
        x = pick;
    }
}

// One pair sample by balanced bidirectional search, the procedure of the
// oracle's sample_one: grow the side with fewer arcs leaving its deepest
// level by one top-down level (side A on ties); stop at the first new
// level holding vertices the other side already reached (set M), or when a
// side's new level is empty (v unreachable).  z in M is drawn with
// probability sigma_A(z) sigma_B(z) / sigma_uv -- the first z in
// increasing original id whose running weight exceeds the draw, found by a
// binary search on the id threshold with one block reduction per step --
// then the block walks z -> v on side B (draw stream 5) and z -> u on side
// A (stream 3).  Interior vertices are counted and, for inspection, written
// from v's side towards u.  The records of every listed vertex are reset at
// the end, so the next sample starts from unreached records.
template <int BLOCK, class Recs>
__device__ void bidir_sample(const Params &p, Tile<BLOCK> &sm, BiState &bs, const Recs &R, uint32_t *filt,
                             const Scr &sa, const Scr &sb, const GView &g, int32_t u, int32_t v, long long j,
                             long long task, int32_t lcap, Counters &c) {
    const int tid = threadIdx.x;
    if (tid == 0) bs.full = 0;
    for (int i = tid; i < 2 * kPairFilterWords; i += BLOCK) filt[i] = 0u;
    __syncthreads();
    if (tid < 2) {
        // (one thread claims each root: u != v, and an empty table has room)
        const Scr &x = tid == 0 ? sa : sb;
        const int32_t r = tid == 0 ? u : v;
        const int32_t a0 = g.rp[r], dg = g.rp[r + 1] - a0;
        PairRec *er = R.claim(r);
        er->sig[tid] = 1ULL;
        er->d[tid] = 0;
        x.lv[0] = r;
        x.la[0] = a0;
        x.ld[0] = dg;
        if (Recs::kHashed) x.ls[0] = R.slot(er);
        bs.lo[tid] = 0;
        bs.hi[tid] = 1;
        bs.depth[tid] = 0;
        bs.cost[tid] = dg;
        bs.dsum[tid] = dg;
        bs.small[tid] = 1;
        filter_add(filt + tid * kPairFilterWords, r);
    }
    if (tid == 0) {
        bs.result = 0;
        bs.nm = 0;
        bs.pad = 0;   // set when any weight or partial sum wraps
    }
    __syncthreads();
    sub_start<BLOCK>(sm);

    // ---- search
    while (bs.result == 0) {
        const int X = bs.cost[0] <= bs.cost[1] ? 0 : 1;
        const Scr &sx = X == 0 ? sa : sb;
        const int32_t lo = bs.lo[X], hi = bs.hi[X], dep = bs.depth[X];
        // probe when the level may well be the last: the arcs leaving X's
        // frontier times the share of all arcs that belong to vertices the
        // other side has listed is the expected number of arcs that meet
        const bool probed = bs.small[X] != 0 &&
                            (double)bs.cost[X] * (double)bs.dsum[1 - X] >= kProbeMeets * (double)g.m;
        if (probed) {
            // the meeting set first; a last level ends the search here
            pair_probe<BLOCK>(p, sm, R, X, sx, g, lo, hi, dep, sa.cand, &bs.nm, lcap, &bs.full,
                              filt + (1 - X) * kPairFilterWords, c);
            __syncthreads();
            const bool deferred = Recs::kHashed && bs.full;
            const bool met = bs.nm > 0;
            __syncthreads();
            if (deferred || met) {
                if (tid == 0) {
                    bs.result = deferred ? -4 : 1;
                    c.td++;
                }
                __syncthreads();
                break;
            }
        }
        // hashed records: a level that could take the table past half full
        // (each arc leaving the frontier may add a vertex) is not run
        if (Recs::kHashed && (long long)bs.hi[0] + bs.hi[1] + bs.cost[X] > (long long)(lcap >> 1)) {
            __syncthreads();
            if (tid == 0) bs.result = -4;
            __syncthreads();
            break;
        }
        __syncthreads();
        if (tid == 0) {
            sm.count = 0;
            bs.newcost = 0;
            bs.tsum = 0;
            bs.tover = 0;
            c.td++;
        }
        __syncthreads();
        pair_level<BLOCK>(p, sm, bs, R, X, sx, g, lo, hi, dep, sa.cand, &bs.nm,
                          reinterpret_cast<unsigned long long *>(&bs.newcost), lcap, &bs.full, !probed,
                          filt + X * kPairFilterWords, c);
        __syncthreads();
        const int32_t nnew = sm.count < lcap - hi ? sm.count : lcap - hi;
        if (tid == 0) {
            bs.lo[X] = hi;
            bs.hi[X] = hi + nnew;
            bs.depth[X] = dep + 1;
            bs.cost[X] = bs.newcost;
            bs.dsum[X] += bs.newcost;
            bs.small[X] = bs.tover ? 0 : 1;
            // hashed records: a full table, or one past half full (long
            // probes), leaves the sample to the one-record-per-vertex launch
            if (Recs::kHashed && (bs.full || bs.hi[0] + bs.hi[1] > (lcap >> 1)))
                bs.result = -4;
            else if (nnew == 0)
                bs.result = -1;
            else if (bs.nm > 0)
                bs.result = 1;
        }
        __syncthreads();
    }
    if (tid == 0) c.reached += (unsigned long long)(bs.hi[0] + bs.hi[1]);
    sub_mark<BLOCK>(sm, kSbPairSearch);

    // ---- meeting vertex
    if (bs.result == 1) {
        const int32_t nm = bs.nm;
        unsigned long long *wt = reinterpret_cast<unsigned long long *>(sa.dacc);
        unsigned long long mine = 0ULL;
        bool wrap = false;
        int32_t idlo = 0x7fffffff, idhi = -1;
        for (int32_t i = tid; i < nm; i += BLOCK) {
            const int32_t z = sa.cand[i];
            const PairRec *ez = R.find(z);
            const unsigned long long a = ez->sig[0], b = ez->sig[1];
            const unsigned long long w = a * b;
            if (__umul64hi(a, b) != 0ULL) wrap = true;
            wt[i] = w;
            const unsigned long long nw = mine + w;
            if (nw < mine) wrap = true;
            mine = nw;
            const int32_t oid = p.inv ? p.inv[z] : z;
            idlo = min(idlo, oid);
            idhi = max(idhi, oid);
            // one entry per thread when M fits the block: ids and weights in
            // the tile (its arrays are free once the search has ended)
            if (nm <= BLOCK) {
                sm.v[tid] = oid;
                sm.val.u[tid] = w;
            }
        }
        if (wrap) {
            atomicOr(&p.st->err, kErrOverflow);
            bs.pad = 1;
        }
        unsigned long long tlo, thi;
        block_sum_u128<BLOCK>(mine, bs, tlo, thi);   // its barriers publish bs.pad
        const bool anywrap = bs.pad != 0;             // block-uniform from here on
        // id range of M for the threshold search
        idlo = wave_min(idlo);
        idhi = -wave_min(-idhi);
        if (tid == 0) {
            sm.redmin = 0x7fffffff;
            sm.levels = -1;
        }
        __syncthreads();
        if (lane_id() == 0) {
            atomicMin(&sm.redmin, idlo);
            atomicMax(&sm.levels, idhi);
        }
        __syncthreads();
        int32_t tlo_id = sm.redmin, thi_id = sm.levels;
        __syncthreads();
        if (thi != 0ULL || anywrap) {
            if (tid == 0) {
                bs.result = -3;
                atomicOr(&p.st->err, kErrOverflow);
            }
        } else {
            const unsigned long long r0 = bounded(draw(p.seed, 4, (unsigned long long)j, 0), tlo);
            if (nm <= BLOCK) {
                // the z whose weights of smaller ids sum to at most r0 and,
                // with its own weight, above it (ids are distinct and the
                // total is below 2^64): one thread finds itself.  Weights of
                // zero (counts that wrapped, already reported as overflow)
                // can leave no such z; then z is the largest id, as the
                // threshold search would end, so that z is always a vertex.
                if (tid < nm && sm.v[tid] == thi_id) bs.z = sa.cand[tid];
                __syncthreads();
                if (tid < nm) {
                    const int32_t me = sm.v[tid];
                    unsigned long long below = 0ULL;
                    for (int32_t k = 0; k < nm; ++k)
                        if (sm.v[k] < me) below += sm.val.u[k];
                    if (below <= r0 && r0 - below < mine) bs.z = sa.cand[tid];
                }
                tlo_id = thi_id;   // the threshold search below has nothing to do
            }
            // smallest original-id threshold T with sum of weights of ids <= T above r0
            while (tlo_id < thi_id) {
                const int32_t mid = tlo_id + ((thi_id - tlo_id) >> 1);
                unsigned long long part = 0ULL;
                for (int32_t i = tid; i < nm; i += BLOCK) {
                    const int32_t z = sa.cand[i];
                    const int32_t oid = p.inv ? p.inv[z] : z;
                    if (oid <= mid) part += wt[i];
                }
                unsigned long long flo, fhi;
                block_sum_u128<BLOCK>(part, bs, flo, fhi);
                if (flo > r0)
                    thi_id = mid;
                else
                    tlo_id = mid + 1;
            }
            for (int32_t i = tid; i < nm && nm > BLOCK; i += BLOCK) {
                const int32_t z = sa.cand[i];
                if ((p.inv ? p.inv[z] : z) == tlo_id) bs.z = z;
            }
        }
        __syncthreads();
    }
    sub_mark<BLOCK>(sm, kSbPairSelect);
    // ---- walks (all threads; thread 0 records)
    if (bs.result == -4) {
        // left for the launch with one record per vertex
    } else if (bs.result == -1) {
        if (tid == 0 && p.p_len) p.p_len[task] = -1;
    } else if (bs.result == -3) {
        if (tid == 0 && p.p_len) p.p_len[task] = -3;
    } else {
        const int32_t z = bs.z;
        const PairRec *ez = R.find(z);
        const int32_t kb = ez->d[1], ha = ez->d[0];
        const int32_t nb = kb >= 1 ? kb - 1 : 0;
        const int32_t zc = (kb >= 1 && ha >= 1) ? 1 : 0;
        const int32_t len = nb + zc + (ha >= 1 ? ha - 1 : 0);
        auto put = [&](int32_t pos, int32_t vtx) {
            if (p.counts) atomicAdd(&p.counts[vtx], 1u);
            if (p.p_path && pos < p.maxlen) p.p_path[task * p.maxlen + pos] = p.inv ? p.inv[vtx] : vtx;
        };
        // side B: steps 1 .. kb-1 are interior, listed from v's side
        bool ok = walk_block<BLOCK>(p, bs, R, 1, filt + kPairFilterWords, g, z, v, 5, j,
                                    [&](int32_t i, int32_t vtx) {
                                        if (i < kb) put(kb - 1 - i, vtx);
                                    });
        if (tid == 0 && zc) put(nb, z);
        if (ok)
            ok = walk_block<BLOCK>(p, bs, R, 0, filt, g, z, u, 3, j, [&](int32_t i, int32_t vtx) {
                if (i < ha) put(nb + zc + i - 1, vtx);
            });
        if (!ok && tid == 0) atomicOr(&p.st->err, kErrInternal);
        if (tid == 0 && p.p_len) p.p_len[task] = !ok ? -3 : (len > p.maxlen ? -2 : len);
    }
    __syncthreads();
    sub_mark<BLOCK>(sm, kSbPairWalk);

    // ---- reset the records of every listed vertex (both sides); hashed
    // records also free their entries (no probe runs any more)
    // (four list entries per thread at a time, their loads issued together)
    for (int k = 0; k < 2; ++k) {
        const Scr &x = k == 0 ? sa : sb;
        const int32_t hk = bs.hi[k];
        for (int32_t i0 = tid; i0 < hk; i0 += 4 * BLOCK) {
            PairRec *rc[4];
#pragma unroll
            for (int q = 0; q < 4; ++q) rc[q] = i0 + q * BLOCK < hk ? R.listed(x, i0 + q * BLOCK) : nullptr;
#pragma unroll
            for (int q = 0; q < 4; ++q) {
                if (rc[q]) {
                    rc[q]->sig[0] = 0ULL;
                    rc[q]->sig[1] = 0ULL;
                    rc[q]->d[0] = -1;
                    rc[q]->d[1] = -1;
                    if (Recs::kHashed) rc[q]->key = 0;
                }
            }
        }
    }
    __syncthreads();
    sub_mark<BLOCK>(sm, kSbPairClear);
}

// ------------------------------------------------------------ the kernel --

template <int BLOCK, bool BMLDS, int MODE>
__global__ __launch_bounds__(BLOCK) void k_brandes(Params p) {
    extern __shared__ uint32_t lds_bm[];
    __shared__ Tile<BLOCK> sm;
    __shared__ BiState bs;
    const int tid = threadIdx.x;
    if (tid == 0) sm.flag = p.st->err & kErrGraph;
    __syncthreads();
    if (sm.flag) return;
    __syncthreads();

    const long long slot = blockIdx.x;
    const long long off = slot * p.stride;
    constexpr bool PAIR = MODE == kModePair || MODE == kModePairHash;
    Scr s;
    // pair mode keeps its path counts and distances in records instead
    s.sigma = PAIR ? nullptr : p.sigma + off;
    s.dacc = p.dacc + off;
    s.ldeg = PAIR ? nullptr : p.ldeg + off;
    s.d = PAIR ? nullptr : p.d + off;
    s.lv = p.lv + off;
    s.la = p.la + off;
    s.ld = p.ld + off;
    s.lvl = PAIR ? nullptr : p.lvl + off;
    s.cand = p.cand + off;
    s.dist = p.dist ? p.dist + off : nullptr;
    s.mark = p.mark ? p.mark + off : nullptr;
    s.wl0 = p.wl0 ? p.wl0 + off : nullptr;
    s.wl1 = p.wl1 ? p.wl1 + off : nullptr;
    s.wl2 = p.wl2 ? p.wl2 + off : nullptr;
    s.dagm = p.dagm ? p.dagm + slot * p.dag_words : nullptr;
    s.bvec = p.bvec ? p.bvec + off * kBisK : nullptr;
    uint32_t *bm = (BMLDS || PAIR) ? lds_bm : p.bmg + slot * p.bm_words;
    // pair mode: per-vertex records of both search sides, and the target
    // side's level lists
    s.ls = MODE == kModePairHash ? p.ls + off : nullptr;
    Scr s2 = s;
    PairRec *rec = nullptr;
    if (PAIR) {
        rec = reinterpret_cast<PairRec *>(p.pair_rec) + slot * p.stride;
        s2.lv = p.lv2 + slot * p.stride;
        s2.la = p.la2 + slot * p.stride;
        s2.ld = p.ld2 + slot * p.stride;
        s2.ls = MODE == kModePairHash ? p.ls2 + slot * p.stride : nullptr;
    }

    Counters c = {0, 0, 0, 0, 0, 0, 0, 0, 0};
    if (tid < 8) {
        sm.cyc[tid] = 0;
        sm.sub[tid] = 0;
    }
    __syncthreads();
    const long long t_kernel = clock64();
    int32_t ep = 0;                                   // weighted mode: round counter
    __shared__ unsigned long long wsd[MODE == kModeWeighted ? BLOCK : 1];   // distances of staged vertices
    // pair modes: the two search sides' filters
    __shared__ uint32_t pfilt[MODE == kModePair || MODE == kModePairHash ? 2 * kPairFilterWords : 1];
    (void)ep;
    (void)wsd;
    (void)pfilt;
    for (;;) {
        if (tid == 0) sm.task = (long long)atomicAdd(&p.st->head, 1ULL);
        __syncthreads();
        const long long task = sm.task;
        __syncthreads();
        if (task >= p.ntasks) break;

        GView g;
        int32_t src = 0, target = -1;
        long long j = 0;
        if (p.G > 0) {
            int32_t lo = 0, hi = p.G - 1;
            while (lo < hi) {
                const int32_t mid = (lo + hi + 1) >> 1;
                if (p.g_task[mid] <= task) lo = mid; else hi = mid - 1;
            }
            const int32_t gid = p.g_order[lo];
            const long long v0 = p.g_vtx[gid];
            g.rp = p.rowptr + v0 + gid;
            g.ci = p.colidx + p.g_arc[gid];
            g.n = (int32_t)(p.g_vtx[gid + 1] - v0);
            g.m = (int32_t)(p.g_arc[gid + 1] - p.g_arc[gid]);
            g.vbase = v0;
            g.trp = g.rp;
            g.tci = g.ci;
            src = (int32_t)(task - p.g_task[lo]);
        } else {
            g.rp = p.rowptr;
            g.ci = p.colidx;
            g.n = p.n;
            g.m = p.m;
            g.vbase = 0;
            g.trp = p.trowptr ? p.trowptr : p.rowptr;
            g.tci = p.trowptr ? p.tcolidx : p.colidx;
            if (PAIR) {
                // the sample this task runs (a task list maps tasks to samples)
                const long long tt = p.task_list ? p.task_list[task] : task;
                j = p.j0 + tt;
                const int32_t a = (int32_t)bounded(draw(p.seed, 1, (unsigned long long)j, 0), (unsigned long long)p.n);
                int32_t b = (int32_t)bounded(draw(p.seed, 2, (unsigned long long)j, 0), (unsigned long long)(p.n - 1));
                if (b >= a) b += 1;
                if (tid == 0 && p.p_uv) {
                    p.p_uv[2 * tt] = a;
                    p.p_uv[2 * tt + 1] = b;
                }
                src = p.perm ? p.perm[a] : a;
                target = p.perm ? p.perm[b] : b;
            } else {
                src = p.sources ? p.sources[task] : (int32_t)task;
            }
        }
        if (src < 0 || src >= g.n) {
            if (tid == 0) atomicOr(&p.st->err, kErrArg);
            continue;
        }
        if constexpr (PAIR) {
            const long long tt = j - p.j0;
            // an isolated endpoint leaves the pair unreachable
            if (g.rp[target + 1] == g.rp[target] || g.rp[src + 1] == g.rp[src]) {
                if (tid == 0 && p.p_len) p.p_len[tt] = -1;
                if (tid == 0) {
                    c.tasks++;
                    atomicAdd(&p.st->stat[kStDone], 1ULL);
                }
                continue;
            }
            phase_start<BLOCK>(sm);
            // work counters count finished samples only (a deferred one is
            // counted by the launch that runs it)
            const Counters c0 = c;
            if constexpr (MODE == kModePairHash) {
                const HashRecs hr{rec, (1u << p.ph_log2) - 1u, 32 - p.ph_log2};
                bidir_sample<BLOCK>(p, sm, bs, hr, pfilt, s, s2, g, src, target, j, tt,
                                    (int32_t)min<long long>(p.stride, g.n), c);
            } else {
                bidir_sample<BLOCK>(p, sm, bs, DirectRecs{rec}, pfilt, s, s2, g, src, target, j, tt, g.n, c);
            }
            if (bs.result == -4) c = c0;
            if (tid == 0) {
                if (bs.result == -4) {
                    // too many vertices for the table: a later launch with one
                    // record per vertex runs this sample
                    const unsigned long long q = atomicAdd(p.defer_count, 1ULL);
                    p.defer[q] = tt;
                    atomicAdd(&p.st->stat[kStDeferred], 1ULL);
                } else {
                    c.tasks++;
                    atomicAdd(&p.st->stat[kStDone], 1ULL);
                }
            }
            phase_end<BLOCK>(sm, kPhTd);
            continue;
        } else if constexpr (MODE == kModeWeighted) {
            phase_start<BLOCK>(sm);
            const int32_t nreach = w_distances<BLOCK>(p, sm, bm, s, g, src, ep, wsd, c);
            phase_end<BLOCK>(sm, kPhTd);
            phase_start<BLOCK>(sm);
            // the distance-bucket histogram sits at the start of the dynamic
            // LDS (the settled bitmap's place when that is in LDS; it is not
            // needed past the distance rounds)
            const int32_t Ld = w_layers<BLOCK>(p, sm, s, g, src, nreach, reinterpret_cast<int32_t *>(lds_bm), wsd, c);
            phase_end<BLOCK>(sm, kPhBu);
            phase_start<BLOCK>(sm);
            // the rows' ends of the sweep's tiles go where the staged
            // distances were
            w_backward<BLOCK>(sm, s, g, Ld, p.bc, reinterpret_cast<int32_t *>(wsd), c);
            phase_end<BLOCK>(sm, kPhPull);
            phase_start<BLOCK>(sm);
            for (int32_t i = tid; i < nreach; i += BLOCK) {
                const int32_t v = s.cand[i];
                s.sigma[v] = 0ULL;
                s.dist[v] = kInf;
            }
            {
                // the sweep cleared the DAG bits of every layer but the
                // source's; the words of the source's arcs hold no others now
                const int32_t a = g.rp[src], b = g.rp[src + 1];
                if (b > a)
                    for (int32_t wd = (a >> 5) + tid; wd <= ((b - 1) >> 5); wd += BLOCK) s.dagm[wd] = 0u;
            }
            if (tid == 0) {
                c.reached += (unsigned long long)nreach;
                c.tasks++;
                atomicAdd(&p.st->stat[kStDone], 1ULL);
            }
            __syncthreads();
            phase_end<BLOCK>(sm, kPhReset);
            continue;
        } else {

        const int32_t Ld = forward<BLOCK, MODE>(p, sm, bm, s, g, p.G > 0 ? nullptr : p.iso, src, c);
        const int32_t nreached = s.lvl[Ld + 1];
        if (tid == 0) {
            c.reached += (unsigned long long)nreached;
            c.tasks++;
        }

        if (MODE == kModeClose) {
            if (p.close_out && tid == 0) {
                // distance sum from the level sizes; generalised closeness
                long long far = 0;
                for (int32_t l = 1; l <= Ld; ++l) far += (long long)l * (s.lvl[l + 1] - s.lvl[l]);
                const int32_t o = p.inv ? p.inv[src] : src;
                p.close_out[o] = (nreached <= 1 || g.n <= 1)
                                     ? 0.0
                                     : ((double)(nreached - 1) / (double)(g.n - 1)) *
                                           ((double)(nreached - 1) / (double)far);
            }
            if (p.close_acc) {
                for (int32_t l = 1; l <= Ld; ++l)
                    for (int32_t i = s.lvl[l] + tid; i < s.lvl[l + 1]; i += BLOCK)
                        atomicAdd(p.close_acc + s.lv[i], (unsigned long long)l);
            }
        } else if (MODE == kModeBC || MODE == kModeBisect) {
            backward<BLOCK, MODE == kModeBisect>(p, sm, bm, s, g, Ld, p.bc + g.vbase, c);
        } else if (MODE == kModeSSSP) {
            const long long row = task * (long long)g.n;
            for (int32_t i = tid; i < nreached; i += BLOCK) {
                const int32_t v = s.lv[i];
                const int32_t o = p.inv ? p.inv[v] : v;
                p.d_out[row + o] = s.d[v];
                p.sigma_out[row + o] = s.sigma[v];
            }
        }
        __syncthreads();
        phase_start<BLOCK>(sm);
        for (int32_t i = tid; i < nreached; i += BLOCK) s.sigma[s.lv[i]] = 0ULL;
        if (tid == 0) atomicAdd(&p.st->stat[kStDone], 1ULL);
        __syncthreads();
        phase_end<BLOCK>(sm, kPhReset);
        }  // non-pair modes
    }

    // counters: wave sums, one atomic per wave and counter
    unsigned long long dag = wave_sum<unsigned long long>(c.dag);
    if (lane_id() == 0) atomicAdd(&p.st->stat[kStDag], dag);
    // (every thread of the weighted sweep counts its own rows' arcs)
    unsigned long long abw = wave_sum<unsigned long long>(c.arcs_bwd);
    if (lane_id() == 0) atomicAdd(&p.st->stat[kStArcsBwd], abw);
    if (tid == 0) {
        atomicAdd(&p.st->stat[kStSources], c.tasks);
        atomicAdd(&p.st->stat[kStReached], c.reached);
        atomicAdd(&p.st->stat[kStArcsFwd], c.arcs_fwd);
        atomicAdd(&p.st->stat[kStTd], c.td);
        atomicAdd(&p.st->stat[kStBu], c.bu);
        atomicAdd(&p.st->stat[kStArcsReached], c.arcs_reached);
        atomicAdd(&p.st->stat[kStBwPush], c.bw_push);
        unsigned long long known = 0;
        for (int i = 0; i < kNumPhases; ++i) {
            if (i != kPhOther) known += sm.cyc[i];
        }
        const unsigned long long total = (unsigned long long)(clock64() - t_kernel);
        sm.cyc[kPhOther] = total > known ? total - known : 0;
        for (int i = 0; i < kNumPhases; ++i) atomicAdd(&p.st->cycles[i], sm.cyc[i]);
        for (int i = 0; i < kNumSub; ++i) atomicAdd(&p.st->sub[i], sm.sub[i]);
    }
}

template <int BLOCK, bool BMLDS, int MODE>
static void launch_brandes(dim3 grid, dim3 block, size_t lds, hipStream_t s, const Params &p) {
    hipLaunchKernelGGL((k_brandes<BLOCK, BMLDS, MODE>), grid, block, lds, s, p);
}

template <int BLOCK, bool BMLDS, int MODE>
static KernelRef ref() {
    return KernelRef{(const void *)&k_brandes<BLOCK, BMLDS, MODE>, &launch_brandes<BLOCK, BMLDS, MODE>};
}

template <int MODE>
static KernelRef ref_mode(int block, bool lds) {
    switch (block) {
        case 256: return lds ? ref<256, true, MODE>() : ref<256, false, MODE>();
        case 512: return lds ? ref<512, true, MODE>() : ref<512, false, MODE>();
        default: return lds ? ref<1024, true, MODE>() : ref<1024, false, MODE>();
    }
}

KernelRef brandes_kernel(int mode, int block, bool bitmap_in_lds) {
    switch (mode) {
        case kModeBC: return ref_mode<kModeBC>(block, bitmap_in_lds);
        case kModeSSSP: return ref_mode<kModeSSSP>(block, bitmap_in_lds);
        case kModePair: return ref_mode<kModePair>(block, bitmap_in_lds);
        case kModePairHash: return ref_mode<kModePairHash>(block, bitmap_in_lds);
        case kModeClose: return ref_mode<kModeClose>(block, bitmap_in_lds);
        case kModeBisect: return ref_mode<kModeBisect>(block, bitmap_in_lds);
        case kModeWeighted: return ref_mode<kModeWeighted>(block, bitmap_in_lds);
        default: return ref_mode<kModeBC>(block, bitmap_in_lds);
    }
}

// ---------------------------------------------------------- small kernels --

__global__ void k_status_init(DevStatus *st) {
    const int t = threadIdx.x;
    if (t == 0) {
        st->err = 0;
        st->pad = 0;
        st->head = 0ULL;
    }
    if (t < kNumStats) st->stat[t] = 0ULL;
    if (t < kNumPhases) st->cycles[t] = 0ULL;
    if (t < 8) st->sub[t] = 0ULL;
    if (t < 8) st->info[t] = (t == 1) ? 0x7fffffff : 0;
}

__global__ void k_validate(const int32_t *rowptr, const int32_t *colidx, int32_t n, int64_t m, DevStatus *st) {
    const long long tid = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const long long stride = (long long)gridDim.x * blockDim.x;
    int bad = 0;
    if (tid == 0 && (rowptr[0] != 0 || (int64_t)rowptr[n] != m)) bad = 1;
    for (long long i = tid; i < n; i += stride)
        if (rowptr[i + 1] < rowptr[i]) bad = 1;
    for (long long e = tid; e < m; e += stride) {
        const int32_t c = colidx[e];
        if (c < 0 || c >= n) bad = 1;
    }
    if (bad) atomicOr(&st->err, kErrGraph);
}

// Simple-graph checks; runs only after the structural checks passed.
__global__ void k_validate_strict(const int32_t *rowptr, const int32_t *colidx, int32_t n, DevStatus *st) {
    if (st->err & kErrGraph) return;
    const long long tid = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    const long long stride = (long long)gridDim.x * blockDim.x;
    int bad = 0;
    for (long long u = tid; u < n; u += stride) {
        const int32_t a0 = rowptr[u], a1 = rowptr[u + 1];
        for (int32_t e = a0; e < a1; ++e) {
            const int32_t v = colidx[e];
            if (v == u || (e > a0 && colidx[e - 1] >= v)) { bad = 1; break; }
            int32_t lo = rowptr[v], hi = rowptr[v + 1];
            bool found = false;
            while (lo < hi) {
                const int32_t mid = (lo + hi) >> 1;
                const int32_t x = colidx[mid];
                if (x == (int32_t)u) { found = true; break; }
                if (x < (int32_t)u) lo = mid + 1; else hi = mid;
            }
            if (!found) { bad = 1; break; }
        }
    }
    if (bad) atomicOr(&st->err, kErrGraph);
}

__global__ void k_validate_weights(const int32_t *wts, long long m, DevStatus *st) {
    const long long stride = (long long)gridDim.x * blockDim.x;
    bool bad = false;
    for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < m; e += stride) bad |= wts[e] < 1;
    if (__ballot(bad) != 0ULL && lane_id() == 0) atomicOr(&st->err, kErrGraph);
}

__global__ void k_sum_weights(const int32_t *wts, long long m, unsigned long long *sum) {
    const long long stride = (long long)gridDim.x * blockDim.x;
    unsigned long long t = 0;
    for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < m; e += stride)
        t += (unsigned long long)(uint32_t)wts[e];
    t = wave_sum<unsigned long long>(t);
    if (lane_id() == 0 && t) atomicAdd(sum, t);
}

__global__ void k_iso_bitmap(const int32_t *rowptr, int32_t n, uint32_t *iso) {
    const int32_t nw = (n + 31) >> 5;
    const int32_t wi = blockIdx.x * blockDim.x + threadIdx.x;
    if (wi >= nw) return;
    uint32_t x = 0;
    for (int b = 0; b < 32; ++b) {
        const int32_t v = wi * 32 + b;
        if (v < n && rowptr[v + 1] == rowptr[v]) x |= 1u << b;
    }
    iso[wi] = x;
}

template <typename T>
__global__ void k_fill(T *p, T v, long long count) {
    const long long stride = (long long)gridDim.x * blockDim.x;
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += stride) p[i] = v;
}

__global__ void k_scale(double *p, double scale, long long count) {
    const long long stride = (long long)gridDim.x * blockDim.x;
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += stride) p[i] *= scale;
}

__global__ void k_counts_to_bc(const uint32_t *cnt, double *bc, double scale, long long count) {
    const long long stride = (long long)gridDim.x * blockDim.x;
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += stride)
        bc[i] = (double)cnt[i] * scale;
}

// key = (degree << 32) | (0xffffffff - id): the maximum is the highest
// degree with the lowest id.
__global__ void k_argmax_degree(const int32_t *rowptr, int32_t n, unsigned long long *key) {
    const long long stride = (long long)gridDim.x * blockDim.x;
    unsigned long long best = 0ULL;
    for (long long v = (long long)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += stride) {
        const unsigned long long dg = (unsigned long long)(rowptr[v + 1] - rowptr[v]);
        const unsigned long long k = (dg << 32) | (0xffffffffULL - (unsigned long long)v);
        best = k > best ? k : best;
    }
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) {
        const unsigned long long y = __shfl_xor(best, off, kWave);
        best = y > best ? y : best;
    }
    // one global atomic per workgroup (same-address atomics serialise)
    __shared__ unsigned long long part[1024 / kWave];
    if (lane_id() == 0) part[wave_id()] = best;
    __syncthreads();
    if (threadIdx.x == 0) {
        for (int w = 1; w < (int)(blockDim.x / kWave); ++w) best = part[w] > best ? part[w] : best;
        atomicMax(key, best);
    }
}

__global__ void k_pair_table_init(PairRec *rec, long long count) {
    const long long stride = (long long)gridDim.x * blockDim.x;
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += stride) {
        rec[i].sig[0] = 0ULL;
        rec[i].sig[1] = 0ULL;
        rec[i].d[0] = -1;
        rec[i].d[1] = -1;
        rec[i].key = 0;
        rec[i].pad = 0;
    }
}

// Record block fill (layout at pair_block_head_bytes): the degree field of
// every record of `slots` slots, and with `full` the unreached state too;
// the row pointers rp[0..n] kept at the head.  Without `full` the launch
// does nothing unless the head was found stale.  Threads walk vertices in
// x and slots in y, so neighbouring threads write neighbouring records.
__global__ void k_pair_block_fill(char *blk, long long slots, long long stride, const int32_t *rp, int32_t n,
                                  int32_t full) {
    int32_t *head = reinterpret_cast<int32_t *>(blk);
    if (!full && head[1] == 0) return;
    int32_t *kept = head + 64;
    PairRec *rec = reinterpret_cast<PairRec *>(blk + pair_block_head_bytes(stride));
    const long long step = (long long)gridDim.x * blockDim.x;
    const long long v0 = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    for (long long v = v0; v < stride; v += step) {
        const int32_t dg = v < n ? rp[v + 1] - rp[v] : 0;
        for (long long sl = blockIdx.y; sl < slots; sl += gridDim.y) {
            PairRec *e = rec + sl * stride + v;
            if (full) {
                e->sig[0] = 0ULL;
                e->sig[1] = 0ULL;
                e->d[0] = -1;
                e->d[1] = -1;
                e->pad = 0;
            }
            e->key = dg;
        }
    }
    if (blockIdx.y == 0) {
        for (long long v = v0; v <= n; v += step) kept[v] = rp[v];
        if (v0 == 0) {
            head[0] = n;
            if (full) head[1] = 0;
        }
    }
}

// Sets the head's stale flag (cleared before) when the kept row pointers
// are not rp[0..n].  The kept array has stride + 1 >= n + 1 entries.
__global__ void k_pair_block_check(char *blk, const int32_t *rp, int32_t n) {
    int32_t *head = reinterpret_cast<int32_t *>(blk);
    const int32_t *kept = head + 64;
    const long long step = (long long)gridDim.x * blockDim.x;
    const long long v0 = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    bool diff = v0 == 0 && head[0] != n;
    for (long long v = v0; v <= n; v += step) diff |= kept[v] != rp[v];
    if (diff) head[1] = 1;
}

__global__ void k_close_finish(const unsigned long long *acc, const int32_t *perm, int32_t n, int32_t k,
                               double *out) {
    const long long stride = (long long)gridDim.x * blockDim.x;
    for (long long o = (long long)blockIdx.x * blockDim.x + threadIdx.x; o < n; o += stride) {
        const unsigned long long a = acc[perm ? perm[o] : o];
        const double F = (double)n / (double)k * (double)a;
        out[o] = F > 0.0 ? (double)(n - 1) / F : 0.0;
    }
}

static inline unsigned grid_for(long long count, int block) {
    long long g = (count + block - 1) / block;
    if (g < 1) g = 1;
    if (g > 65536) g = 65536;
    return (unsigned)g;
}

hipError_t launch_pair_table_init(void *rec, long long count, hipStream_t s) {
    hipLaunchKernelGGL(k_pair_table_init, dim3(grid_for(count, 256)), dim3(256), 0, s,
                       reinterpret_cast<PairRec *>(rec), count);
    return hipGetLastError();
}

// whole slots of a record block of `bytes` bytes
static long long pair_block_slots(size_t bytes, long long stride) {
    const long long head = pair_block_head_bytes(stride);
    return (long long)bytes > head ? ((long long)bytes - head) / (32 * stride) : 0;
}

static hipError_t launch_pair_block_fill(void *blk, size_t bytes, long long stride, const int32_t *rowptr, int32_t n,
                                         int32_t full, hipStream_t s) {
    const long long slots = pair_block_slots(bytes, stride);
    const unsigned gx = grid_for(stride, 256) < 1024 ? grid_for(stride, 256) : 1024;
    const unsigned gy = slots < 8 ? (unsigned)(slots > 0 ? slots : 1) : 8;
    hipLaunchKernelGGL(k_pair_block_fill, dim3(gx, gy), dim3(256), 0, s, reinterpret_cast<char *>(blk), slots, stride,
                       rowptr, n, full);
    return hipGetLastError();
}

hipError_t launch_pair_block_init(void *blk, size_t bytes, long long stride, const int32_t *rowptr, int32_t n,
                                  hipStream_t s) {
    return launch_pair_block_fill(blk, bytes, stride, rowptr, n, 1, s);
}

hipError_t launch_pair_block_refresh(void *blk, size_t bytes, long long stride, const int32_t *rowptr, int32_t n,
                                     hipStream_t s) {
    hipError_t e = launch_fill_i32(reinterpret_cast<int32_t *>(blk) + 1, 0, 1, s);
    if (e != hipSuccess) return e;
    const unsigned g = grid_for((long long)n + 1, 256) < 2048 ? grid_for((long long)n + 1, 256) : 2048;
    hipLaunchKernelGGL(k_pair_block_check, dim3(g), dim3(256), 0, s, reinterpret_cast<char *>(blk), rowptr, n);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    return launch_pair_block_fill(blk, bytes, stride, rowptr, n, 0, s);
}

hipError_t launch_close_finish(const unsigned long long *acc, const int32_t *perm, int32_t n, int32_t k, double *out,
                               hipStream_t s) {
    hipLaunchKernelGGL(k_close_finish, dim3(grid_for(n, 256)), dim3(256), 0, s, acc, perm, n, k, out);
    return hipGetLastError();
}

hipError_t launch_status_init(DevStatus *st, hipStream_t s) {
    hipLaunchKernelGGL(k_status_init, dim3(1), dim3(64), 0, s, st);
    return hipGetLastError();
}

hipError_t launch_validate(const int32_t *rowptr, const int32_t *colidx, int32_t n, int64_t m, int32_t strict,
                           DevStatus *st, hipStream_t s) {
    hipLaunchKernelGGL(k_validate, dim3(grid_for(m > n ? m : n, 256)), dim3(256), 0, s, rowptr, colidx, n, m, st);
    if (strict) hipLaunchKernelGGL(k_validate_strict, dim3(grid_for(n, 256)), dim3(256), 0, s, rowptr, colidx, n, st);
    return hipGetLastError();
}

hipError_t launch_iso_bitmap(const int32_t *rowptr, int32_t n, uint32_t *iso, hipStream_t s) {
    const long long nw = ((long long)n + 31) / 32;
    hipLaunchKernelGGL(k_iso_bitmap, dim3(grid_for(nw, 256)), dim3(256), 0, s, rowptr, n, iso);
    return hipGetLastError();
}

hipError_t launch_fill_f64(double *p, double v, long long count, hipStream_t s) {
    hipLaunchKernelGGL(k_fill<double>, dim3(grid_for(count, 256)), dim3(256), 0, s, p, v, count);
    return hipGetLastError();
}
hipError_t launch_fill_u32(uint32_t *p, uint32_t v, long long count, hipStream_t s) {
    hipLaunchKernelGGL(k_fill<uint32_t>, dim3(grid_for(count, 256)), dim3(256), 0, s, p, v, count);
    return hipGetLastError();
}
hipError_t launch_fill_i32(int32_t *p, int32_t v, long long count, hipStream_t s) {
    hipLaunchKernelGGL(k_fill<int32_t>, dim3(grid_for(count, 256)), dim3(256), 0, s, p, v, count);
    return hipGetLastError();
}
hipError_t launch_fill_u64(unsigned long long *p, unsigned long long v, long long count, hipStream_t s) {
    hipLaunchKernelGGL(k_fill<unsigned long long>, dim3(grid_for(count, 256)), dim3(256), 0, s, p, v, count);
    return hipGetLastError();
}
hipError_t launch_scale_f64(double *p, double scale, long long count, hipStream_t s) {
    hipLaunchKernelGGL(k_scale, dim3(grid_for(count, 256)), dim3(256), 0, s, p, scale, count);
    return hipGetLastError();
}
hipError_t launch_counts_to_bc(const uint32_t *counts, double *bc, double scale, long long count, hipStream_t s) {
    hipLaunchKernelGGL(k_counts_to_bc, dim3(grid_for(count, 256)), dim3(256), 0, s, counts, bc, scale, count);
    return hipGetLastError();
}
hipError_t launch_validate_weights(const int32_t *wts, long long m, DevStatus *st, hipStream_t s) {
    hipLaunchKernelGGL(k_validate_weights, dim3(grid_for(m, 256)), dim3(256), 0, s, wts, m, st);
    return hipGetLastError();
}
hipError_t launch_sum_weights(const int32_t *wts, long long m, unsigned long long *sum, hipStream_t s) {
    const unsigned g = grid_for(m, 256);
    hipLaunchKernelGGL(k_sum_weights, dim3(g < 1024 ? g : 1024), dim3(256), 0, s, wts, m, sum);
    return hipGetLastError();
}
hipError_t launch_argmax_degree(const int32_t *rowptr, int32_t n, unsigned long long *key, hipStream_t s) {
    const unsigned g = grid_for(n, 256);
    hipLaunchKernelGGL(k_argmax_degree, dim3(g < 1024 ? g : 1024), dim3(256), 0, s, rowptr, n, key);
    return hipGetLastError();
}

}  // namespace nk
