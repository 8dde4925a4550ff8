// Multi-source Brandes kernel: one workgroup runs B sources at once.
//
// Brandes' two phases (Brandes 2001, the algorithm the paper cites for
// betweenness in "Heuristics and Approximation Algorithms" and Table 1) are
// run for a group of B sources together, level by level, over the union of
// their frontiers:
//
//   union level l  = every vertex v that is at distance l from at least one
//                    source of the group, listed once, with the mask f(v)
//                    of those sources;
//   forward        top-down: for each listed v and arc (v, w), the sources
//                  in f(v) that have not reached w add sigma_b(v) to
//                  sigma_b(w) (64-bit atomics); bottom-up: every vertex some
//                  source has not reached sums sigma_b over neighbours that
//                  source has reached (they are exactly its level l);
//   backward       for levels from deepest to 1, every listed v pulls, for
//                  each b in f(v), coef_b(w) = (1 + delta_b(w)) / sigma_b(w)
//                  over neighbours w one level deeper for b, and adds
//                  sum over b of delta_b(v) to bc[v] in one FP64 atomic.
//
// Every CSR row is read once per union level it appears on instead of once
// per source, and the per-source state of a vertex is interleaved
// (sigma[v * B + b], one cache line holding a vertex's B counts), so a
// random access to a vertex serves every source that needs it.
//
// Visited state is a B-bit mask per vertex (bit b: source b has reached the
// vertex at the current level or before): in LDS for the first ms_nl
// vertices, in per-slot global memory for the rest.  During the forward
// phase an unset bit b of a neighbour of a level-l vertex of source b means
// the neighbour is at level l + 1 of source b; during the backward phase
// levels are cleared from the deepest up, so the same test finds level
// l + 1 again.  Sources newly reaching a vertex during a level are gathered
// in nx[v] (atomic OR); the first contributor appends v to the next union
// level, and the marking pass moves nx[v] into the list entry and the mask.
#include "nk_kernels.h"

namespace nk {

constexpr int kMsChunk = 4;
// Sources handled by one lane in the arc loops: an arc is taken by B / kSpl
// neighbouring lanes.
constexpr int kSpl = 4;

// Work counters: DAG arcs per lane (summed over the workgroup at the end);
// the others in the tile (MsTile::ctr, indexed by kC*).
struct Counters {
    unsigned long long dag;
};
enum { kCArcsFwd = 0, kCArcsBwd, kCReached, kCArcsReached, kCTasks, kCTd, kCBu, kNumC };

// Visited-mask field per vertex: one byte for up to 8 sources, two for 16.
template <int B>
struct MsVis {
    static constexpr int kBits = B <= 8 ? 8 : 16;
    static constexpr int kPerWord = 32 / kBits;
    static constexpr uint32_t kField = (B <= 8) ? 0xFFu : 0xFFFFu;
};

template <int BLOCK, int B>
struct MsTile {
    // tile rows: their B 8-byte values fill 32 * BLOCK bytes
    static constexpr int TR = 4 * BLOCK / B;
    int32_t v[TR];
    int32_t a0[TR];
    int32_t pre[TR + 1];
    uint32_t f[TR];
    union {
        unsigned long long u[TR * B];   // forward: sigma of the rows' sources; bottom-up: path-count sums
        double d[TR * B];               // backward: sums of coef over the successors
    } val;
    int32_t wsum[BLOCK / kWave + 1];
    long long task;
    long long mf;        // arcs of the current union level
    long long mu;        // arcs of vertices some source has not reached
    long long acc_mf, acc_full;
    int32_t count;       // append counter (next level / candidates)
    int32_t nsrc;
    uint32_t amask;
    int32_t flag;
    int32_t lvl_lo[2];
    int32_t src[B];
    unsigned long long ctr[kNumC];
    unsigned long long cyc[8];
    long long t0;
};

// A workgroup slot's state for the current task.
template <int B>
struct MsSlot {
    const int32_t *rp;
    const int32_t *ci;
    int32_t n;
    int32_t nl;                  // vertices whose mask sits in LDS
    long long m;
    long long vbase;
    unsigned long long *sig;     // [n * B]
    uint32_t *nx;
    uint32_t *visl;              // LDS masks
    uint32_t *visg;              // global masks (vertices nl and up)
    const uint32_t *iso;         // isolated vertices of a single graph, or NULL
    int32_t *lv, *la, *ld;
    uint32_t *lm;
    int32_t *lvl;
    int32_t *cand;
    long long cap;               // list entries per slot
    uint32_t amask;
};

// Plain loads of values other lanes of the workgroup wrote (with stores or
// atomics) before a barrier: the waves of a workgroup share one compute
// unit's vector cache, which keeps them coherent with no cache maintenance.
__device__ __forceinline__ unsigned long long ld_u64(const unsigned long long *p) { return *p; }
__device__ __forceinline__ uint32_t ld_u32(const uint32_t *p) { return *p; }

// The lane's kSpl path counts (or coefficient bits) of one vertex, as
// 16-byte loads (32-byte aligned: the row is B * 8 bytes, the lane's part
// kSpl * 8); x[t] = 0 where bit t of `mine` is clear, and no load at all
// when `mine` is 0.
__device__ __forceinline__ void load_row(const unsigned long long *row, uint32_t mine,
                                         unsigned long long (&x)[kSpl]) {
    if (mine) {
        const ulonglong2 *r2 = reinterpret_cast<const ulonglong2 *>(row);
#pragma unroll
        for (int h = 0; h < kSpl / 2; ++h) {
            const ulonglong2 v = r2[h];
            x[2 * h] = ((mine >> (2 * h)) & 1u) ? v.x : 0ULL;
            x[2 * h + 1] = ((mine >> (2 * h + 1)) & 1u) ? v.y : 0ULL;
        }
    } else {
#pragma unroll
        for (int t = 0; t < kSpl; ++t) x[t] = 0ULL;
    }
}

template <int B>
__device__ __forceinline__ uint32_t vis_get(const MsSlot<B> &S, int32_t v) {
    using V = MsVis<B>;
    const int sh = (v % V::kPerWord) * V::kBits;
    const uint32_t w = v < S.nl ? S.visl[v / V::kPerWord] : ld_u32(S.visg + v / V::kPerWord);
    return (w >> sh) & V::kField;
}

template <int B>
__device__ __forceinline__ uint32_t vis_or(const MsSlot<B> &S, int32_t v, uint32_t bits) {
    using V = MsVis<B>;
    const int sh = (v % V::kPerWord) * V::kBits;
    uint32_t *w = v < S.nl ? S.visl : S.visg;
    return (atomicOr(w + v / V::kPerWord, bits << sh) >> sh) & V::kField;
}

template <int B>
__device__ __forceinline__ void vis_clear(const MsSlot<B> &S, int32_t v, uint32_t bits) {
    using V = MsVis<B>;
    const int sh = (v % V::kPerWord) * V::kBits;
    uint32_t *w = v < S.nl ? S.visl : S.visg;
    atomicAnd(w + v / V::kPerWord, ~(bits << sh));
}

__device__ __forceinline__ bool iso_bit(const uint32_t *iso, int32_t v) { return (iso[v >> 5] >> (v & 31)) & 1u; }

// Values every lane holds alike, moved to scalar registers.
__device__ __forceinline__ int32_t uni(int32_t x) { return __builtin_amdgcn_readfirstlane(x); }
__device__ __forceinline__ long long uni(long long x) {
    const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)(unsigned long long)x);
    const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)((unsigned long long)x >> 32));
    return (long long)(((unsigned long long)hi << 32) | lo);
}
template <typename T>
__device__ __forceinline__ T *uni(T *x) {
    return reinterpret_cast<T *>(uni((long long)reinterpret_cast<uintptr_t>(x)));
}

// Block-wide exclusive scan (barriers inside; every thread calls it).
template <int BLOCK>
__device__ __forceinline__ int32_t ms_scan(int32_t x, int32_t *wsum, int32_t &total) {
    constexpr int NW = BLOCK / kWave;
    const int lane = lane_id(), wid = wave_id();
    const int32_t incl = wave_incl_scan<int32_t>(x);
    if (lane == kWave - 1) wsum[wid] = incl;
    __syncthreads();
    if (wid == 0) {
        const int32_t s = lane < NW ? wsum[lane] : 0;
        const int32_t si = wave_incl_scan<int32_t>(s);
        if (lane < NW) wsum[lane] = si - s;
        if (lane == NW - 1) wsum[NW] = si;
    }
    __syncthreads();
    total = wsum[NW];
    const int32_t r = incl - x + wsum[wid];
    __syncthreads();
    return r;
}

// Stages union-list entries [tb, tb + cnt) (vertex, first arc, mask, degree
// prefix); returns the tile's arc count.  The caller synchronises before
// reading the tile.
template <int BLOCK, int B>
__device__ __forceinline__ int32_t ms_stage(MsTile<BLOCK, B> &sm, const MsSlot<B> &S, int32_t tb, int32_t cnt) {
    const int tid = threadIdx.x;
    int32_t dg = 0;
    if (tid < cnt) {
        sm.v[tid] = S.lv[tb + tid];
        sm.a0[tid] = S.la[tb + tid];
        sm.f[tid] = S.lm[tb + tid];
        dg = S.ld[tb + tid];
    }
    int32_t total;
    const int32_t ex = ms_scan<BLOCK>(dg, sm.wsum, total);
    if (tid < cnt) sm.pre[tid] = ex;
    if (tid == 0) sm.pre[cnt] = total;
    return total;
}

// Column indices of arcs [i0, i0 + kMsChunk) of the tile; kk[j] = row, -1
// past the end.
template <int BLOCK, int B>
__device__ __forceinline__ void ms_chunk(const MsTile<BLOCK, B> &sm, const MsSlot<B> &S, int32_t cnt, int32_t total,
                                         int32_t i0, int32_t (&kk)[kMsChunk], int32_t (&w)[kMsChunk]) {
    int32_t k = (i0 < total) ? tile_search(sm.pre, cnt, i0) : 0;
#pragma unroll
    for (int j = 0; j < kMsChunk; ++j) {
        const int32_t i = i0 + j;
        kk[j] = -1;
        w[j] = 0;
        if (i < total) {
            while (sm.pre[k + 1] <= i) ++k;
            kk[j] = k;
            w[j] = S.ci[sm.a0[k] + (i - sm.pre[k])];
        }
    }
}

// Top-down expansion of union level [f0, f1) into the list from f1.  The
// arcs of a tile are taken kMsChunk at a time by groups of B / kSpl lanes;
// lane q of a group handles sources q * kSpl .. q * kSpl + kSpl - 1, so the B
// path counts of an arc's head are read by neighbouring lanes.  Every source
// of the row that has not reached the head adds its count; the head's mask
// in nx gains those sources, and the lane whose OR finds nx clear appends
// the head to the next level.
template <int BLOCK, int B>
__device__ void ms_td(const Params &p, MsTile<BLOCK, B> &sm, const MsSlot<B> &S, int32_t f0, int32_t f1,
                      Counters &c) {
    constexpr int TR = MsTile<BLOCK, B>::TR;
    constexpr int G = B / kSpl;            // lanes per arc
    constexpr int GROUPS = BLOCK / G;
    const int tid = threadIdx.x;
    const int grp = tid / G, q = tid % G;
    for (int32_t tb = f0; tb < f1; tb += TR) {
        const int32_t cnt = min(TR, f1 - tb);
        const int32_t total = ms_stage<BLOCK, B>(sm, S, tb, cnt);
        for (int32_t i = tid; i < cnt * B; i += BLOCK) {
            const int32_t r = i / B, bb = i % B;
            sm.val.u[i] = ((sm.f[r] >> bb) & 1u) ? ld_u64(S.sig + (long long)sm.v[r] * B + bb) : 0ULL;
        }
        __syncthreads();
        if (tid == 0) sm.ctr[kCArcsFwd] += (unsigned long long)total;
        bool ovf = false;
        for (int32_t rb = 0; rb < total; rb += GROUPS * kMsChunk) {
            int32_t kk[kMsChunk], w[kMsChunk];
            ms_chunk<BLOCK, B>(sm, S, cnt, total, rb + grp * kMsChunk, kk, w);
            uint32_t nb[kMsChunk];
#pragma unroll
            for (int j = 0; j < kMsChunk; ++j) nb[j] = kk[j] >= 0 ? (sm.f[kk[j]] & ~vis_get<B>(S, w[j])) : 0u;
#pragma unroll
            for (int j = 0; j < kMsChunk; ++j) {
                const uint32_t mine = (nb[j] >> (q * kSpl)) & ((1u << kSpl) - 1u);
                if (mine) {
                    unsigned long long *row = S.sig + (long long)w[j] * B + q * kSpl;
                    const unsigned long long *sv = sm.val.u + kk[j] * B + q * kSpl;
                    unsigned long long add[kSpl], old[kSpl];
#pragma unroll
                    for (int t = 0; t < kSpl; ++t) {
                        add[t] = ((mine >> t) & 1u) ? sv[t] : 0ULL;
                        old[t] = add[t] ? atomicAdd(row + t, add[t]) : 0ULL;
                    }
#pragma unroll
                    for (int t = 0; t < kSpl; ++t) ovf |= old[t] + add[t] < old[t];
                }
                const bool lead = q == 0 && nb[j] != 0u;
                const bool fresh = lead && atomicOr(S.nx + w[j], nb[j]) == 0u;
                if (lead) c.dag += (unsigned long long)__popc(nb[j]);
                wave_append(fresh, w[j], S.lv + f1, &sm.count, (int32_t)min<long long>(S.cap - f1, 0x7fffffffLL),
                            &p.st->err);
            }
        }
        if (ovf) atomicOr(&p.st->err, kErrOverflow);
        __syncthreads();
    }
}

// Bottom-up expansion: every vertex some source of the task has not reached
// sums, per such source, sigma over neighbours that source has reached.
template <int BLOCK, int B>
__device__ void ms_bu(const Params &p, MsTile<BLOCK, B> &sm, const MsSlot<B> &S, int32_t f1, Counters &c) {
    constexpr int TR = MsTile<BLOCK, B>::TR;
    constexpr int G = B / kSpl;
    constexpr int GROUPS = BLOCK / G;
    const int tid = threadIdx.x;
    const int grp = tid / G, q = tid % G;
    if (tid == 0) sm.count = 0;
    __syncthreads();
    for (int32_t v0 = 0; v0 < S.n; v0 += BLOCK) {
        const int32_t v = v0 + tid;
        const bool cand = v < S.n && (~vis_get<B>(S, v) & S.amask) != 0u && !(S.iso && iso_bit(S.iso, v));
        wave_append(cand, v, S.cand, &sm.count, S.n, &p.st->err);
    }
    __syncthreads();
    const int32_t nc = sm.count;
    __syncthreads();
    if (tid == 0) sm.count = 0;
    for (int32_t tb = 0; tb < nc; tb += TR) {
        const int32_t cnt = min(TR, nc - tb);
        int32_t dg = 0;
        if (tid < cnt) {
            const int32_t w = S.cand[tb + tid];
            const int32_t a0 = S.rp[w];
            dg = S.rp[w + 1] - a0;
            sm.v[tid] = w;
            sm.a0[tid] = a0;
            sm.f[tid] = ~vis_get<B>(S, w) & S.amask;
        }
        int32_t total;
        const int32_t ex = ms_scan<BLOCK>(dg, sm.wsum, total);
        if (tid < cnt) sm.pre[tid] = ex;
        if (tid == 0) sm.pre[cnt] = total;
        for (int32_t i = tid; i < cnt * B; i += BLOCK) sm.val.u[i] = 0ULL;
        __syncthreads();
        if (tid == 0) sm.ctr[kCArcsFwd] += (unsigned long long)total;
        bool ovf = false;
        for (int32_t rb = 0; rb < total; rb += GROUPS * kMsChunk) {
            int32_t kk[kMsChunk], vv[kMsChunk];
            ms_chunk<BLOCK, B>(sm, S, cnt, total, rb + grp * kMsChunk, kk, vv);
            uint32_t bits[kMsChunk];
#pragma unroll
            for (int j = 0; j < kMsChunk; ++j) bits[j] = kk[j] >= 0 ? (sm.f[kk[j]] & vis_get<B>(S, vv[j])) : 0u;
            unsigned long long x[kMsChunk][kSpl];
#pragma unroll
            for (int j = 0; j < kMsChunk; ++j) {
                const uint32_t mine = (bits[j] >> (q * kSpl)) & ((1u << kSpl) - 1u);
                load_row(S.sig + (long long)vv[j] * B + q * kSpl, mine, x[j]);
            }
            int32_t kcur = kk[0];
            unsigned long long acc[kSpl];
#pragma unroll
            for (int t = 0; t < kSpl; ++t) acc[t] = 0ULL;
#pragma unroll
            for (int j = 0; j < kMsChunk; ++j) {
                if (kk[j] < 0) continue;
                if (q == 0) c.dag += (unsigned long long)__popc(bits[j]);
                if (kk[j] != kcur) {
#pragma unroll
                    for (int t = 0; t < kSpl; ++t) {
                        if (acc[t]) {
                            const unsigned long long o = atomicAdd(&sm.val.u[kcur * B + q * kSpl + t], acc[t]);
                            ovf |= o + acc[t] < o;
                        }
                        acc[t] = 0ULL;
                    }
                    kcur = kk[j];
                }
#pragma unroll
                for (int t = 0; t < kSpl; ++t) {
                    const unsigned long long nacc = acc[t] + x[j][t];
                    ovf |= nacc < acc[t];
                    acc[t] = nacc;
                }
            }
#pragma unroll
            for (int t = 0; t < kSpl; ++t) {
                if (acc[t]) {
                    const unsigned long long o = atomicAdd(&sm.val.u[kcur * B + q * kSpl + t], acc[t]);
                    ovf |= o + acc[t] < o;
                }
            }
        }
        if (ovf) atomicOr(&p.st->err, kErrOverflow);
        __syncthreads();
        // rows with new sources: their path counts, their mask in nx, and
        // an entry in the next level
        bool fresh = false;
        int32_t w = 0;
        if (tid < cnt) {
            w = sm.v[tid];
            uint32_t F = 0u;
            unsigned long long *row = S.sig + (long long)w * B;
#pragma unroll
            for (int bb = 0; bb < B; ++bb) {
                const unsigned long long x = sm.val.u[tid * B + bb];
                if (x) {
                    row[bb] = x;
                    F |= 1u << bb;
                }
            }
            if (F) {
                atomicOr(S.nx + w, F);
                fresh = true;
            }
        }
        wave_append(fresh, w, S.lv + f1, &sm.count, (int32_t)min<long long>(S.cap - f1, 0x7fffffffLL), &p.st->err);
        __syncthreads();
    }
}

// Marks the new union level list[f1, f1 + nnew): masks from nx into the
// entries and the visited masks, first arc and degree of each vertex; sums
// for the direction choice and the work counters.
template <int BLOCK, int B>
__device__ void ms_mark(MsTile<BLOCK, B> &sm, const MsSlot<B> &S, int32_t f1, int32_t nnew, Counters &c) {
    const int tid = threadIdx.x;
    long long dsum = 0, dfull = 0;
    unsigned long long rsum = 0, asum = 0;
    for (int32_t i = f1 + tid; i < f1 + nnew; i += BLOCK) {
        const int32_t w = S.lv[i];
        const uint32_t F = atomicExch(S.nx + w, 0u);
        S.lm[i] = F;
        const uint32_t old = vis_or<B>(S, w, F);
        const int32_t a0 = S.rp[w];
        const int32_t dg = S.rp[w + 1] - a0;
        S.la[i] = a0;
        S.ld[i] = dg;
        dsum += dg;
        if (((old | F) & S.amask) == S.amask) dfull += dg;
        rsum += (unsigned long long)__popc(F);
        asum += (unsigned long long)__popc(F) * (unsigned long long)dg;
    }
    dsum = wave_sum<long long>(dsum);
    dfull = wave_sum<long long>(dfull);
    rsum = wave_sum<unsigned long long>(rsum);
    asum = wave_sum<unsigned long long>(asum);
    if (lane_id() == 0) {
        if (dsum) atomicAdd((unsigned long long *)&sm.acc_mf, (unsigned long long)dsum);
        if (dfull) atomicAdd((unsigned long long *)&sm.acc_full, (unsigned long long)dfull);
        if (rsum) atomicAdd(&sm.ctr[kCReached], rsum);
        if (asum) atomicAdd(&sm.ctr[kCArcsReached], asum);
    }
}

// Backward union level [lo, hi) by pull: every (v, b in f(v)) sums coef_b
// over neighbours whose bit b is clear (its level l + 1), then takes
// delta_b(v) = sigma_b(v) * sum, coef_b(v) = (1 + delta_b(v)) / sigma_b(v),
// and v's score gains the sum of delta_b(v) over f(v).
template <int BLOCK, int B>
__device__ void ms_pull(MsTile<BLOCK, B> &sm, const MsSlot<B> &S, int32_t lo, int32_t hi, double *bcg, double wfac,
                        Counters &c) {
    constexpr int TR = MsTile<BLOCK, B>::TR;
    constexpr int G = B / kSpl;
    constexpr int GROUPS = BLOCK / G;
    const int tid = threadIdx.x;
    const int grp = tid / G, q = tid % G;
    for (int32_t tb = lo; tb < hi; tb += TR) {
        const int32_t cnt = min(TR, hi - tb);
        const int32_t total = ms_stage<BLOCK, B>(sm, S, tb, cnt);
        for (int32_t i = tid; i < cnt * B; i += BLOCK) sm.val.d[i] = 0.0;
        __syncthreads();
        if (tid == 0) sm.ctr[kCArcsBwd] += (unsigned long long)total;
        for (int32_t rb = 0; rb < total; rb += GROUPS * kMsChunk) {
            int32_t kk[kMsChunk], w[kMsChunk];
            ms_chunk<BLOCK, B>(sm, S, cnt, total, rb + grp * kMsChunk, kk, w);
            uint32_t bits[kMsChunk];
#pragma unroll
            for (int j = 0; j < kMsChunk; ++j) bits[j] = kk[j] >= 0 ? (sm.f[kk[j]] & ~vis_get<B>(S, w[j])) : 0u;
            double x[kMsChunk][kSpl];
#pragma unroll
            for (int j = 0; j < kMsChunk; ++j) {
                const uint32_t mine = (bits[j] >> (q * kSpl)) & ((1u << kSpl) - 1u);
                unsigned long long raw[kSpl];
                load_row(S.sig + (long long)w[j] * B + q * kSpl, mine, raw);
#pragma unroll
                for (int t = 0; t < kSpl; ++t) x[j][t] = __longlong_as_double((long long)raw[t]);
            }
            int32_t kcur = kk[0];
            double acc[kSpl];
#pragma unroll
            for (int t = 0; t < kSpl; ++t) acc[t] = 0.0;
#pragma unroll
            for (int j = 0; j < kMsChunk; ++j) {
                if (kk[j] < 0) continue;
                if (kk[j] != kcur) {
#pragma unroll
                    for (int t = 0; t < kSpl; ++t) {
                        if (acc[t] != 0.0) atomicAdd(&sm.val.d[kcur * B + q * kSpl + t], acc[t]);
                        acc[t] = 0.0;
                    }
                    kcur = kk[j];
                }
#pragma unroll
                for (int t = 0; t < kSpl; ++t) acc[t] += x[j][t];
            }
#pragma unroll
            for (int t = 0; t < kSpl; ++t)
                if (acc[t] != 0.0) atomicAdd(&sm.val.d[kcur * B + q * kSpl + t], acc[t]);
        }
        __syncthreads();
        // finalize: B consecutive threads per row, then one score atomic per row
        for (int32_t i0 = 0; i0 < cnt * B; i0 += BLOCK) {
            const int32_t i = i0 + tid;
            double delta = 0.0;
            if (i < cnt * B) {
                const int32_t r = i / B, b = i % B;
                if ((sm.f[r] >> b) & 1u) {
                    unsigned long long *cell = S.sig + (long long)sm.v[r] * B + b;
                    const double sg = (double)ld_u64(cell);
                    delta = sg * sm.val.d[i] * wfac;
                    *cell = (unsigned long long)__double_as_longlong((1.0 + delta) / sg);
                }
            }
#pragma unroll
            for (int off = B / 2; off > 0; off >>= 1) delta += __shfl_xor(delta, off, kWave);
            if (i < cnt * B && (i % B) == 0 && delta != 0.0) atomicAdd(bcg + sm.v[i / B], delta);
        }
        __syncthreads();
    }
}

template <int BLOCK, int B>
__global__ __launch_bounds__(BLOCK) void k_brandes_ms(Params p) {
    extern __shared__ uint32_t lds_vis[];
    __shared__ MsTile<BLOCK, B> sm;
    const int tid = threadIdx.x;
    if (tid == 0) sm.flag = p.st->err & kErrGraph;
    __syncthreads();
    if (sm.flag) return;
    __syncthreads();

    const long long slot = blockIdx.x;
    MsSlot<B> S;
    S.sig = p.sigma + slot * p.stride * B;
    S.nx = p.nx + slot * p.stride;
    S.visl = lds_vis;
    S.visg = p.visg + slot * p.visg_words;
    S.lv = p.lv + slot * p.ms_cap;
    S.la = p.la + slot * p.ms_cap;
    S.ld = p.ld + slot * p.ms_cap;
    S.lm = p.lm + slot * p.ms_cap;
    S.lvl = p.lvl + slot * p.stride;
    S.cand = p.cand + slot * p.stride;
    S.cap = p.ms_cap;

    Counters c = {0};
    if (tid < 8) sm.cyc[tid] = 0;
    if (tid < kNumC) sm.ctr[tid] = 0;
    __syncthreads();
    const long long t_kernel = clock64();
    for (;;) {
        if (tid == 0) sm.task = (long long)atomicAdd(&p.st->head, 1ULL);
        __syncthreads();
        const long long task = sm.task;
        __syncthreads();
        if (task >= p.ntasks) break;
        if (tid == 0) sm.t0 = clock64();

        // the task's graph and sources
        long long first;   // first source index of the task
        if (p.G > 0) {
            int32_t lo = 0, hi = p.G - 1;
            while (lo < hi) {
                const int32_t mid = (lo + hi + 1) >> 1;
                if (p.g_task[mid] <= task) lo = mid; else hi = mid - 1;
            }
            const int32_t gid = p.g_order[lo];
            const long long v0 = p.g_vtx[gid];
            S.rp = p.rowptr + v0 + gid;
            S.ci = p.colidx + p.g_arc[gid];
            S.n = (int32_t)(p.g_vtx[gid + 1] - v0);
            S.m = p.g_arc[gid + 1] - p.g_arc[gid];
            S.vbase = v0;
            S.iso = nullptr;
            first = (task - p.g_task[lo]) * B;
            if (tid == 0) sm.nsrc = (int32_t)min<long long>(B, S.n - first);
        } else {
            S.rp = p.rowptr;
            S.ci = p.colidx;
            S.n = p.n;
            S.m = p.m;
            S.vbase = 0;
            S.iso = p.iso;
            first = task * B;
            if (tid == 0) sm.nsrc = (int32_t)min<long long>(B, p.nsources - first);
        }
        S.rp = uni(S.rp);
        S.ci = uni(S.ci);
        S.n = uni(S.n);
        S.m = uni(S.m);
        S.vbase = uni(S.vbase);
        S.iso = uni(S.iso);
        first = uni(first);
        S.nl = min(p.ms_nl, S.n);
        if (tid < B) {
            int32_t s = -1;
            const long long idx = first + tid;
            if (p.G > 0) {
                if (idx < S.n) s = (int32_t)idx;
            } else if (idx < p.nsources) {
                s = p.sources ? p.sources[idx] : (int32_t)idx;
            }
            sm.src[tid] = s;
        }
        __syncthreads();
        const int32_t nsrc = uni(sm.nsrc);
        bool bad = false;
        for (int b = 0; b < nsrc; ++b) bad |= sm.src[b] < 0 || sm.src[b] >= S.n;
        if (bad) {
            if (tid == 0) atomicOr(&p.st->err, kErrArg);
            __syncthreads();
            continue;
        }
        S.amask = (uint32_t)uni((int32_t)(nsrc >= 32 ? 0xFFFFFFFFu : ((1u << nsrc) - 1u)));
        // LDS masks start clear (global ones are cleared by the reset pass)
        {
            using V = MsVis<B>;
            const int32_t words = (S.nl + V::kPerWord - 1) / V::kPerWord;
            for (int32_t i = tid; i < words; i += BLOCK) S.visl[i] = 0u;
        }
        if (tid == 0) sm.count = 0;
        __syncthreads();
        // level 0: the sources (a repeated source is one entry with several bits)
        if (tid < kWave) {
            bool fresh = false;
            int32_t s = 0;
            if (tid < nsrc) {
                s = sm.src[tid];
                S.sig[(long long)s * B + tid] = 1ULL;
                fresh = atomicOr(S.nx + s, 1u << tid) == 0u;
            }
            wave_append(fresh, s, S.lv, &sm.count, (int32_t)min<long long>(S.cap, 0x7fffffffLL), &p.st->err);
        }
        if (tid == 0) {
            sm.acc_mf = 0;
            sm.acc_full = 0;
            sm.mu = S.m;
        }
        __syncthreads();
        const int32_t n0 = sm.count;
        ms_mark<BLOCK, B>(sm, S, 0, n0, c);
        __syncthreads();
        if (tid == 0) {
            S.lvl[0] = 0;
            S.lvl[1] = n0;
            sm.mf = sm.acc_mf;
            sm.mu -= sm.acc_full;
            sm.lvl_lo[0] = 0;
            sm.lvl_lo[1] = n0;
            sm.cyc[kPhInit] += (unsigned long long)(clock64() - sm.t0);
        }
        __syncthreads();
        int32_t lvl = 0;
        for (;;) {
            const int32_t f0 = sm.lvl_lo[0], f1 = sm.lvl_lo[1];
            const bool bu = (p.bu_ratio > 0.0f) && ((double)sm.mu < (double)p.bu_ratio * (double)sm.mf);
            __syncthreads();
            if (tid == 0) {
                sm.count = 0;
                sm.acc_mf = 0;
                sm.acc_full = 0;
                sm.ctr[bu ? kCBu : kCTd] += 1ULL;
                sm.t0 = clock64();
            }
            __syncthreads();
            if (bu)
                ms_bu<BLOCK, B>(p, sm, S, f1, c);
            else
                ms_td<BLOCK, B>(p, sm, S, f0, f1, c);
            __syncthreads();
            if (tid == 0) {
                sm.cyc[bu ? kPhBu : kPhTd] += (unsigned long long)(clock64() - sm.t0);
                sm.t0 = clock64();
            }
            const int32_t nnew = (long long)sm.count < S.cap - f1 ? sm.count : (int32_t)(S.cap - f1);
            ms_mark<BLOCK, B>(sm, S, f1, nnew, c);
            __syncthreads();
            if (tid == 0) {
                S.lvl[lvl + 2] = f1 + nnew;
                sm.lvl_lo[0] = f1;
                sm.lvl_lo[1] = f1 + nnew;
                sm.mf = sm.acc_mf;
                sm.mu -= sm.acc_full;
                sm.cyc[kPhMark] += (unsigned long long)(clock64() - sm.t0);
            }
            __syncthreads();
            if (nnew == 0) break;
            // a union level deeper than n - 1 cannot happen; stop rather
            // than loop if it ever did
            if (lvl + 1 >= S.n) {
                if (tid == 0) atomicOr(&p.st->err, kErrInternal);
                break;
            }
            ++lvl;
        }
        const int32_t Ld = lvl;   // deepest non-empty union level
        const int32_t total = S.lvl[Ld + 1];
        if (tid == 0) {
            sm.ctr[kCTasks] += (unsigned long long)nsrc;
            sm.t0 = clock64();
        }
        // backward: the deepest level's coefficients are 1 / sigma
        if (Ld > 0) {
            const int32_t lo = S.lvl[Ld], hi = S.lvl[Ld + 1];
            for (long long i = (long long)lo * B + tid; i < (long long)hi * B; i += BLOCK) {
                const int32_t e = (int32_t)(i / B), b = (int32_t)(i % B);
                const uint32_t f = S.lm[e];
                if ((f >> b) & 1u) {
                    unsigned long long *cell = S.sig + (long long)S.lv[e] * B + b;
                    *cell = (unsigned long long)__double_as_longlong(1.0 / (double)ld_u64(cell));
                }
            }
            for (int32_t e = lo + tid; e < hi; e += BLOCK) vis_clear<B>(S, S.lv[e], S.lm[e]);
            __syncthreads();
            double *bcg = p.bc + S.vbase;
            for (int32_t l = Ld - 1; l >= 1; --l) {
                const int32_t llo = S.lvl[l], lhi = S.lvl[l + 1];
                const double wfac = p.linear ? (double)l / (double)(l + 1) : 1.0;
                ms_pull<BLOCK, B>(sm, S, llo, lhi, bcg, wfac, c);
                for (int32_t e = llo + tid; e < lhi; e += BLOCK) vis_clear<B>(S, S.lv[e], S.lm[e]);
                __syncthreads();
            }
        }
        if (tid == 0) {
            sm.cyc[kPhPull] += (unsigned long long)(clock64() - sm.t0);
            sm.t0 = clock64();
        }
        // reset: path counts of every listed vertex, global masks
        for (long long i = tid; i < (long long)total * B; i += BLOCK) S.sig[(long long)S.lv[i / B] * B + (i % B)] = 0ULL;
        for (int32_t e = tid; e < total; e += BLOCK) {
            const int32_t v = S.lv[e];
            if (v >= S.nl) vis_clear<B>(S, v, MsVis<B>::kField);
        }
        __syncthreads();
        if (tid == 0) {
            sm.cyc[kPhReset] += (unsigned long long)(clock64() - sm.t0);
            atomicAdd(&p.st->stat[kStDone], (unsigned long long)nsrc);
        }
    }

    // counters: wave sums of the DAG arcs, one atomic per wave; the rest
    // from the tile
    const unsigned long long dag = wave_sum<unsigned long long>(c.dag);
    if (lane_id() == 0 && dag) atomicAdd(&p.st->stat[kStDag], dag);
    if (tid == 0) {
        atomicAdd(&p.st->stat[kStSources], sm.ctr[kCTasks]);
        atomicAdd(&p.st->stat[kStReached], sm.ctr[kCReached]);
        atomicAdd(&p.st->stat[kStArcsReached], sm.ctr[kCArcsReached]);
        atomicAdd(&p.st->stat[kStArcsFwd], sm.ctr[kCArcsFwd]);
        atomicAdd(&p.st->stat[kStArcsBwd], sm.ctr[kCArcsBwd]);
        atomicAdd(&p.st->stat[kStTd], sm.ctr[kCTd]);
        atomicAdd(&p.st->stat[kStBu], sm.ctr[kCBu]);
        unsigned long long known = 0;
        for (int i = 0; i < kNumPhases; ++i)
            if (i != kPhOther) known += sm.cyc[i];
        const unsigned long long tot = (unsigned long long)(clock64() - t_kernel);
        sm.cyc[kPhOther] = tot > known ? tot - known : 0;
        for (int i = 0; i < kNumPhases; ++i) atomicAdd(&p.st->cycles[i], sm.cyc[i]);
    }
}

template <int BLOCK, int B>
static void launch_ms(dim3 grid, dim3 block, size_t lds, hipStream_t s, const Params &p) {
    hipLaunchKernelGGL((k_brandes_ms<BLOCK, B>), grid, block, lds, s, p);
}

template <int BLOCK, int B>
static KernelRef ms_ref() {
    return KernelRef{(const void *)&k_brandes_ms<BLOCK, B>, &launch_ms<BLOCK, B>};
}

template <int B>
static KernelRef ms_ref_b(int block) {
    switch (block) {
        case 256: return ms_ref<256, B>();
        case 512: return ms_ref<512, B>();
        default: return ms_ref<1024, B>();
    }
}

KernelRef brandes_ms_kernel(int block, int b) {
    switch (b) {
        case 4: return ms_ref_b<4>(block);
        case 16: return ms_ref_b<16>(block);
        default: return ms_ref_b<8>(block);
    }
}

int ms_mask_bytes(int b) { return b <= 8 ? 1 : 2; }

}  // namespace nk
