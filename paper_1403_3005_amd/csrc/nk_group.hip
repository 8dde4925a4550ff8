// Group Brandes kernel: the workgroups that share one XCD run one source at
// a time together.
//
// A source's path counts and coefficients (8 bytes per vertex) are read at
// random positions once per DAG arc.  When every workgroup runs a source of
// its own, 32 workgroups of an XCD keep 32 such arrays live against one
// 4 MB L2 (and 256 of them against the 256 MB Infinity Cache), and almost
// every access leaves the XCD.  Here the workgroups of an XCD split into
// groups of S (a tuning value, 4 by default), each group sharing one
// source's arrays: S = 32 keeps a graph of a few hundred thousand vertices
// in the XCD's L2, smaller groups keep all sources in flight within the
// Infinity Cache while leaving each member enough of a level to overlap
// its memory round trips.  The algorithm per source is the same as the
// one-workgroup kernel's (nk_kernels.hip): level-synchronous forward search
// counting shortest paths (top-down with 64-bit atomics, or bottom-up),
// then the dependency pull level by level from the deepest (Brandes 2001,
// the algorithm the paper uses for betweenness), with the levels split
// over the group's workgroups and one group barrier per level.
//
// Group membership comes from the XCC_ID hardware register, read by each
// workgroup at start, so it does not depend on how workgroups are
// dispatched.  Every workgroup of the launch must be resident at once (the
// launch is sized to one workgroup per compute unit, all but one compute
// unit, and made cooperative where the runtime allows); a registration
// count checks this.  A 1024-thread workgroup holds all of its compute
// unit's vector registers, so the compute unit left free is where the
// runtime's copy kernels run meanwhile (a progress read during the launch).
//
// Data exchange inside a group relies on the XCD's L2 being the point of
// coherence for all its compute units: a workgroup's stores reach L2 before
// it arrives at a group barrier (it waits for its outstanding memory
// operations first), and every read of data that other workgroups of the
// group write goes through loads at agent scope, which bypass the compute
// unit's vector cache.  Atomics are performed at L2.  The graph itself is
// read-only and read with plain loads.  No agent-scope fence is needed
// within the group, which keeps a barrier near one microsecond.
//
// Every wait (registration, group barriers) is bounded by the wall clock;
// a workgroup that times out raises kErrInternal and the group's abort flag,
// and every workgroup of the group then leaves its task loop.
#include "nk_kernels.h"

namespace nk {

namespace {

constexpr int kGChunk = 4;     // arcs per thread per pass of an arc loop
constexpr int kAccSlots = 4;   // rotating per-level accumulators

struct alignas(128) GroupLine {
    unsigned long long v;
    unsigned long long w;
    char pad[112];
};

// Control block of one group (zeroed before the launch).
struct GroupCtl {
    GroupLine bar;                  // barrier arrivals (v), monotonic
    GroupLine acc[kAccSlots];       // per level: appended vertices (v) and their degree sum (w)
    GroupLine task[2];              // task broadcast, double-buffered by task parity
    GroupLine abort;                // nonzero: a member timed out
};

static_assert(sizeof(GroupCtl) == 128 * (3 + kAccSlots + 1), "group control layout");

// Relaxed loads at agent scope: they bypass the compute unit's vector cache
// and read the XCD's L2, where the group's stores and atomics land.
__device__ __forceinline__ unsigned long long ldg_u64(const unsigned long long *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ int32_t ldg_i32(const int32_t *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint32_t ldg_u32(const uint32_t *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ double f64_of(unsigned long long x) { return __longlong_as_double((long long)x); }
__device__ __forceinline__ unsigned long long u64_of(double x) { return (unsigned long long)__double_as_longlong(x); }

__device__ __forceinline__ bool lbit(const uint32_t *bm, int32_t v) { return (bm[v >> 5] >> (v & 31)) & 1u; }

// XCC (XCD) index of the executing compute unit.
__device__ __forceinline__ int32_t xcc_id() {
    return (int32_t)(__builtin_amdgcn_s_getreg((3 << 11) | (0 << 6) | 20) & 15u);
}

// Workgroup-wide scalars (LDS).
struct GState {
    int32_t group, rank, gsize, flag;
    unsigned long long epoch;       // group barriers passed
    long long task;
    int32_t count;                  // bottom-up candidates of this workgroup
    unsigned long long dsum;        // degree sum of the vertices this workgroup appended this level
};

struct GCount {
    unsigned long long arcs_fwd, arcs_bwd, dag, reached, tasks, td, bu, arcs_reached;
};

// Group barrier.  Contains block barriers: every thread calls it.  Returns
// false when the group has aborted.
__device__ bool group_sync(GState &gs, GroupCtl *ctl, const Params &p) {
    // this wave's stores and atomics have reached L2
    asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
    __syncthreads();
    if (threadIdx.x == 0) {
        const unsigned long long target = (gs.epoch + 1ULL) * (unsigned long long)gs.gsize;
        atomicAdd(&ctl->bar.v, 1ULL);
        gs.epoch += 1ULL;
        const unsigned long long t0 = wall_clock64();
        int32_t ok = 1;
        while (ldg_u64(&ctl->bar.v) < target) {
            if (ldg_u64(&ctl->abort.v) != 0ULL) {
                ok = 0;
                break;
            }
            if ((long long)(wall_clock64() - t0) > p.xg_timeout) {
                atomicOr(&p.st->err, kErrInternal);
                atomicAdd(&ctl->abort.v, 1ULL);
                ok = 0;
                break;
            }
            __builtin_amdgcn_s_sleep(1);
        }
        if (ok && ldg_u64(&ctl->abort.v) != 0ULL) ok = 0;
        gs.flag = ok;
    }
    __syncthreads();
    return gs.flag != 0;
}

// Block-wide exclusive scan (three block barriers).
template <int BLOCK>
__device__ __forceinline__ int32_t gscan(int32_t x, int32_t *wsum, int32_t &total) {
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

// The thread's kGChunk arcs starting at tile arc i0: row kk[j] (or -1 past
// the end) and head w[j].
template <int BLOCK>
__device__ __forceinline__ void gchunk(const Tile<BLOCK> &sm, const int32_t *ci, int32_t cnt, int32_t total,
                                       int32_t i0, int32_t (&kk)[kGChunk], int32_t (&w)[kGChunk]) {
    int32_t k = (i0 < total) ? tile_search(sm.pre, cnt, i0) : 0;
#pragma unroll
    for (int j = 0; j < kGChunk; ++j) {
        const int32_t i = i0 + j;
        kk[j] = -1;
        w[j] = 0;
        if (i < total) {
            while (sm.pre[k + 1] <= i) ++k;
            kk[j] = k;
            w[j] = ci[sm.a0[k] + (i - sm.pre[k])];
        }
    }
}

// Appends the lanes' new vertices (fresh[j]: vertex v[j], first arc a0[j],
// degree dg[j]) to the group's level list at [base_off + position): one
// global atomic per wave for the positions; the degrees are summed into
// the workgroup's LDS accumulator *dsum.
template <int K>
__device__ __forceinline__ void gappend(const bool (&fresh)[K], const int32_t (&v)[K], const int32_t (&a0)[K],
                                        const int32_t (&dg)[K], int32_t *lv, int32_t *la, int32_t *ld,
                                        int32_t base_off, int32_t cap, GroupLine *acc, unsigned long long *dsum,
                                        DevStatus *st) {
    int32_t nf = 0;
    long long ds = 0;
#pragma unroll
    for (int j = 0; j < K; ++j) {
        nf += fresh[j] ? 1 : 0;
        ds += fresh[j] ? (long long)dg[j] : 0LL;
    }
    const int32_t incl = wave_incl_scan<int32_t>(nf);
    const int32_t tot = __shfl(incl, kWave - 1, kWave);
    if (tot == 0) return;
    const int lane = lane_id();
    int32_t base = 0;
    if (lane == kWave - 1) base = (int32_t)atomicAdd(&acc->v, (unsigned long long)tot);
    base = __shfl(base, kWave - 1, kWave);
    ds = wave_sum<long long>(ds);
    if (lane == 0) atomicAdd(dsum, (unsigned long long)ds);
    int32_t pos = base + incl - nf;
#pragma unroll
    for (int j = 0; j < K; ++j) {
        if (fresh[j]) {
            if (pos < cap) {
                lv[base_off + pos] = v[j];
                la[base_off + pos] = a0[j];
                ld[base_off + pos] = dg[j];
            } else {
                atomicOr(&st->err, kErrInternal);
            }
            ++pos;
        }
    }
}

// Stages list entries [tb, tb + cnt) into the tile (vertex, first arc,
// degree prefix); val = the entries' path counts when want_sigma.
template <int BLOCK>
__device__ __forceinline__ int32_t gstage(Tile<BLOCK> &sm, const int32_t *lv, const int32_t *la, const int32_t *ld,
                                          const unsigned long long *sig, int32_t tb, int32_t cnt) {
    const int tid = threadIdx.x;
    int32_t dg = 0;
    if (tid < cnt) {
        const int32_t v = ldg_i32(lv + tb + tid);
        sm.v[tid] = v;
        sm.a0[tid] = ldg_i32(la + tb + tid);
        dg = ldg_i32(ld + tb + tid);
        sm.val.u[tid] = ldg_u64(sig + v);
    }
    int32_t total;
    const int32_t ex = gscan<BLOCK>(dg, sm.wsum, total);
    if (tid < cnt) sm.pre[tid] = ex;
    if (tid == 0) sm.pre[cnt] = total;
    return total;
}

}  // namespace

template <int BLOCK>
// 1024 threads: one workgroup per compute unit; 512: two (4 waves per SIMD)
__global__ __launch_bounds__(BLOCK, BLOCK == 512 ? 4 : 1) void k_brandes_group(Params p) {
    extern __shared__ uint32_t lbm[];     // visited bitmap of the current source
    __shared__ Tile<BLOCK> sm;
    __shared__ GState gs;
    const int tid = threadIdx.x;
    GroupCtl *ctls = reinterpret_cast<GroupCtl *>(p.xg_ctl);
    unsigned int *reg = p.xg_reg;   // [0, 16): workgroups per XCC id; [16]: total

    // registration: group = (dense XCD index, rank modulo groups per XCD)
    if (tid == 0) {
        gs.flag = 1;
        gs.epoch = 0ULL;
        if (p.st->err & kErrGraph) gs.flag = 0;
        const int32_t x = xcc_id();
        const int32_t r = (int32_t)atomicAdd(&reg[x], 1u);
        atomicAdd(&reg[16], 1u);
        const unsigned long long t0 = wall_clock64();
        while (ldg_u32(&reg[16]) < gridDim.x) {
            if ((long long)(wall_clock64() - t0) > p.xg_timeout) {
                atomicOr(&p.st->err, kErrInternal);
                gs.flag = 0;
                break;
            }
            __builtin_amdgcn_s_sleep(2);
        }
        int32_t xd = 0, distinct = 0;
        for (int32_t i = 0; i < 16; ++i) {
            const bool used = ldg_u32(&reg[i]) > 0u;
            if (i < x) xd += used ? 1 : 0;
            distinct += used ? 1 : 0;
        }
        const int32_t cnt = (int32_t)ldg_u32(&reg[x]);
        const int32_t gpx = p.xg_gpx;
        const int32_t sub = r % gpx;
        gs.group = xd * gpx + sub;
        gs.rank = r / gpx;
        gs.gsize = (cnt - sub + gpx - 1) / gpx;
        // (candidate segments are sized for at most 64 members; a group must
        // not span XCDs, so every XCD the device has must report its own id)
        if (gs.group >= p.xg_groups || gs.gsize > 64 || distinct != p.xg_nxcc) {
            atomicOr(&p.st->err, kErrInternal);
            gs.flag = 0;
        }
    }
    __syncthreads();
    if (!gs.flag) return;
    const int32_t G = gs.gsize, rank = gs.rank, grp = gs.group;
    GroupCtl *ctl = ctls + grp;
    const long long off = (long long)grp * p.stride;
    unsigned long long *sig = p.sigma + off;
    int32_t *lv = p.lv + off;
    int32_t *la = p.la + off;
    int32_t *ld = p.ld + off;
    int32_t *lvl = p.lvl + off;
    GCount c = {0, 0, 0, 0, 0, 0, 0, 0};
    const bool lead = rank == 0;

    for (long long it = 0;; ++it) {
        // the leader takes the next task and broadcasts it; the reset of the
        // previous task is complete (barrier at the end of the loop)
        if (lead && tid == 0) {
            const long long t = (long long)atomicAdd(&p.st->head, 1ULL);
            ctl->task[it & 1].v = (unsigned long long)t;
        }
        if (!group_sync(gs, ctl, p)) break;
        if (tid == 0) gs.task = (long long)ldg_u64(&ctl->task[it & 1].v);
        __syncthreads();
        const long long task = gs.task;
        if (task >= p.ntasks) break;

        // graph and source of the task
        const int32_t *rp = p.rowptr;
        const int32_t *ci = p.colidx;
        int32_t n = p.n;
        long long vbase = 0;
        int32_t src;
        const uint32_t *iso = p.iso;
        if (p.G > 0) {
            int32_t lo = 0, hi = p.G - 1;
            while (lo < hi) {
                const int32_t mid = (lo + hi + 1) >> 1;
                if (p.g_task[mid] <= task) lo = mid; else hi = mid - 1;
            }
            const int32_t gid = p.g_order[lo];
            const long long v0 = p.g_vtx[gid];
            rp = p.rowptr + v0 + gid;
            ci = p.colidx + p.g_arc[gid];
            n = (int32_t)(p.g_vtx[gid + 1] - v0);
            vbase = v0;
            src = (int32_t)(task - p.g_task[lo]);
            iso = nullptr;
        } else {
            src = p.sources ? p.sources[task] : (int32_t)task;
        }
        if (src < 0 || src >= n) {
            if (lead && tid == 0) atomicOr(&p.st->err, kErrArg);
            // keep the group in step: the loop's next barrier follows
            continue;
        }
        const int32_t nw = (n + 31) >> 5;
        const long long m_all = (long long)(rp[n] - rp[0]);
        double *bcg = p.bc + vbase;

        // this workgroup's bitmap: isolated vertices and padding marked
        for (int32_t wi = tid; wi < nw; wi += BLOCK) {
            uint32_t x = iso ? iso[wi] : 0u;
            const int32_t hi = (wi + 1) * 32;
            if (hi > n) x |= ~0u << (32 - (hi - n));
            lbm[wi] = x;
        }
        __syncthreads();
        const int32_t a_src = rp[src];
        const int32_t d_src = rp[src + 1] - a_src;
        if (tid == 0) lbm[src >> 5] |= 1u << (src & 31);
        if (lead && tid == 0) {
            // every member has finished the previous task (the barrier above):
            // the first two levels' accumulators can be cleared
            ctl->acc[0].v = 0ULL;
            ctl->acc[0].w = 0ULL;
            ctl->acc[1].v = 0ULL;
            ctl->acc[1].w = 0ULL;
            sig[src] = 1ULL;
            lv[0] = src;
            la[0] = a_src;
            ld[0] = d_src;
            lvl[0] = 0;
            lvl[1] = 1;
        }
        double mf = (double)d_src;
        double mu = (double)(m_all - d_src);
        int32_t f0 = 0, f1 = 1;
        if (lead && tid == 0) c.arcs_reached += (unsigned long long)d_src;
        // sigma[src] and the source entry are visible to the group
        if (!group_sync(gs, ctl, p)) break;

        // ------------------------------------------------------- forward --
        int32_t d = 0;
        bool ok = true;
        for (;;) {
            GroupLine *acc = &ctl->acc[d & (kAccSlots - 1)];
            const bool bu = (p.bu_ratio > 0.0f) && (mu < (double)p.bu_ratio * mf);
            const int32_t cap = n - f1;
            if (tid == 0) {
                if (bu) c.bu++; else c.td++;
            }
            if (tid == 0) gs.dsum = 0ULL;
            if (bu) {
                // this workgroup's candidates: the unvisited vertices of the
                // bitmap words rank, rank + G, ..., compacted into its segment
                // of the group's candidate array
                const int32_t kw = (nw - rank + G - 1) / G;   // words of this workgroup
                int32_t *cand = p.cand + (long long)grp * p.xg_cand_stride +
                                (long long)rank * (long long)((nw + G - 1) / G) * 32;
                if (tid == 0) gs.count = 0;
                __syncthreads();
                for (int32_t k0 = 0; k0 < kw; k0 += BLOCK) {
                    const int32_t k = k0 + tid;
                    const int32_t wi = rank + G * k;
                    uint32_t bits = (k < kw) ? ~lbm[wi] : 0u;
                    const int32_t nb = __popc(bits);
                    const int32_t incl = wave_incl_scan<int32_t>(nb);
                    const int32_t wtot = __shfl(incl, kWave - 1, kWave);
                    int32_t base = 0;
                    if (lane_id() == kWave - 1 && wtot > 0) base = atomicAdd(&gs.count, wtot);
                    base = __shfl(base, kWave - 1, kWave);
                    int32_t pos = base + incl - nb;
                    while (bits) {
                        const int b = __ffs(bits) - 1;
                        bits &= bits - 1u;
                        cand[pos++] = wi * 32 + b;
                    }
                }
                __syncthreads();
                const int32_t nc = gs.count;
                // each candidate sums the path counts of its marked (= level d)
                // neighbours
                for (int32_t tb = 0; tb < nc; tb += BLOCK) {
                    const int32_t cnt = min(BLOCK, nc - tb);
                    int32_t v = 0, a0 = 0, dg = 0;
                    if (tid < cnt) {
                        v = cand[tb + tid];
                        a0 = rp[v];
                        dg = rp[v + 1] - a0;
                        sm.v[tid] = v;
                        sm.a0[tid] = a0;
                        sm.val.u[tid] = 0ULL;
                    }
                    int32_t total;
                    const int32_t ex = gscan<BLOCK>(dg, sm.wsum, total);
                    if (tid < cnt) sm.pre[tid] = ex;
                    if (tid == 0) sm.pre[cnt] = total;
                    __syncthreads();
                    if (tid == 0) c.arcs_fwd += (unsigned long long)total;
                    for (int32_t rb = 0; rb < total; rb += BLOCK * kGChunk) {
                        int32_t kk[kGChunk], u[kGChunk];
                        gchunk<BLOCK>(sm, ci, cnt, total, rb + tid * kGChunk, kk, u);
                        unsigned long long sv[kGChunk];
#pragma unroll
                        for (int j = 0; j < kGChunk; ++j)
                            sv[j] = (kk[j] >= 0 && lbit(lbm, u[j])) ? ldg_u64(sig + u[j]) : 0ULL;
                        int32_t kcur = kk[0];
                        unsigned long long sacc = 0ULL;
#pragma unroll
                        for (int j = 0; j < kGChunk; ++j) {
                            if (kk[j] < 0) continue;
                            if (kk[j] != kcur) {
                                if (sacc) {
                                    const unsigned long long o = atomicAdd(&sm.val.u[kcur], sacc);
                                    if (o + sacc < o) atomicOr(&p.st->err, kErrOverflow);
                                }
                                kcur = kk[j];
                                sacc = 0ULL;
                            }
                            if (sv[j]) {
                                const unsigned long long ns = sacc + sv[j];
                                if (ns < sacc) atomicOr(&p.st->err, kErrOverflow);
                                sacc = ns;
                                c.dag++;
                            }
                        }
                        if (sacc) {
                            const unsigned long long o = atomicAdd(&sm.val.u[kcur], sacc);
                            if (o + sacc < o) atomicOr(&p.st->err, kErrOverflow);
                        }
                    }
                    __syncthreads();
                    bool fresh[1] = {false};
                    const int32_t vv[1] = {v}, aa[1] = {a0}, dd[1] = {dg};
                    if (tid < cnt) {
                        const unsigned long long sum = sm.val.u[tid];
                        if (sum != 0ULL) {
                            sig[v] = sum;
                            fresh[0] = true;
                        }
                    }
                    gappend<1>(fresh, vv, aa, dd, lv, la, ld, f1, cap, acc, &gs.dsum, p.st);
                    __syncthreads();
                }
            } else {
                // top-down: this workgroup's tiles of the frontier list
                for (int32_t tb = f0 + rank * BLOCK; tb < f1; tb += G * BLOCK) {
                    const int32_t cnt = min(BLOCK, f1 - tb);
                    const int32_t total = gstage<BLOCK>(sm, lv, la, ld, sig, tb, cnt);
                    __syncthreads();
                    if (tid == 0) c.arcs_fwd += (unsigned long long)total;
                    for (int32_t rb = 0; rb < total; rb += BLOCK * kGChunk) {
                        int32_t kk[kGChunk], w[kGChunk];
                        gchunk<BLOCK>(sm, ci, cnt, total, rb + tid * kGChunk, kk, w);
                        bool act[kGChunk], fresh[kGChunk];
                        unsigned long long add[kGChunk], old[kGChunk];
                        int32_t fa[kGChunk], fd[kGChunk];
#pragma unroll
                        for (int j = 0; j < kGChunk; ++j) {
                            act[j] = kk[j] >= 0 && !lbit(lbm, w[j]);
                            add[j] = act[j] ? sm.val.u[kk[j]] : 0ULL;
                        }
#pragma unroll
                        for (int j = 0; j < kGChunk; ++j) old[j] = act[j] ? atomicAdd(sig + w[j], add[j]) : 1ULL;
#pragma unroll
                        for (int j = 0; j < kGChunk; ++j) {
                            fresh[j] = act[j] && old[j] == 0ULL;
                            if (act[j]) {
                                c.dag++;
                                if (old[j] + add[j] < old[j]) atomicOr(&p.st->err, kErrOverflow);
                            }
                            fa[j] = fresh[j] ? rp[w[j]] : 0;
                            fd[j] = fresh[j] ? rp[w[j] + 1] : 0;
                        }
#pragma unroll
                        for (int j = 0; j < kGChunk; ++j) fd[j] -= fa[j];
                        gappend<kGChunk>(fresh, w, fa, fd, lv, la, ld, f1, cap, acc, &gs.dsum, p.st);
                    }
                    __syncthreads();
                }
            }
            __syncthreads();
            if (tid == 0 && gs.dsum) atomicAdd(&acc->w, gs.dsum);
            if (!group_sync(gs, ctl, p)) {
                ok = false;
                break;
            }
            // the new level: size, degree sum; mark it in this workgroup's bitmap
            int32_t nnew = (int32_t)min((unsigned long long)cap, ldg_u64(&acc->v));
            const double mf_new = (double)ldg_u64(&acc->w);
            for (int32_t i = f1 + tid; i < f1 + nnew; i += BLOCK) {
                const int32_t w = ldg_i32(lv + i);
                atomicOr(&lbm[w >> 5], 1u << (w & 31));
            }
            if (lead && tid == 0) {
                lvl[d + 2] = f1 + nnew;
                c.arcs_reached += (unsigned long long)mf_new;
                // level d + 2's accumulator (last read two levels ago)
                GroupLine *nxt = &ctl->acc[(d + 2) & (kAccSlots - 1)];
                nxt->v = 0ULL;
                nxt->w = 0ULL;
            }
            __syncthreads();
            if (nnew == 0) break;
            mu -= mf_new;
            mf = mf_new;
            f0 = f1;
            f1 = f1 + nnew;
            ++d;
        }
        if (!ok) break;
        const int32_t Ld = d;            // deepest non-empty level: list [f0, f1)
        const int32_t nreached = f1;
        if (lead && tid == 0) {
            c.reached += (unsigned long long)nreached;
            c.tasks++;
        }

        // ------------------------------------------------------ backward --
        if (Ld > 0) {
            // deepest level: coef = 1 / sigma; unmark it here
            for (int32_t i = f0 + rank * BLOCK + tid; i < f1; i += G * BLOCK) {
                const int32_t v = ldg_i32(lv + i);
                sig[v] = u64_of(1.0 / (double)ldg_u64(sig + v));
            }
            for (int32_t i = f0 + tid; i < f1; i += BLOCK) {
                const int32_t w = ldg_i32(lv + i);
                atomicAnd(&lbm[w >> 5], ~(1u << (w & 31)));
            }
            if (!group_sync(gs, ctl, p)) break;
            for (int32_t l = Ld - 1; l >= 1; --l) {
                const int32_t lo = ldg_i32(lvl + l), hi = ldg_i32(lvl + l + 1);
                const double wfac = p.linear ? (double)l / (double)(l + 1) : 1.0;
                for (int32_t tb = lo + rank * BLOCK; tb < hi; tb += G * BLOCK) {
                    const int32_t cnt = min(BLOCK, hi - tb);
                    const int32_t total = gstage<BLOCK>(sm, lv, la, ld, sig, tb, cnt);
                    // the rows' path counts move to registers; val takes the sums
                    __syncthreads();
                    const unsigned long long my_sigma = tid < cnt ? sm.val.u[tid] : 0ULL;
                    __syncthreads();
                    sm.val.f[tid] = 0.0;
                    __syncthreads();
                    if (tid == 0) c.arcs_bwd += (unsigned long long)total;
                    for (int32_t rb = 0; rb < total; rb += BLOCK * kGChunk) {
                        int32_t kk[kGChunk], w[kGChunk];
                        gchunk<BLOCK>(sm, ci, cnt, total, rb + tid * kGChunk, kk, w);
                        double cf[kGChunk];
#pragma unroll
                        for (int j = 0; j < kGChunk; ++j)
                            cf[j] = (kk[j] >= 0 && !lbit(lbm, w[j])) ? f64_of(ldg_u64(sig + w[j])) : 0.0;
                        int32_t kcur = kk[0];
                        double s = 0.0;
#pragma unroll
                        for (int j = 0; j < kGChunk; ++j) {
                            if (kk[j] < 0) continue;
                            if (kk[j] != kcur) {
                                if (s != 0.0) atomicAdd(&sm.val.f[kcur], s);
                                kcur = kk[j];
                                s = 0.0;
                            }
                            s += cf[j];
                        }
                        if (s != 0.0) atomicAdd(&sm.val.f[kcur], s);
                    }
                    __syncthreads();
                    if (tid < cnt) {
                        const int32_t v = sm.v[tid];
                        const double sg = (double)my_sigma;
                        const double delta = sg * sm.val.f[tid] * wfac;
                        sig[v] = u64_of((1.0 + delta) / sg);
                        if (delta != 0.0) atomicAdd(bcg + v, delta);
                    }
                    __syncthreads();
                }
                // level l is done in this workgroup: unmark it in its bitmap
                for (int32_t i = lo + tid; i < hi; i += BLOCK) {
                    const int32_t w = ldg_i32(lv + i);
                    atomicAnd(&lbm[w >> 5], ~(1u << (w & 31)));
                }
                // level l's coefficients are visible before level l - 1 pulls
                if (!group_sync(gs, ctl, p)) {
                    ok = false;
                    break;
                }
            }
            if (!ok) break;
        }

        // reset: path counts of the reached vertices back to zero
        for (int32_t i = rank * BLOCK + tid; i < nreached; i += G * BLOCK) sig[ldg_i32(lv + i)] = 0ULL;
        if (lead && tid == 0) atomicAdd(&p.st->stat[kStDone], 1ULL);
    }

    // counters: wave sums, one atomic per wave and counter
    const unsigned long long dag = wave_sum<unsigned long long>(c.dag);
    if (lane_id() == 0 && dag) atomicAdd(&p.st->stat[kStDag], dag);
    if (tid == 0) {
        atomicAdd(&p.st->stat[kStSources], c.tasks);
        atomicAdd(&p.st->stat[kStReached], c.reached);
        atomicAdd(&p.st->stat[kStArcsFwd], c.arcs_fwd);
        atomicAdd(&p.st->stat[kStArcsBwd], c.arcs_bwd);
        atomicAdd(&p.st->stat[kStTd], c.td);
        atomicAdd(&p.st->stat[kStBu], c.bu);
        atomicAdd(&p.st->stat[kStArcsReached], c.arcs_reached);
    }
}

template <int BLOCK>
static void launch_group(dim3 grid, dim3 block, size_t lds, hipStream_t s, const Params &p) {
    hipLaunchKernelGGL((k_brandes_group<BLOCK>), grid, block, lds, s, p);
}

KernelRef brandes_group_kernel(int block) {
    if (block == 512) return KernelRef{(const void *)&k_brandes_group<512>, &launch_group<512>};
    return KernelRef{(const void *)&k_brandes_group<1024>, &launch_group<1024>};
}

size_t group_ctl_bytes() { return sizeof(GroupCtl); }

}  // namespace nk
