// Device-side building blocks for the Brandes kernels (gfx950, wave64).
//
// Everything here runs inside one workgroup: wave-level scans and ballot
// compaction, a block-wide exclusive scan, the counter-based SplitMix64
// draw used by pair sampling, and the LDS tile that stages a slice of a
// vertex list (ids, adjacency starts, degree prefix sums, one 8-byte value
// per vertex) for load-balanced arc processing.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace nk {

constexpr int kWave = 64;

// Error bits raised by kernels; the host maps them to nk_status codes.
enum : int32_t {
    kErrGraph = 1,      // CSR structure check failed
    kErrArg = 2,        // a source id or pair index out of range
    kErrOverflow = 4,   // a path count wrapped past 2^64 - 1
    kErrInternal = 8    // list capacity exceeded (only after a wrap)
};

// Per-call device status block: error bits, the dynamic task counter and
// work counters (see nk_last_stats).
struct DevStatus {
    int32_t err;
    int32_t pad;
    unsigned long long head;
    unsigned long long stat[12];
    int32_t info[8];   // reserved
    unsigned long long cycles[8];  // shader clock cycles per phase, summed over workgroups
    unsigned long long sub[8];     // shader clock cycles per sub-phase
};

enum PhaseIdx { kPhInit = 0, kPhTd, kPhBu, kPhMark, kPhPull, kPhPush, kPhReset, kPhOther, kNumPhases };
// sub-phases of the bottom-up and pull levels (staging + scans, arc loop, finalize)
enum SubIdx { kSbBuStage = 0, kSbBuArcs, kSbBuFin, kSbPlStage, kSbPlArcs, kSbPlFin, kNumSub };
// pair mode reuses the first four slots: search, meeting-vertex choice, walks, clearing
enum PairSubIdx { kSbPairSearch = 0, kSbPairSelect, kSbPairWalk, kSbPairClear };

enum StatIdx {
    kStSources = 0, kStReached, kStArcsFwd, kStArcsBwd, kStDag, kStTd, kStBu, kStArcsReached, kStBwPush,
    kStDone,   // sources (or samples) finished so far, added as each task ends (progress of a long run)
    kStDeferred,   // pair samples left by the hashed-record launch to one with a record per vertex
    kNumStats = 12
};

__device__ __forceinline__ int lane_id() { return threadIdx.x & (kWave - 1); }
__device__ __forceinline__ int wave_id() { return threadIdx.x / kWave; }

// SplitMix64 output function (Steele, Lea, Flood 2014).
__device__ __forceinline__ uint64_t mix64(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

// Counter-based draw: output t+1 of a SplitMix64 stream whose seed is
// output j+1 of a stream whose seed is output stream+1 of the stream
// seeded with `seed` (k-th output of a stream seeded x = mix64(x + k*gamma)).
__device__ __forceinline__ uint64_t draw(uint64_t seed, uint64_t stream, uint64_t j, uint64_t t) {
    const uint64_t g = 0x9E3779B97F4A7C15ULL;
    uint64_t a = mix64(seed + (stream + 1) * g);
    uint64_t b = mix64(a + (j + 1) * g);
    return mix64(b + (t + 1) * g);
}

// floor(x * N / 2^64) (multiply-shift range reduction).
__device__ __forceinline__ uint64_t bounded(uint64_t x, uint64_t N) { return __umul64hi(x, N); }

template <typename T>
__device__ __forceinline__ T wave_incl_scan(T v) {
    const int lane = lane_id();
#pragma unroll
    for (int off = 1; off < kWave; off <<= 1) {
        T y = __shfl_up(v, off, kWave);
        if (lane >= off) v += y;
    }
    return v;
}

template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, kWave);
    return v;
}

__device__ __forceinline__ int32_t wave_min(int32_t v) {
#pragma unroll
    for (int off = kWave / 2; off > 0; off >>= 1) {
        int32_t y = __shfl_xor(v, off, kWave);
        v = y < v ? y : v;
    }
    return v;
}

// Shared-memory tile for BLOCK vertices plus block-level scalars.
template <int BLOCK>
struct Tile {
    int32_t v[BLOCK];          // vertex ids
    int32_t a0[BLOCK];         // rowptr[v]
    int32_t pre[BLOCK + 1];    // exclusive prefix of degrees, pre[cnt] = total arcs
    union {
        unsigned long long u[BLOCK];  // sigma of a frontier vertex / bottom-up path-count sum
        double f[BLOCK];              // backward: sum of (1 + delta_w) / sigma_w
    } val;
    int32_t wsum[BLOCK / kWave + 1];
    // block scalars
    long long task;
    long long mf;              // arcs leaving the current frontier
    long long mu;              // arcs of vertices not yet visited
    long long acc_mf;          // reduction target while marking a new level
    int32_t count;             // append counter (next level / candidates)
    int32_t redmin;
    int32_t flag;
    int32_t levels;
    int32_t lvl_lo[2];
    // timing (thread 0 only)
    unsigned long long cyc[8];
    unsigned long long sub[8];
    long long t0, ts;
};

// Block-wide exclusive scan of one int per thread; returns the thread's
// exclusive prefix and the block total.  Contains barriers: every thread of
// the block must call it.
template <int BLOCK>
__device__ __forceinline__ int32_t block_excl_scan(int32_t x, Tile<BLOCK> &sm, int32_t &total) {
    constexpr int NW = BLOCK / kWave;
    const int lane = lane_id(), wid = wave_id();
    int32_t incl = wave_incl_scan<int32_t>(x);
    if (lane == kWave - 1) sm.wsum[wid] = incl;
    __syncthreads();
    if (wid == 0) {
        int32_t s = lane < NW ? sm.wsum[lane] : 0;
        int32_t si = wave_incl_scan<int32_t>(s);
        if (lane < NW) sm.wsum[lane] = si - s;
        if (lane == NW - 1) sm.wsum[NW] = si;
    }
    __syncthreads();
    total = sm.wsum[NW];
    int32_t r = incl - x + sm.wsum[wid];
    __syncthreads();
    return r;
}

// Ballot compaction: every active lane of the wave calls this; lanes with
// pred write `value` to out[base + rank], where base comes from one LDS
// atomic per wave.  Positions >= cap are dropped and flagged.
__device__ __forceinline__ void wave_append(bool pred, int32_t value, int32_t *out, int32_t *counter,
                                            int32_t cap, int32_t *err) {
    unsigned long long mask = __ballot(pred);
    if (mask == 0ULL) return;
    const int lane = lane_id();
    const int leader = __ffsll((long long)mask) - 1;
    int32_t base = 0;
    if (lane == leader) base = atomicAdd(counter, (int32_t)__popcll(mask));
    base = __shfl(base, leader, kWave);
    if (pred) {
        int32_t pos = base + (int32_t)__popcll(mask & ((1ULL << lane) - 1ULL));
        if (pos < cap)
            out[pos] = value;
        else
            atomicOr(err, kErrInternal);
    }
}

// As wave_append, and returns the lane's position in `out` (or -1 when
// pred is false or the position is past cap).
__device__ __forceinline__ int32_t wave_append_pos(bool pred, int32_t value, int32_t *out, int32_t *counter,
                                                   int32_t cap, int32_t *err) {
    unsigned long long mask = __ballot(pred);
    if (mask == 0ULL) return -1;
    const int lane = lane_id();
    const int leader = __ffsll((long long)mask) - 1;
    int32_t base = 0;
    if (lane == leader) base = atomicAdd(counter, (int32_t)__popcll(mask));
    base = __shfl(base, leader, kWave);
    if (!pred) return -1;
    const int32_t pos = base + (int32_t)__popcll(mask & ((1ULL << lane) - 1ULL));
    if (pos < cap) {
        out[pos] = value;
        return pos;
    }
    atomicOr(err, kErrInternal);
    return -1;
}

// Largest k in [0, cnt) with pre[k] <= i (pre[0] = 0 <= i).
__device__ __forceinline__ int32_t tile_search(const int32_t *pre, int32_t cnt, int32_t i) {
    int32_t lo = 0, hi = cnt - 1;
    while (lo < hi) {
        int32_t mid = (lo + hi + 1) >> 1;
        if (pre[mid] <= i) lo = mid; else hi = mid - 1;
    }
    return lo;
}

}  // namespace nk
