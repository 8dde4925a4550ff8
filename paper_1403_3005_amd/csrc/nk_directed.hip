// Directed graphs: the in-arc CSR (transpose) that bottom-up levels scan,
// and a consistency check of a caller-supplied one.
//
// The transpose is built by one radix sort of the arc keys (head << 32 |
// tail): rows come out sorted by tail, the row offsets are read off the
// sorted heads.  The check compares every vertex's in-degree, counted from
// the out-arcs, with the row lengths of the supplied in-arc CSR.
#include <hipcub/hipcub.hpp>

#include "nk_runtime.h"

namespace nk {

namespace {

unsigned grid_of(long long count, int block) {
    long long g = (count + block - 1) / block;
    if (g < 1) g = 1;
    if (g > 65536) g = 65536;
    return (unsigned)g;
}

// One wave per vertex writes the keys of its out-arcs.
__global__ void k_arc_keys(const int32_t *rowptr, const int32_t *colidx, int32_t n, unsigned long long *keys) {
    const long long waves = (long long)gridDim.x * (blockDim.x / kWave);
    const int lane = lane_id();
    for (long long v = (long long)blockIdx.x * (blockDim.x / kWave) + wave_id(); v < n; v += waves) {
        const int32_t a = rowptr[v], b = rowptr[v + 1];
        for (int32_t e = a + lane; e < b; e += kWave)
            keys[e] = ((unsigned long long)(uint32_t)colidx[e] << 32) | (unsigned long long)v;
    }
}

// Sorted keys -> in-arc CSR: tcolidx[e] = tail; trowptr[u] = first sorted
// position whose head is >= u.
__global__ void k_keys_to_csr(const unsigned long long *keys, long long m, int32_t n, int32_t *trowptr,
                              int32_t *tcolidx) {
    const long long stride = (long long)gridDim.x * blockDim.x;
    for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < m; e += stride) {
        const unsigned long long k = keys[e];
        const int32_t head = (int32_t)(k >> 32);
        tcolidx[e] = (int32_t)(k & 0xffffffffULL);
        const int32_t prev = e > 0 ? (int32_t)(keys[e - 1] >> 32) : -1;
        for (int32_t u = prev + 1; u <= head; ++u) trowptr[u] = (int32_t)e;
        if (e == m - 1)
            for (int32_t u = head + 1; u <= n; ++u) trowptr[u] = (int32_t)m;
    }
}

__global__ void k_in_degree(const int32_t *colidx, long long m, int32_t *cnt) {
    const long long stride = (long long)gridDim.x * blockDim.x;
    for (long long e = (long long)blockIdx.x * blockDim.x + threadIdx.x; e < m; e += stride) atomicAdd(&cnt[colidx[e]], 1);
}

__global__ void k_check_in_degree(const int32_t *cnt, const int32_t *trowptr, int32_t n, DevStatus *st) {
    const long long stride = (long long)gridDim.x * blockDim.x;
    bool bad = false;
    for (long long v = (long long)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += stride)
        bad |= cnt[v] != trowptr[v + 1] - trowptr[v];
    if (__ballot(bad) != 0ULL && lane_id() == 0) atomicOr(&st->err, kErrGraph);
}

}  // namespace

nk_status transpose_graph(const int32_t *rowptr, const int32_t *colidx, int32_t n, int64_t m, int32_t *trowptr,
                          int32_t *tcolidx, Scratch &scr, hipStream_t s) {
    if (m == 0) return launch_fill_i32(trowptr, 0, (long long)n + 1, s) == hipSuccess ? NK_OK : fail(NK_E_HIP, "fill");
    unsigned long long *k0, *k1;
    nk_status st;
    if ((st = scr.get(m, &k0)) != NK_OK) return st;
    if ((st = scr.get(m, &k1)) != NK_OK) return st;
    int bits = 1;
    while (bits < 31 && ((long long)1 << bits) <= (long long)n) ++bits;
    size_t tb = 0;
    NK_HIP(hipcub::DeviceRadixSort::SortKeys(nullptr, tb, k0, k1, (int)m, 0, 32 + bits, s));
    void *tmp;
    if ((st = scr.get(tb > 0 ? tb : 1, &tmp)) != NK_OK) return st;
    hipLaunchKernelGGL(k_arc_keys, dim3(grid_of((long long)n * kWave, 256)), dim3(256), 0, s, rowptr, colidx, n, k0);
    NK_HIP(hipGetLastError());
    NK_HIP(hipcub::DeviceRadixSort::SortKeys(tmp, tb, k0, k1, (int)m, 0, 32 + bits, s));
    hipLaunchKernelGGL(k_keys_to_csr, dim3(grid_of(m, 256)), dim3(256), 0, s, k1, (long long)m, n, trowptr, tcolidx);
    NK_HIP(hipGetLastError());
    return NK_OK;
}

nk_status check_transpose(const int32_t *colidx, int32_t n, int64_t m, const int32_t *trowptr, DevStatus *dst,
                          Scratch &scr, hipStream_t s) {
    int32_t *cnt;
    nk_status st;
    if ((st = scr.get((long long)n, &cnt)) != NK_OK) return st;
    NK_HIP(launch_fill_i32(cnt, 0, n, s));
    hipLaunchKernelGGL(k_in_degree, dim3(grid_of(m, 256)), dim3(256), 0, s, colidx, (long long)m, cnt);
    NK_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_check_in_degree, dim3(grid_of(n, 256)), dim3(256), 0, s, cnt, trowptr, n, dst);
    NK_HIP(hipGetLastError());
    return NK_OK;
}

}  // namespace nk
