// Degree-descending vertex relabelling.
//
// Before a run the library renumbers the vertices of a single graph by
// non-increasing degree (ties by original id): hubs get the smallest ids, so
// the per-source path counts that nearly every shortest-path DAG arc touches
// share a few cache lines, and isolated vertices move to the end.  Each
// adjacency list keeps its original order (only the ids are renamed), so a
// scan of a list meets neighbours in the same order as in the input -- the
// path walk of pair sampling therefore picks the same vertices.  Results
// are mapped back to original ids before they are returned.
#include <hipcub/hipcub.hpp>

#include "nk_runtime.h"

namespace nk {

__global__ void k_deg_keys(const int32_t *rowptr, int32_t n, uint32_t *key, int32_t *id, const DevStatus *st) {
    if (st->err & kErrGraph) return;
    const long long stride = (long long)gridDim.x * blockDim.x;
    for (long long v = (long long)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += stride) {
        key[v] = 0x7fffffffu - (uint32_t)(rowptr[v + 1] - rowptr[v]);
        id[v] = (int32_t)v;
    }
}

__global__ void k_perm_degrees(const int32_t *rowptr, const int32_t *inv, int32_t n, int32_t *perm, int32_t *deg_new,
                               const DevStatus *st) {
    if (st->err & kErrGraph) return;
    const long long stride = (long long)gridDim.x * blockDim.x;
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i <= n; i += stride) {
        if (i == n) {
            deg_new[n] = 0;
            continue;
        }
        const int32_t o = inv[i];
        perm[o] = (int32_t)i;
        deg_new[i] = rowptr[o + 1] - rowptr[o];
    }
}

// One wave per internal vertex copies its adjacency list, renamed.
__global__ void k_relabel_arcs(const int32_t *rowptr, const int32_t *colidx, const int32_t *inv, const int32_t *perm,
                               const int32_t *rp_new, int32_t n, int32_t *ci_new, const DevStatus *st) {
    if (st->err & kErrGraph) return;
    const long long waves = (long long)gridDim.x * (blockDim.x / kWave);
    const int lane = lane_id();
    for (long long i = (long long)blockIdx.x * (blockDim.x / kWave) + wave_id(); i < n; i += waves) {
        const int32_t o = inv[i];
        const int32_t a = rowptr[o], b = rowptr[o + 1], base = rp_new[i];
        for (int32_t j = lane; j < b - a; j += kWave) ci_new[base + j] = perm[colidx[a + j]];
    }
}

__global__ void k_map_sources(const int32_t *src, int32_t k, const int32_t *perm, int32_t n, int32_t *out) {
    const long long stride = (long long)gridDim.x * blockDim.x;
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i < k; i += stride) {
        const int32_t v = src[i];
        out[i] = (v >= 0 && v < n) ? perm[v] : -1;
    }
}

__global__ void k_gather_scale(const double *in, const int32_t *perm, int32_t n, double scale, double *out) {
    const long long stride = (long long)gridDim.x * blockDim.x;
    for (long long v = (long long)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += stride)
        out[v] = in[perm[v]] * scale;
}

__global__ void k_gather_u32(const uint32_t *in, const int32_t *perm, int32_t n, uint32_t *out) {
    const long long stride = (long long)gridDim.x * blockDim.x;
    for (long long v = (long long)blockIdx.x * blockDim.x + threadIdx.x; v < n; v += stride) out[v] = in[perm[v]];
}

// Per-arc values of the relabelled CSR back to the caller's arc order: the
// relabelling keeps each adjacency list's order, so arc j of internal
// vertex i is arc j of original vertex inv[i].  One wave per vertex.
__global__ void k_arcs_back(const double *in, const int32_t *rp_new, const int32_t *inv, const int32_t *rowptr,
                            int32_t n, double *out) {
    const long long waves = (long long)gridDim.x * (blockDim.x / kWave);
    const int lane = lane_id();
    for (long long i = (long long)blockIdx.x * (blockDim.x / kWave) + wave_id(); i < n; i += waves) {
        const int32_t a = rp_new[i], b = rp_new[i + 1], o = rowptr[inv[i]];
        for (int32_t j = lane; j < b - a; j += kWave) out[o + j] = in[a + j];
    }
}

// Per-arc int32 values into the relabelled arc order (the inverse of
// k_arcs_back): arc j of internal vertex i is arc j of original vertex inv[i].
__global__ void k_arcs_fwd_i32(const int32_t *in, const int32_t *rp_new, const int32_t *inv, const int32_t *rowptr,
                               int32_t n, int32_t *out, const DevStatus *st) {
    if (st->err & kErrGraph) return;
    const long long waves = (long long)gridDim.x * (blockDim.x / kWave);
    const int lane = lane_id();
    for (long long i = (long long)blockIdx.x * (blockDim.x / kWave) + wave_id(); i < n; i += waves) {
        const int32_t a = rp_new[i], b = rp_new[i + 1], o = rowptr[inv[i]];
        for (int32_t j = lane; j < b - a; j += kWave) out[a + j] = in[o + j];
    }
}

// Row lengths of a second CSR over the same vertices (the in-arcs of a
// directed graph) in internal order, plus a zero at n for the scan.
__global__ void k_inv_degrees(const int32_t *rowptr, const int32_t *inv, int32_t n, int32_t *deg_new,
                              const DevStatus *st) {
    if (st->err & kErrGraph) return;
    const long long stride = (long long)gridDim.x * blockDim.x;
    for (long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x; i <= n; i += stride) {
        if (i == n) {
            deg_new[n] = 0;
            continue;
        }
        const int32_t o = inv[i];
        deg_new[i] = rowptr[o + 1] - rowptr[o];
    }
}

static unsigned grid_of(long long count, int block) {
    long long g = (count + block - 1) / block;
    return (unsigned)(g < 1 ? 1 : (g > 65536 ? 65536 : g));
}

nk_status relabel_graph(const int32_t *rowptr, const int32_t *colidx, int32_t n, int64_t m, const DevStatus *st,
                        Scratch &scr, hipStream_t s, Relabeled *out) {
    nk_status rc;
    uint32_t *key_in, *key_out;
    int32_t *id_in, *inv, *perm, *deg_new, *rp_new, *ci_new;
    if ((rc = scr.get(n, &key_in)) != NK_OK) return rc;
    if ((rc = scr.get(n, &key_out)) != NK_OK) return rc;
    if ((rc = scr.get(n, &id_in)) != NK_OK) return rc;
    if ((rc = scr.get(n, &inv)) != NK_OK) return rc;
    if ((rc = scr.get(n, &perm)) != NK_OK) return rc;
    if ((rc = scr.get((long long)n + 1, &deg_new)) != NK_OK) return rc;
    if ((rc = scr.get((long long)n + 1, &rp_new)) != NK_OK) return rc;
    if ((rc = scr.get(m > 0 ? m : 1, &ci_new)) != NK_OK) return rc;
    hipLaunchKernelGGL(k_deg_keys, dim3(grid_of(n, 256)), dim3(256), 0, s, rowptr, n, key_in, id_in, st);
    NK_HIP(hipGetLastError());
    size_t sort_bytes = 0, scan_bytes = 0;
    NK_HIP(hipcub::DeviceRadixSort::SortPairs(nullptr, sort_bytes, key_in, key_out, id_in, inv, n, 0, 32, s));
    NK_HIP(hipcub::DeviceScan::ExclusiveSum(nullptr, scan_bytes, deg_new, rp_new, n + 1, s));
    void *tmp;
    if ((rc = scr.get(std::max(sort_bytes, scan_bytes), &tmp)) != NK_OK) return rc;
    NK_HIP(hipcub::DeviceRadixSort::SortPairs(tmp, sort_bytes, key_in, key_out, id_in, inv, n, 0, 32, s));
    hipLaunchKernelGGL(k_perm_degrees, dim3(grid_of((long long)n + 1, 256)), dim3(256), 0, s, rowptr, inv, n, perm,
                       deg_new, st);
    NK_HIP(hipGetLastError());
    NK_HIP(hipcub::DeviceScan::ExclusiveSum(tmp, scan_bytes, deg_new, rp_new, n + 1, s));
    hipLaunchKernelGGL(k_relabel_arcs, dim3(grid_of((long long)n * kWave, 256)), dim3(256), 0, s, rowptr, colidx, inv,
                       perm, rp_new, n, ci_new, st);
    NK_HIP(hipGetLastError());
    out->rowptr = rp_new;
    out->colidx = ci_new;
    out->perm = perm;
    out->inv = inv;
    return NK_OK;
}

nk_status relabel_weights(const int32_t *wts, const int32_t *rowptr, int32_t n, int64_t m, const Relabeled &g,
                          const DevStatus *st, Scratch &scr, hipStream_t s, int32_t **out) {
    nk_status rc;
    if ((rc = scr.get(m > 0 ? m : 1, out)) != NK_OK) return rc;
    if (m == 0) return NK_OK;
    hipLaunchKernelGGL(k_arcs_fwd_i32, dim3(grid_of((long long)n * kWave, 256)), dim3(256), 0, s, wts, g.rowptr,
                       g.inv, rowptr, n, *out, st);
    NK_HIP(hipGetLastError());
    return NK_OK;
}

nk_status relabel_second_csr(const int32_t *rowptr2, const int32_t *colidx2, int32_t n, int64_t m, const Relabeled &g,
                             const DevStatus *st, Scratch &scr, hipStream_t s, int32_t **rp_out, int32_t **ci_out) {
    nk_status rc;
    int32_t *deg_new, *rp_new, *ci_new;
    if ((rc = scr.get((long long)n + 1, &deg_new)) != NK_OK) return rc;
    if ((rc = scr.get((long long)n + 1, &rp_new)) != NK_OK) return rc;
    if ((rc = scr.get(m > 0 ? m : 1, &ci_new)) != NK_OK) return rc;
    size_t scan_bytes = 0;
    NK_HIP(hipcub::DeviceScan::ExclusiveSum(nullptr, scan_bytes, deg_new, rp_new, n + 1, s));
    void *tmp;
    if ((rc = scr.get(scan_bytes > 0 ? scan_bytes : 1, &tmp)) != NK_OK) return rc;
    hipLaunchKernelGGL(k_inv_degrees, dim3(grid_of((long long)n + 1, 256)), dim3(256), 0, s, rowptr2, g.inv, n,
                       deg_new, st);
    NK_HIP(hipGetLastError());
    NK_HIP(hipcub::DeviceScan::ExclusiveSum(tmp, scan_bytes, deg_new, rp_new, n + 1, s));
    hipLaunchKernelGGL(k_relabel_arcs, dim3(grid_of((long long)n * kWave, 256)), dim3(256), 0, s, rowptr2, colidx2,
                       g.inv, g.perm, rp_new, n, ci_new, st);
    NK_HIP(hipGetLastError());
    *rp_out = rp_new;
    *ci_out = ci_new;
    return NK_OK;
}

hipError_t launch_map_sources(const int32_t *src, int32_t k, const int32_t *perm, int32_t n, int32_t *out,
                              hipStream_t s) {
    hipLaunchKernelGGL(k_map_sources, dim3(grid_of(k, 256)), dim3(256), 0, s, src, k, perm, n, out);
    return hipGetLastError();
}

hipError_t launch_gather_scale(const double *in, const int32_t *perm, int32_t n, double scale, double *out,
                               hipStream_t s) {
    hipLaunchKernelGGL(k_gather_scale, dim3(grid_of(n, 256)), dim3(256), 0, s, in, perm, n, scale, out);
    return hipGetLastError();
}

hipError_t launch_arcs_back(const double *in, const int32_t *rp_new, const int32_t *inv, const int32_t *rowptr,
                            int32_t n, double *out, hipStream_t s) {
    hipLaunchKernelGGL(k_arcs_back, dim3(grid_of((long long)n * kWave, 256)), dim3(256), 0, s, in, rp_new, inv, rowptr,
                       n, out);
    return hipGetLastError();
}

hipError_t launch_gather_u32(const uint32_t *in, const int32_t *perm, int32_t n, uint32_t *out, hipStream_t s) {
    hipLaunchKernelGGL(k_gather_u32, dim3(grid_of(n, 256)), dim3(256), 0, s, in, perm, n, out);
    return hipGetLastError();
}

}  // namespace nk
