// Graph preparation on the device: CSR validation, candidate ranking.
//
// Ranking follows the candidate order of sections II-C / III-E at the top level of the
// search: candidates of degree > 0 in ascending (degree, id).  Degree-0 vertices are left
// out because they belong to no biclique with two non-empty sides.

#include <rocprim/device/device_radix_sort.hpp>
#include <rocprim/device/device_segmented_radix_sort.hpp>

#include "mbe_internal.h"

namespace mbe {

namespace {

// Offsets: off[0] = 0, non-decreasing, off[n] = n_edges.  Rows: ids in [0, n_cols), strictly
// ascending.  Transpose: every (r, c) in this CSR appears as (c, r) in the other one (with
// equal edge counts and duplicate-free rows on both sides this makes them transposes).  Both
// directions in one launch (blockIdx.y = 1: the V-side CSR against the U-side one), one
// thread per offset and one per edge: an edge finds its row by binary search over the
// offsets (a hub row no longer rests on one thread).  Every read stays in bounds whatever
// the offsets hold; offsets that break the rules flag the graph whatever the edges say.
__global__ void validate_kernel(int32_t n_u, int32_t n_v, int32_t n_edges, const int32_t *u_off,
                                const int32_t *u_adj, const int32_t *v_off, const int32_t *v_adj,
                                unsigned int *flags) {
    const bool rev = blockIdx.y == 1;
    const int32_t n_rows = rev ? n_v : n_u, n_cols = rev ? n_u : n_v;
    const int32_t *off = rev ? v_off : u_off, *adj = rev ? v_adj : u_adj;
    const int32_t *t_off = rev ? u_off : v_off, *t_adj = rev ? u_adj : v_adj;
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const int64_t t0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    bool bad = false;
    for (int64_t r = t0; r <= n_rows; r += stride) {
        const int32_t o = off[r];
        if (o < 0 || o > n_edges || (r == 0 && o != 0) || (r == n_rows && o != n_edges) || (r > 0 && off[r - 1] > o))
            bad = true;
    }
    for (int64_t p = t0; p < n_edges; p += stride) {
        // the last row whose first edge is at or before p
        int32_t lo = 0, hi = n_rows - 1;
        while (lo < hi) {
            const int32_t mid = (int32_t)(((int64_t)lo + hi + 1) >> 1);
            if (off[mid] <= p) lo = mid;
            else hi = mid - 1;
        }
        const int32_t r = lo;
        const int32_t cidx = adj[p];
        if (cidx < 0 || cidx >= n_cols) {
            bad = true;
            continue;
        }
        if (p > 0 && p > off[r] && adj[p - 1] >= cidx) bad = true;  // (same row: ascending)
        int32_t a = t_off[cidx], b = t_off[cidx + 1];
        if (a < 0 || b > n_edges || a > b) {
            bad = true;
            continue;
        }
        const int32_t end = b;
        while (a < b) {
            const int32_t mid = a + (b - a) / 2;
            if (t_adj[mid] < r) a = mid + 1;
            else b = mid;
        }
        if (a >= end || t_adj[a] != r) bad = true;
    }
    if (__ballot(bad) && (threadIdx.x & 63) == 0) atomicOr(flags, (unsigned int)FLAG_BAD_GRAPH);
}

// keys[v] = (deg << 32) | v; stats[0] = number of degree-0 vertices, stats[1 + c] = number of
// candidates in mask class c (degree <= 64 << c), stats[8] = max degree, stats[9] = max over
// candidates of the 2-hop walk count sum_{w in N(v)} deg w (bounds a local universe).
__global__ void rank_keys_kernel(int32_t nc, const int32_t *c_off, const int32_t *c_adj, const int32_t *o_off,
                                 unsigned long long *keys, unsigned long long *stats) {
    // tallied per thread over its candidates, then summed (or maxed) over the wave: one atomic
    // per wave and statistic instead of one per candidate
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    unsigned long long cnt[8] = {0, 0, 0, 0, 0, 0, 0, 0};  // [0] degree 0, [1 + c] class c (c <= 6)
    unsigned long long dmax = 0, wmax = 0;
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < nc; v += stride) {
        const int32_t b = c_off[v], e = c_off[v + 1];
        const uint32_t d = (uint32_t)(e - b);
        keys[v] = ((unsigned long long)d << 32) | (unsigned long long)(uint32_t)v;
        if (d == 0) {
            ++cnt[0];
        } else {
            int cls = 0;
            while (cls < 6 && d > (64u << cls)) ++cls;
#pragma unroll
            for (int q = 0; q < 7; ++q)
                if (q == cls) ++cnt[1 + q];
            dmax = d > dmax ? d : dmax;
            unsigned long long walks = 0;
            for (int32_t p = b; p < e; ++p) {
                const int32_t w = c_adj[p];
                walks += (unsigned long long)(o_off[w + 1] - o_off[w]);
            }
            wmax = walks > wmax ? walks : wmax;
        }
    }
    const bool lead = (threadIdx.x & 63) == 0;
#pragma unroll
    for (int q = 0; q < 8; ++q) {
        unsigned long long x = cnt[q];
        for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o);
        if (lead && x) atomicAdd(&stats[q], x);
    }
    for (int o = 32; o > 0; o >>= 1) {
        const unsigned long long y = __shfl_xor(dmax, o), z = __shfl_xor(wmax, o);
        dmax = y > dmax ? y : dmax;
        wmax = z > wmax ? z : wmax;
    }
    if (lead && dmax) atomicMax(&stats[8], dmax);
    if (lead && wmax) atomicMax(&stats[9], wmax);
}

__global__ void rank_scatter_kernel(int32_t nc, int32_t nzero, const unsigned long long *sorted,
                                    int32_t *order, int32_t *rank) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nc; i += stride) {
        const int32_t v = (int32_t)(sorted[i] & 0xFFFFFFFFull);
        if (i < nzero) {
            rank[v] = -1;
        } else {
            order[i - nzero] = v;
            rank[v] = (int32_t)(i - nzero);
        }
    }
}

// Packed batch: graph g owns candidate ids [cbase[g], cbase[g+1]).  keys[v] = (deg << 32) |
// local id; gstats[g]: [0] degree-0 candidates, [1] max 2-hop walk count; stats[8] = max
// degree over the batch.
__global__ void batch_keys_kernel(int32_t nc, const int32_t *c_off, const int32_t *c_adj, const int32_t *o_off,
                                  const int32_t *graph_of, const int32_t *cbase, unsigned long long *keys,
                                  unsigned long long *gstats, unsigned long long *stats) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < nc; v += stride) {
        const int32_t g = graph_of[v];
        const int32_t b = c_off[v], e = c_off[v + 1];
        const uint32_t d = (uint32_t)(e - b);
        keys[v] = ((unsigned long long)d << 32) | (unsigned long long)(uint32_t)(v - cbase[g]);
        if (d == 0) {
            atomicAdd(&gstats[2 * g], 1ull);
        } else {
            atomicMax(&stats[8], (unsigned long long)d);
            unsigned long long walks = 0;
            for (int32_t p = b; p < e; ++p) {
                const int32_t w = c_adj[p];
                walks += (unsigned long long)(o_off[w + 1] - o_off[w]);
            }
            atomicMax(&gstats[2 * g + 1], walks);
        }
    }
}

// After the per-graph sort: order / rank of every candidate, one task per candidate of degree
// > 0 keyed so that a radix sort groups tasks by mask class, largest degree first, and the
// graph descriptors.
__global__ void batch_scatter_kernel(int32_t nc, const unsigned long long *sorted, const int32_t *graph_of,
                                     const int32_t *cbase, const unsigned long long *gstats, int32_t *order,
                                     int32_t *rank, unsigned int *task_key, unsigned long long *task,
                                     const int32_t *tbase) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < nc; i += stride) {
        const int32_t g = graph_of[i];  // sorted position i lies in graph g's segment
        const int32_t nzero = (int32_t)gstats[2 * g];
        const unsigned long long key = sorted[i];
        const int32_t v = cbase[g] + (int32_t)(key & 0xFFFFFFFFull);
        const uint32_t d = (uint32_t)(key >> 32);
        const int32_t li = (int32_t)(i - cbase[g]);
        if (li < nzero) {
            rank[v] = -1;
        } else {
            const int32_t r = li - nzero;
            order[cbase[g] + r] = v;
            rank[v] = r;
            uint32_t cls = 0;
            while (cls < 6 && d > (64u << cls)) ++cls;
            const uint32_t dk = d < 2047u ? d : 2047u;
            const int32_t t = tbase[g] + r;
            task_key[t] = (cls << 11) | (2047u - dk);
            task[t] = ((unsigned long long)(uint32_t)g << 32) | (unsigned long long)(uint32_t)r;
        }
    }
}

// Zero fill of rows runs of words 32-bit words, run r starting at base + r * pitch bytes (a
// plain fill kernel rather than a runtime memset, so that the clears of a call are ordinary
// kernel launches on its stream).
__global__ void zero_2d_kernel(char *base, size_t pitch, int64_t words, int64_t rows) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    const int64_t total = words * rows;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < total; t += stride) {
        const int64_t r = t / words, w = t - r * words;
        reinterpret_cast<uint32_t *>(base + (size_t)r * pitch)[w] = 0u;
    }
}

// Twins (candidates with equal neighbour rows), for the candidate pruning of section II-C:
// key[v] = a hash of v's degree and row (order-independent SplitMix64 sum), ~0 for degree-0
// candidates, so that a sort groups equal rows; val[v] = v.
__device__ __forceinline__ unsigned long long prep_mix(unsigned long long z) {
    z ^= z >> 30;
    z *= 0xBF58476D1CE4E5B9ull;
    z ^= z >> 27;
    z *= 0x94D049BB133111EBull;
    z ^= z >> 31;
    return z;
}

__global__ void row_key_kernel(int32_t nc, const int32_t *c_off, const int32_t *c_adj, unsigned long long *key,
                               unsigned int *val) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t v = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; v < nc; v += stride) {
        const int32_t b = c_off[v], e = c_off[v + 1];
        unsigned long long h = prep_mix(0x9E3779B97F4A7C15ull * (unsigned long long)(e - b + 1));
        for (int32_t p = b; p < e; ++p) h += prep_mix(0x9E3779B97F4A7C15ull * (unsigned long long)(c_adj[p] + 7));
        key[v] = e > b ? h : ~0ull;
        val[v] = (unsigned int)v;
    }
}

// After the sort by key: twin[v] = the lowest rank among the candidates whose row equals v's
// (v's own rank when none ranks lower); rows are compared in full within each run of equal
// keys, so a hash collision never makes twins.
__global__ void twin_kernel(int32_t nc, const unsigned long long *key, const unsigned int *val, const int32_t *c_off,
                            const int32_t *c_adj, const int32_t *rank, int32_t *twin) {
    const int64_t stride = (int64_t)gridDim.x * blockDim.x;
    for (int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; p < nc; p += stride) {
        const unsigned long long k = key[p];
        const int32_t v = (int32_t)val[p];
        if (k == ~0ull) {
            twin[v] = -1;
            continue;
        }
        int64_t s = p;
        while (s > 0 && key[s - 1] == k) --s;
        const int32_t vb = c_off[v], d = c_off[v + 1] - vb;
        int32_t best = rank[v];
        for (int64_t q = s; q < nc && key[q] == k; ++q) {
            const int32_t u = (int32_t)val[q];
            if (rank[u] >= best) continue;
            const int32_t ub = c_off[u];
            if (c_off[u + 1] - ub != d) continue;
            bool same = true;
            for (int32_t t = 0; t < d && same; ++t) same = c_adj[ub + t] == c_adj[vb + t];
            if (same) best = rank[u];
        }
        twin[v] = best;
    }
}

int grid_for(int64_t n, int block) {
    int64_t g = (n + block - 1) / block;
    if (g < 1) g = 1;
    if (g > 4096) g = 4096;
    return (int)g;
}

}  // namespace

hipError_t launch_validate(int32_t n_u, int32_t n_v, int32_t n_edges, const int32_t *u_off, const int32_t *u_adj,
                           const int32_t *v_off, const int32_t *v_adj, unsigned int *flags, hipStream_t s) {
    if (n_u == 0 || n_v == 0) return hipSuccess;
    const int64_t work = std::max<int64_t>(n_edges, (int64_t)std::max(n_u, n_v) + 1);
    hipLaunchKernelGGL(validate_kernel, dim3(grid_for(work, 256), 2), dim3(256), 0, s, n_u, n_v, n_edges, u_off,
                       u_adj, v_off, v_adj, flags);
    return hipGetLastError();
}

hipError_t launch_rank_keys(int32_t nc, const int32_t *c_off, const int32_t *c_adj, const int32_t *o_off,
                            unsigned long long *keys, unsigned long long *stats, hipStream_t s) {
    if (nc == 0) return hipSuccess;
    hipLaunchKernelGGL(rank_keys_kernel, dim3(grid_for(nc, 256)), dim3(256), 0, s, nc, c_off, c_adj, o_off, keys,
                       stats);
    return hipGetLastError();
}

hipError_t launch_rank_scatter(int32_t nc, int32_t nzero, const unsigned long long *sorted,
                               int32_t *order, int32_t *rank, hipStream_t s) {
    if (nc == 0) return hipSuccess;
    hipLaunchKernelGGL(rank_scatter_kernel, dim3(grid_for(nc, 256)), dim3(256), 0, s, nc, nzero, sorted,
                       order, rank);
    return hipGetLastError();
}

hipError_t launch_batch_keys(int32_t nc, const int32_t *c_off, const int32_t *c_adj, const int32_t *o_off,
                             const int32_t *graph_of, const int32_t *cbase, unsigned long long *keys,
                             unsigned long long *gstats, unsigned long long *stats, hipStream_t s) {
    if (nc == 0) return hipSuccess;
    hipLaunchKernelGGL(batch_keys_kernel, dim3(grid_for(nc, 256)), dim3(256), 0, s, nc, c_off, c_adj, o_off, graph_of,
                       cbase, keys, gstats, stats);
    return hipGetLastError();
}

hipError_t launch_batch_scatter(int32_t nc, const unsigned long long *sorted, const int32_t *graph_of,
                                const int32_t *cbase, const unsigned long long *gstats, int32_t *order, int32_t *rank,
                                unsigned int *task_key, unsigned long long *task, const int32_t *tbase,
                                hipStream_t s) {
    if (nc == 0) return hipSuccess;
    hipLaunchKernelGGL(batch_scatter_kernel, dim3(grid_for(nc, 256)), dim3(256), 0, s, nc, sorted, graph_of, cbase,
                       gstats, order, rank, task_key, task, tbase);
    return hipGetLastError();
}

hipError_t launch_row_keys(int32_t nc, const int32_t *c_off, const int32_t *c_adj, unsigned long long *key,
                           unsigned int *val, hipStream_t s) {
    if (nc == 0) return hipSuccess;
    hipLaunchKernelGGL(row_key_kernel, dim3(grid_for(nc, 256)), dim3(256), 0, s, nc, c_off, c_adj, key, val);
    return hipGetLastError();
}

hipError_t launch_twins(int32_t nc, const unsigned long long *key, const unsigned int *val, const int32_t *c_off,
                        const int32_t *c_adj, const int32_t *rank, int32_t *twin, hipStream_t s) {
    if (nc == 0) return hipSuccess;
    hipLaunchKernelGGL(twin_kernel, dim3(grid_for(nc, 256)), dim3(256), 0, s, nc, key, val, c_off, c_adj, rank, twin);
    return hipGetLastError();
}

hipError_t sort_pairs_u64_u32(void *temp, size_t *temp_bytes, const unsigned long long *kin, unsigned long long *kout,
                              const unsigned int *vin, unsigned int *vout, int32_t n, hipStream_t s) {
    return rocprim::radix_sort_pairs(temp, *temp_bytes, kin, kout, vin, vout, (unsigned int)n, 0, 64, s);
}

hipError_t launch_zero(void *p, size_t bytes, hipStream_t s) {
    return launch_zero_2d(p, 0, bytes, 1, s);
}

hipError_t launch_zero_2d(void *base, size_t pitch, size_t width_bytes, size_t rows, hipStream_t s) {
    const int64_t words = (int64_t)(width_bytes / 4);
    if (words == 0 || rows == 0) return hipSuccess;
    hipLaunchKernelGGL(zero_2d_kernel, dim3(grid_for(words * (int64_t)rows, 256)), dim3(256), 0, s,
                       static_cast<char *>(base), pitch, words, (int64_t)rows);
    return hipGetLastError();
}

hipError_t segmented_sort_u64(void *temp, size_t *temp_bytes, const unsigned long long *in, unsigned long long *out,
                              int32_t n, int32_t nseg, const int32_t *seg_begin, const int32_t *seg_end, int end_bit,
                              hipStream_t s) {
    return rocprim::segmented_radix_sort_keys(temp, *temp_bytes, in, out, (unsigned int)n, (unsigned int)nseg,
                                              seg_begin, seg_end, 0, end_bit, s);
}

hipError_t sort_pairs_u32_u64(void *temp, size_t *temp_bytes, const unsigned int *kin, unsigned int *kout,
                              const unsigned long long *vin, unsigned long long *vout, int32_t n, int end_bit,
                              hipStream_t s) {
    return rocprim::radix_sort_pairs(temp, *temp_bytes, kin, kout, vin, vout, (unsigned int)n, 0, end_bit, s);
}

hipError_t radix_sort_u64(void *temp, size_t *temp_bytes, const unsigned long long *in,
                          unsigned long long *out, int32_t n, int end_bit, hipStream_t s) {
    return rocprim::radix_sort_keys(temp, *temp_bytes, in, out, (unsigned int)n, 0, end_bit, s);
}

}  // namespace mbe
