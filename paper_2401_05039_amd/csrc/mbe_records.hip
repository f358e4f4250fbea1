// Canonical order of enumerated bicliques (device side).
//
// The search writes records [|A|, |B|, A..., B...] in whatever order its waves finish.  The
// canonical output sorts each side ascending and the records by A lexicographically; A
// determines B (B = N(A)), so the order is total.

#include <rocprim/device/device_merge_sort.hpp>
#include <rocprim/device/device_scan.hpp>

#include "mbe_internal.h"

namespace mbe {

namespace {

__device__ void heap_sort(int32_t *a, int n) {
    // in-place heapsort, ascending
    auto sift = [&](int start, int end) {
        int root = start;
        while (2 * root + 1 < end) {
            int child = 2 * root + 1;
            if (child + 1 < end && a[child] < a[child + 1]) ++child;
            if (a[root] < a[child]) {
                const int32_t t = a[root];
                a[root] = a[child];
                a[child] = t;
                root = child;
            } else {
                return;
            }
        }
    };
    for (int s = n / 2 - 1; s >= 0; --s) sift(s, n);
    for (int e = n - 1; e > 0; --e) {
        const int32_t t = a[0];
        a[0] = a[e];
        a[e] = t;
        sift(0, e);
    }
}

__global__ void sort_sides_kernel(int32_t *rec, const unsigned long long *offs, unsigned long long n) {
    const unsigned long long stride = (unsigned long long)gridDim.x * blockDim.x;
    for (unsigned long long i = (unsigned long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        int32_t *r = rec + offs[i];
        const int na = r[0], nb = r[1];
        heap_sort(r + 2, na);
        heap_sort(r + 2 + na, nb);
    }
}

struct RecordLess {
    const int32_t *rec;
    __device__ bool operator()(const unsigned long long &x, const unsigned long long &y) const {
        const int32_t *a = rec + x;
        const int32_t *b = rec + y;
        const int na = a[0], nb = b[0];
        const int n = na < nb ? na : nb;
        for (int i = 0; i < n; ++i) {
            const int32_t p = a[2 + i], q = b[2 + i];
            if (p != q) return p < q;
        }
        return na < nb;
    }
};

__global__ void lengths_kernel(const int32_t *rec, const unsigned long long *offs, unsigned long long n,
                               unsigned long long *lens) {
    const unsigned long long stride = (unsigned long long)gridDim.x * blockDim.x;
    for (unsigned long long i = (unsigned long long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += stride) {
        const int32_t *r = rec + offs[i];
        lens[i] = 2ull + (unsigned long long)r[0] + (unsigned long long)r[1];
    }
}

// one wave per record: copy it to its place in the output
__global__ void gather_kernel(const int32_t *rec, const unsigned long long *offs, const unsigned long long *dst,
                              unsigned long long n, int32_t *out) {
    const int lane = (int)__lane_id();
    const unsigned long long wave = ((unsigned long long)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const unsigned long long nwaves = ((unsigned long long)gridDim.x * blockDim.x) >> 6;
    for (unsigned long long i = wave; i < n; i += nwaves) {
        const int32_t *r = rec + offs[i];
        const unsigned long long len = 2ull + (unsigned long long)r[0] + (unsigned long long)r[1];
        int32_t *o = out + dst[i];
        for (unsigned long long q = lane; q < len; q += 64) o[q] = r[q];
    }
}

int grid_for(unsigned long long n, int block) {
    unsigned long long g = (n + block - 1) / block;
    if (g < 1) g = 1;
    if (g > 8192) g = 8192;
    return (int)g;
}

}  // namespace

// rec: record arena; offs[n_rec]: record start offsets (reordered in place into canonical
// order); offs_tmp, lens: n_rec scratch each; out: destination (sum of lengths ints).  With
// temp == NULL only *temp_bytes is set.
hipError_t canonical_records(const int32_t *rec, unsigned long long *offs, unsigned long long n_rec,
                             unsigned long long *offs_tmp, unsigned long long *lens, int32_t *out,
                             void *temp, size_t *temp_bytes, hipStream_t s) {
    RecordLess less{rec};
    size_t t_sort = 0, t_scan = 0;
    hipError_t e = rocprim::merge_sort(nullptr, t_sort, offs, offs_tmp, (size_t)n_rec, less, s);
    if (e != hipSuccess) return e;
    e = rocprim::exclusive_scan(nullptr, t_scan, lens, offs, 0ull, (size_t)n_rec, rocprim::plus<unsigned long long>(), s);
    if (e != hipSuccess) return e;
    const size_t need = (t_sort > t_scan ? t_sort : t_scan) + 256;
    if (temp == nullptr) {
        *temp_bytes = need;
        return hipSuccess;
    }
    if (*temp_bytes < need) return hipErrorInvalidValue;
    if (n_rec == 0) return hipSuccess;
    hipLaunchKernelGGL(sort_sides_kernel, dim3(grid_for(n_rec, 256)), dim3(256), 0, s, const_cast<int32_t *>(rec),
                       offs, n_rec);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    e = rocprim::merge_sort(temp, t_sort, offs, offs_tmp, (size_t)n_rec, less, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(lengths_kernel, dim3(grid_for(n_rec, 256)), dim3(256), 0, s, rec, offs_tmp, n_rec, lens);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    // offs now receives the destination offsets of the sorted records
    e = rocprim::exclusive_scan(temp, t_scan, lens, offs, 0ull, (size_t)n_rec, rocprim::plus<unsigned long long>(), s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(gather_kernel, dim3(grid_for(n_rec * 64, 256)), dim3(256), 0, s, rec, offs_tmp, offs,
                       n_rec, out);
    return hipGetLastError();
}

}  // namespace mbe
