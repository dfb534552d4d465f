// slab16.hip - the column-slab form with 16-bit slab-relative column indices,
// built on the GPU once per pattern.
//
// The paper's host sends each nonzero's column as a 16-bit offset inside the
// column range a worker row owns, and groups nonzeros by that owner
// (Section III-A, Optimization 1).  Here the owners are column slabs of W
// columns (W <= 65536), one launch of a product per slab, and the grouping is
// slab-major: all runs of slab 0 (row by row), then slab 1, and so on.  A run
// is the part of a row whose columns fall in the slab, a contiguous piece of
// the row in A's storage (rows are sorted), so the form needs no value copy:
// entry k of run (s, i) has A's value at apos[s m + i] + k.
//   seg[S m + 1]  slab-major start of every run (seg[S m] = nnz)
//   apos[S m]     A position of every run's first entry
//   col16[nnz]    column - s W, slab-major
// All integer work, in a fixed order: the result is unique.
#include "common.h"
#include "internal.h"

namespace spk {

// First position in [lo, hi) whose column is >= key (hi when none).
__device__ __forceinline__ int64_t first_at_least(const int32_t *__restrict__ ci, int64_t lo, int64_t hi,
                                                  int64_t key) {
    while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if (static_cast<int64_t>(ci[mid]) < key) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

// Run (s, i): its A range by two binary searches; seg receives the length.
__global__ void slab16_runs_kernel(int64_t m, const int32_t *__restrict__ rp, const int32_t *__restrict__ ci,
                                   int64_t W, int64_t S, int32_t *__restrict__ seg, int32_t *__restrict__ apos) {
    const int64_t idx = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (idx >= S * m) return;
    const int64_t s = idx / m, i = idx - s * m;
    const int64_t lo = rp[i], hi = rp[i + 1];
    const int64_t a = s == 0 ? lo : first_at_least(ci, lo, hi, s * W);
    const int64_t b = s == S - 1 ? hi : first_at_least(ci, a, hi, (s + 1) * W);
    apos[idx] = static_cast<int32_t>(a);
    seg[idx] = static_cast<int32_t>(b - a);
}

__global__ void slab16_zero_kernel(int32_t *__restrict__ p) { *p = 0; }

// One wave per row: every entry finds its run by its slab and writes its
// offset there.
__global__ __launch_bounds__(kBlock) void slab16_fill_kernel(int64_t m, const int32_t *__restrict__ rp,
                                                             const int32_t *__restrict__ ci, int64_t W,
                                                             const int32_t *__restrict__ seg,
                                                             const int32_t *__restrict__ apos,
                                                             uint16_t *__restrict__ col16) {
    const int64_t row = static_cast<int64_t>(blockIdx.x) * (kBlock / kWave) + threadIdx.x / kWave;
    if (row >= m) return;
    for (int64_t p = rp[row] + (threadIdx.x & (kWave - 1)); p < rp[row + 1]; p += kWave) {
        const int64_t c = ci[p];
        const int64_t s = c / W;
        const int64_t run = s * m + row;
        col16[seg[run] + (p - apos[run])] = static_cast<uint16_t>(c - s * W);
    }
}

size_t slab16_ws_bytes(int64_t m, int64_t S) { return scan_ws_bytes_i32(S * m + 1); }

hipError_t slab16_build_launch(int64_t m, int64_t nnz, const int32_t *rp, const int32_t *ci, int64_t W, int64_t S,
                               int32_t *seg, int32_t *apos, uint16_t *col16, void *ws, hipStream_t s) {
    const int64_t runs = S * m;
    hipLaunchKernelGGL(slab16_zero_kernel, dim3(1), dim3(1), 0, s, seg + runs);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (runs > 0) {
        hipLaunchKernelGGL(slab16_runs_kernel, dim3(static_cast<unsigned>((runs + kBlock - 1) / kBlock)), dim3(kBlock), 0,
                           s, m, rp, ci, W, S, seg, apos);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    if ((e = exclusive_scan_i32(seg, runs + 1, ws, s)) != hipSuccess) return e;
    if (nnz == 0 || m == 0) return hipSuccess;
    constexpr int rows_per_block = kBlock / kWave;
    hipLaunchKernelGGL(slab16_fill_kernel, dim3(static_cast<unsigned>((m + rows_per_block - 1) / rows_per_block)),
                       dim3(kBlock), 0, s, m, rp, ci, W, seg, apos, col16);
    return hipGetLastError();
}

}  // namespace spk
