// hyper.hip - preprocessing for the hyper-sparse region (above 99%
// sparsity, where the paper's design falls back towards the CPU, Sections I
// and IV-C, and its first future-work item, Section V).
//
// Doubly compressed rows: a row-split product over CSR spends a group on
// every row, empty or not; the DCSR order lists the rows holding an entry
// first (ascending), then the empty ones (ascending), so a product launches
// groups for the non-empty rows alone and a plain store writes the empty
// rows' zeros.  A stable partition by a flag scan: unique.
//
// COO row index: the row of every entry, so that an SDDMM can take entries
// in flat runs with no per-row structure at all.
#include "common.h"
#include "internal.h"

namespace spk {

__global__ void nonempty_flags_kernel(int64_t m, const int32_t *__restrict__ rp, int32_t *__restrict__ f) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < m) f[i] = rp[i + 1] > rp[i] ? 1 : 0;
    else if (i == m) f[m] = 0;
}

// f holds the exclusive scan of the flags (f[m] = number of non-empty rows).
__global__ void nonempty_scatter_kernel(int64_t m, const int32_t *__restrict__ rp, const int32_t *__restrict__ f,
                                        int32_t *__restrict__ order, int32_t *__restrict__ count) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= m) return;
    const int32_t nr = f[m];
    if (rp[i + 1] > rp[i]) order[f[i]] = static_cast<int32_t>(i);
    else order[nr + (i - f[i])] = static_cast<int32_t>(i);
    if (i == 0) *count = nr;
}

size_t nonempty_order_ws_bytes(int64_t m) { return align_up(sizeof(int32_t) * static_cast<size_t>(m + 1)) + scan_ws_bytes_i32(m + 1); }

hipError_t nonempty_order_launch(int64_t m, const int32_t *rp, int32_t *order, int32_t *count_dev, void *ws_,
                                 hipStream_t s) {
    char *ws = static_cast<char *>(ws_);
    int32_t *f = reinterpret_cast<int32_t *>(ws);
    void *scan_ws = ws + align_up(sizeof(int32_t) * static_cast<size_t>(m + 1));
    const unsigned nb = static_cast<unsigned>((m + 1 + kBlock - 1) / kBlock);
    hipLaunchKernelGGL(nonempty_flags_kernel, dim3(nb), dim3(kBlock), 0, s, m, rp, f);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if ((e = exclusive_scan_i32(f, m + 1, scan_ws, s)) != hipSuccess) return e;
    hipLaunchKernelGGL(nonempty_scatter_kernel, dim3(nb), dim3(kBlock), 0, s, m, rp, f, order, count_dev);
    return hipGetLastError();
}

// One wave per row (striding over the rows past the grid) writes the row's
// number over its range.
__global__ __launch_bounds__(kBlock) void row_index_kernel(int64_t m, const int32_t *__restrict__ rp,
                                                           int32_t *__restrict__ rowidx) {
    const int64_t step = static_cast<int64_t>(gridDim.x) * (kBlock / kWave);
    for (int64_t row = static_cast<int64_t>(blockIdx.x) * (kBlock / kWave) + threadIdx.x / kWave; row < m;
         row += step)
        for (int64_t p = rp[row] + (threadIdx.x & (kWave - 1)); p < rp[row + 1]; p += kWave)
            rowidx[p] = static_cast<int32_t>(row);
}

hipError_t row_index_launch(int64_t m, const int32_t *rp, int32_t *rowidx, hipStream_t s) {
    if (m == 0) return hipSuccess;
    hipLaunchKernelGGL(row_index_kernel, dim3(wave_rows_grid(m)), dim3(kBlock), 0, s, m, rp, rowidx);
    return hipGetLastError();
}

}  // namespace spk
