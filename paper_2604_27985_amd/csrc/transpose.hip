// transpose.hip - stable CSR transpose and CSR validation for gfx950.
//
// The transpose of A's pattern is a stable sort of A's entries by column:
// entries are visited in storage order (row-major), so sorting the pairs
// (col, position) stably by col lists, for each column j, the rows holding j
// in increasing order.  The sort is a least-significant-digit radix sort on
// 8-bit digits, one pass per digit of the largest column index:
//
//   1. per 2048-entry tile, count each digit (LDS integer atomics);
//   2. exclusive scan of the counts laid out digit-major, giving every
//      (digit, tile) its output offset;
//   3. per tile, rank every entry among the earlier entries of the same
//      digit (wavefront ballots give the rank inside a wave, LDS counters
//      across waves and rounds) and scatter it to offset + rank.
//
// Ranks follow storage order, so each pass is stable and the result is the
// unique stable order.  Row pointers of A^T come from a column histogram and
// the same scan; column indices of A^T are the rows of the sorted positions.
#include "common.h"
#include "internal.h"

namespace spk {

constexpr int kRadixBits = 8;
constexpr int kRadix = 1 << kRadixBits;
constexpr int kItems = 8;                 // rounds per tile
constexpr int kTile = kBlock * kItems;    // 2048 entries per tile
constexpr int kScanTile = kBlock * 8;     // elements per scan block

// ---------------------------------------------------------------- scan
// In-place exclusive scan of int32 data in tiles of kScanTile; each block
// writes its tile total to sums[blockIdx.x].
__global__ __launch_bounds__(kBlock) void scan_tiles_kernel(int32_t *__restrict__ data, int64_t count,
                                                            int32_t *__restrict__ sums) {
    __shared__ int32_t warp_tot[kBlock / kWave];
    const int64_t base = static_cast<int64_t>(blockIdx.x) * kScanTile + threadIdx.x * 8;
    int32_t v[8];
    int32_t run = 0;
#pragma unroll
    for (int i = 0; i < 8; ++i) {
        const int64_t idx = base + i;
        v[i] = idx < count ? data[idx] : 0;
        const int32_t t = v[i];
        v[i] = run;  // exclusive within the thread
        run += t;
    }
    // exclusive scan of per-thread totals across the block
    const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
    int32_t incl = run;
#pragma unroll
    for (int s = 1; s < kWave; s <<= 1) {
        const int32_t o = __shfl_up(incl, s, kWave);
        if (lane >= s) incl += o;
    }
    if (lane == kWave - 1) warp_tot[w] = incl;
    __syncthreads();
    int32_t wbase = 0;
    for (int i = 0; i < w; ++i) wbase += warp_tot[i];
    const int32_t excl = wbase + incl - run;
#pragma unroll
    for (int i = 0; i < 8; ++i) {
        const int64_t idx = base + i;
        if (idx < count) data[idx] = v[i] + excl;
    }
    if (threadIdx.x == kBlock - 1) sums[blockIdx.x] = excl + run;
}

__global__ __launch_bounds__(kBlock) void scan_add_kernel(int32_t *__restrict__ data, int64_t count,
                                                          const int32_t *__restrict__ offs) {
    const int64_t base = static_cast<int64_t>(blockIdx.x) * kScanTile;
    const int32_t o = offs[blockIdx.x];
    for (int i = threadIdx.x; i < kScanTile; i += kBlock) {
        const int64_t idx = base + i;
        if (idx < count) data[idx] += o;
    }
}

static size_t scan_ws_bytes(int64_t count) {
    size_t total = 0;
    while (count > 1) {
        const int64_t nb = (count + kScanTile - 1) / kScanTile;
        total += align_up(sizeof(int32_t) * static_cast<size_t>(nb));
        count = nb;
    }
    return total + kAlign;
}

// Exclusive scan of `count` int32 values in place; ws holds scan_ws_bytes(count).
static hipError_t exclusive_scan(int32_t *data, int64_t count, char *ws, hipStream_t s) {
    if (count <= 0) return hipSuccess;
    const int64_t nb = (count + kScanTile - 1) / kScanTile;
    int32_t *sums = reinterpret_cast<int32_t *>(ws);
    hipLaunchKernelGGL(scan_tiles_kernel, dim3(static_cast<unsigned>(nb)), dim3(kBlock), 0, s, data, count, sums);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || nb == 1) return e;
    e = exclusive_scan(sums, nb, ws + align_up(sizeof(int32_t) * static_cast<size_t>(nb)), s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(scan_add_kernel, dim3(static_cast<unsigned>(nb)), dim3(kBlock), 0, s, data, count, sums);
    return hipGetLastError();
}

size_t scan_ws_bytes_i32(int64_t count) { return scan_ws_bytes(count); }

hipError_t exclusive_scan_i32(int32_t *data, int64_t count, void *ws, hipStream_t s) {
    return exclusive_scan(data, count, static_cast<char *>(ws), s);
}

// ---------------------------------------------------------------- histogram
__global__ void column_count_kernel(int64_t nnz, const int32_t *__restrict__ ci, int32_t *__restrict__ cnt) {
    const int64_t p = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (p < nnz) atomicAdd(&cnt[ci[p]], 1);
}

__global__ void fill_i32_kernel(int32_t *__restrict__ a, int64_t count, int32_t v) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i < count) a[i] = v;
}

// rowid[p] = row of entry p: one wave per row (striding over the rows past
// the grid) writes its range.
__global__ __launch_bounds__(kBlock) void row_ids_kernel(int64_t m, const int32_t *__restrict__ rp,
                                                         int32_t *__restrict__ rowid) {
    const int64_t step = static_cast<int64_t>(gridDim.x) * (kBlock / kWave);
    for (int64_t row = static_cast<int64_t>(blockIdx.x) * (kBlock / kWave) + threadIdx.x / kWave; row < m;
         row += step)
        for (int64_t p = rp[row] + (threadIdx.x & (kWave - 1)); p < rp[row + 1]; p += kWave)
            rowid[p] = static_cast<int32_t>(row);
}

// ---------------------------------------------------------------- radix sort
// Key and value of entry t: pass 0 reads the column indices and uses the
// position itself as the value.
__device__ __forceinline__ void load_pair(const int32_t *kin, const int32_t *vin, int64_t t, int32_t &k, int32_t &v) {
    k = kin[t];
    v = vin ? vin[t] : static_cast<int32_t>(t);
}

__global__ __launch_bounds__(kBlock) void radix_count_kernel(int64_t count, const int32_t *__restrict__ kin, int shift,
                                                             int64_t ntiles, int32_t *__restrict__ hist) {
    __shared__ int32_t c[kRadix];
    c[threadIdx.x] = 0;
    __syncthreads();
    const int64_t base = static_cast<int64_t>(blockIdx.x) * kTile;
#pragma unroll
    for (int r = 0; r < kItems; ++r) {
        const int64_t t = base + r * kBlock + threadIdx.x;
        if (t < count) atomicAdd(&c[(kin[t] >> shift) & (kRadix - 1)], 1);
    }
    __syncthreads();
    hist[static_cast<int64_t>(threadIdx.x) * ntiles + blockIdx.x] = c[threadIdx.x];
}

__global__ __launch_bounds__(kBlock) void radix_scatter_kernel(int64_t count, const int32_t *__restrict__ kin,
                                                               const int32_t *__restrict__ vin, int shift, int64_t ntiles,
                                                               const int32_t *__restrict__ offs,
                                                               int32_t *__restrict__ kout, int32_t *__restrict__ vout) {
    __shared__ int32_t running[kRadix];                 // entries of each digit placed so far
    __shared__ int32_t wcount[kBlock / kWave][kRadix];  // this round, per wave
    const int lane = threadIdx.x & (kWave - 1), w = threadIdx.x / kWave;
    running[threadIdx.x] = offs[static_cast<int64_t>(threadIdx.x) * ntiles + blockIdx.x];
    const int64_t base = static_cast<int64_t>(blockIdx.x) * kTile;
    const uint64_t below = (lane == 0) ? 0ull : (~0ull >> (kWave - lane));
    for (int r = 0; r < kItems; ++r) {
#pragma unroll
        for (int q = 0; q < kBlock / kWave; ++q) wcount[q][threadIdx.x] = 0;
        __syncthreads();
        const int64_t t = base + r * kBlock + threadIdx.x;
        const bool valid = t < count;
        int32_t k = 0, v = 0;
        if (valid) load_pair(kin, vin, t, k, v);
        const int d = valid ? ((k >> shift) & (kRadix - 1)) : 0;
        // lanes of this wave holding the same digit
        uint64_t same = __ballot(valid);
#pragma unroll
        for (int b = 0; b < kRadixBits; ++b) {
            const uint64_t ones = __ballot(valid && ((d >> b) & 1));
            same &= ((d >> b) & 1) ? ones : ~ones;
        }
        const int rank_in_wave = __popcll(same & below);
        if (valid && rank_in_wave == 0) wcount[w][d] = __popcll(same);
        __syncthreads();
        if (valid) {
            int32_t pos = running[d] + rank_in_wave;
            for (int q = 0; q < w; ++q) pos += wcount[q][d];
            kout[pos] = k;
            vout[pos] = v;
        }
        __syncthreads();
        int32_t add = 0;
#pragma unroll
        for (int q = 0; q < kBlock / kWave; ++q) add += wcount[q][threadIdx.x];
        running[threadIdx.x] += add;
        __syncthreads();
    }
}

__global__ void gather_rows_kernel(int64_t nnz, const int32_t *__restrict__ perm, const int32_t *__restrict__ rowid,
                                   int32_t *__restrict__ tci) {
    const int64_t q = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (q < nnz) tci[q] = rowid[perm[q]];
}

static int radix_passes(int64_t n) {
    int bits = 0;
    while (bits < 31 && (static_cast<int64_t>(1) << bits) < n) ++bits;
    return bits == 0 ? 1 : (bits + kRadixBits - 1) / kRadixBits;
}

struct TransposeLayout {
    size_t k0, v0, k1, v1, hist, scan, total;
};

static TransposeLayout transpose_layout(int64_t n, int64_t nnz) {
    TransposeLayout L;
    const int64_t ntiles = (nnz + kTile - 1) / kTile;
    const size_t buf = align_up(sizeof(int32_t) * static_cast<size_t>(nnz > 0 ? nnz : 1));
    const int64_t hist_n = static_cast<int64_t>(kRadix) * (ntiles > 0 ? ntiles : 1);
    const int64_t scan_n = hist_n > n + 1 ? hist_n : n + 1;
    L.k0 = 0;
    L.v0 = L.k0 + buf;
    L.k1 = L.v0 + buf;
    L.v1 = L.k1 + buf;
    L.hist = L.v1 + buf;
    L.scan = L.hist + align_up(sizeof(int32_t) * static_cast<size_t>(hist_n));
    L.total = L.scan + scan_ws_bytes(scan_n);
    return L;
}

size_t transpose_ws_bytes(int64_t m, int64_t n, int64_t nnz) {
    (void)m;
    return transpose_layout(n, nnz).total;
}

static unsigned blocks_for(int64_t count, int per) { return static_cast<unsigned>((count + per - 1) / per); }

hipError_t transpose_launch(int64_t m, int64_t n, int64_t nnz, const int32_t *rp, const int32_t *ci, int32_t *trp,
                            int32_t *tci, int32_t *perm, void *ws_, hipStream_t s) {
    char *ws = static_cast<char *>(ws_);
    const TransposeLayout L = transpose_layout(n, nnz);
    hipError_t e;
    // Row pointers of A^T: column counts, exclusive scan (entry n ends as nnz).
    hipLaunchKernelGGL(fill_i32_kernel, dim3(blocks_for(n + 1, kBlock)), dim3(kBlock), 0, s, trp, n + 1, 0);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if (nnz == 0) return exclusive_scan(trp, n + 1, ws + L.scan, s);
    hipLaunchKernelGGL(column_count_kernel, dim3(blocks_for(nnz, kBlock)), dim3(kBlock), 0, s, nnz, ci, trp);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    if ((e = exclusive_scan(trp, n + 1, ws + L.scan, s)) != hipSuccess) return e;

    // Stable sort of (column, position) by column.
    const int64_t ntiles = (nnz + kTile - 1) / kTile;
    int32_t *hist = reinterpret_cast<int32_t *>(ws + L.hist);
    int32_t *kb[2] = {reinterpret_cast<int32_t *>(ws + L.k0), reinterpret_cast<int32_t *>(ws + L.k1)};
    int32_t *vb[2] = {reinterpret_cast<int32_t *>(ws + L.v0), reinterpret_cast<int32_t *>(ws + L.v1)};
    const int passes = radix_passes(n);
    const int32_t *kin = ci;
    const int32_t *vin = nullptr;
    for (int ps = 0; ps < passes; ++ps) {
        const int shift = ps * kRadixBits;
        const bool last = ps == passes - 1;
        int32_t *kout = kb[ps & 1];
        int32_t *vout = last ? perm : vb[ps & 1];
        hipLaunchKernelGGL(radix_count_kernel, dim3(static_cast<unsigned>(ntiles)), dim3(kBlock), 0, s, nnz, kin, shift,
                           ntiles, hist);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        if ((e = exclusive_scan(hist, kRadix * ntiles, ws + L.scan, s)) != hipSuccess) return e;
        hipLaunchKernelGGL(radix_scatter_kernel, dim3(static_cast<unsigned>(ntiles)), dim3(kBlock), 0, s, nnz, kin, vin,
                           shift, ntiles, hist, kout, vout);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        kin = kout;
        vin = vout;
    }
    // Columns of A^T: the row of each sorted position.
    int32_t *rowid = kb[passes & 1];  // the key buffer the last pass did not write
    hipLaunchKernelGGL(row_ids_kernel, dim3(wave_rows_grid(m)), dim3(kBlock), 0, s, m, rp, rowid);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(gather_rows_kernel, dim3(blocks_for(nnz, kBlock)), dim3(kBlock), 0, s, nnz, perm, rowid, tci);
    return hipGetLastError();
}

// ---------------------------------------------------------------- validation
// Bits of the result flag.
// Rules of canonical CSR, one bit each (the same numbering as spk.h).
enum { kBadStart = 1, kBadEnd = 2, kBadOrder = 4, kBadCol = 8, kBadSort = 16, kBadDup = 32 };

// One wave per row, striding over the rows past the grid: the row's range is
// checked first; only a range inside [0, nnz] is read, so a broken row_ptr
// never sends a load out of bounds.
__global__ __launch_bounds__(kBlock) void validate_kernel(int64_t m, int64_t n, int64_t nnz, const int32_t *__restrict__ rp,
                                                          const int32_t *__restrict__ ci, int32_t *__restrict__ flag) {
    const int lane = threadIdx.x & (kWave - 1);
    const int64_t step = static_cast<int64_t>(gridDim.x) * (kBlock / kWave);
    int bad = 0;
    for (int64_t row = static_cast<int64_t>(blockIdx.x) * (kBlock / kWave) + threadIdx.x / kWave; row < m;
         row += step) {
        if (row == 0 && lane == 0 && rp[0] != 0) bad |= kBadStart;
        if (row == m - 1 && lane == 0 && rp[m] != nnz) bad |= kBadEnd;
        const int64_t a = rp[row], b = rp[row + 1];
        if (b < a || a < 0 || b > nnz) {
            if (lane == 0) bad |= kBadOrder;
            continue;
        }
        for (int64_t p = a + lane; p < b; p += kWave) {
            const int32_t c = ci[p];
            if (c < 0 || c >= n) bad |= kBadCol;
            if (p + 1 < b) {
                const int32_t d = ci[p + 1];
                if (d < c) bad |= kBadSort;
                if (d == c) bad |= kBadDup;
            }
        }
    }
    if (bad) atomicOr(flag, bad);
}

hipError_t validate_launch(int64_t m, int64_t n, int64_t nnz, const int32_t *rp, const int32_t *ci, int32_t *flag,
                           hipStream_t s) {
    hipLaunchKernelGGL(fill_i32_kernel, dim3(1), dim3(kBlock), 0, s, flag, 1, 0);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || m == 0) return e;  // no rows: the caller checks nnz
    hipLaunchKernelGGL(validate_kernel, dim3(wave_rows_grid(m)), dim3(kBlock), 0, s, m, n, nnz, rp, ci, flag);
    return hipGetLastError();
}

}  // namespace spk
