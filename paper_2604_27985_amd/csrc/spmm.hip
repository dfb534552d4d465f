// spmm.hip - SpMM C = A B (Section II-A, Eq. (1)) for gfx950.
//
// The dense operand stays in HBM and the sparse matrix is streamed: each
// stored entry (col, val) is read once, coalesced and non-temporally (so the
// stream does not evict cached rows of B), and the matching row of B is
// gathered.  This keeps the paper's principle of streaming A past a
// stationary dense operand (Section III-A), mapped onto wavefronts instead of
// a PE grid:
//
//   - A group of LANES lanes (4..64, a divisor of the 64-lane wavefront)
//     owns one output row and one slice of LANES*VW columns of C; each lane
//     keeps VW accumulators in registers.
//   - The group reads LANES entries of its row at a time (one per lane), then
//     shares them with ds_bpermute and gathers the B row slices with one
//     8/16-byte load per lane.  Up to eight gathers are issued before their
//     FMAs.  Gathers are unconditional: entries past the end of a row read row
//     0 of B with value 0, so no exec-mask branches sit in the loop.
//   - ROWS: group g takes row g.  MERGE: group g takes an equal share of the
//     (row ends + entries) sequence, so a row of a million entries spreads over
//     thousands of groups; a group's partial sum of a row continuing past its
//     share is written as a carry and a fix-up kernel adds each row's carries
//     in group order.  SLAB: columns are cut into slabs of W columns and one
//     launch per slab adds A[:, slab] B[slab, :] into C, so the slab of B that
//     all waves gather from stays in each XCD's L2 (the paper's column-range
//     split of the dense operand across worker rows, Section III-A).
//   No float atomics anywhere: results are bitwise reproducible run to run.
//
// The backward's A^T G runs through the same kernels on the transpose's CSR,
// with each value read through perm (vals[perm[q]]).
#include "common.h"
#include "internal.h"

namespace spk {

// Pointer to element `off` of a dense operand.  OFF32: every element offset
// of the operand fits in 32 bits, so the offset is formed in 32-bit integer
// arithmetic and added to the (wave-uniform) base.
template <bool OFF32, typename T>
__device__ __forceinline__ const T *elem(const T *base, int32_t row, int64_t ld, int32_t col) {
    if constexpr (OFF32)
        return base + (static_cast<uint32_t>(row) * static_cast<uint32_t>(ld) + static_cast<uint32_t>(col));
    else
        return base + (static_cast<int64_t>(row) * ld + col);
}

// acc += sum_{p in [a, b)} val(p) * B[col(p), koff .. koff+VW).
// a, b are uniform over the LANES-lane group; koff is clamped to a valid
// column for lanes beyond K (their results are never stored).
template <typename TB, typename TV, int VW, int LANES, bool OFF32>
__device__ __forceinline__ void accumulate_entries(int64_t a, int64_t b, const int32_t *__restrict__ ci,
                                                   const TV *__restrict__ vals,
                                                   const int32_t *__restrict__ vperm,
                                                   const TB *__restrict__ B, int64_t ldb, int koff, int gbase,
                                                   int lig, typename acc_of<TB>::type *acc) {
    using A = typename acc_of<TB>::type;
    constexpr int U = LANES < 8 ? LANES : 8;
    for (int64_t p0 = a; p0 < b; p0 += LANES) {
        const int64_t p = p0 + lig;
        int c = 0;
        A v = A(0);
        if (p < b) {
            c = __builtin_nontemporal_load(ci + p);
            if (vals) {
                const int64_t pv = vperm ? static_cast<int64_t>(__builtin_nontemporal_load(vperm + p)) : p;
                v = static_cast<A>(vals[pv]);
            } else {
                v = A(1);
            }
        }
        const int cnt = static_cast<int>(b - p0 < LANES ? b - p0 : LANES);
        for (int t = 0; t < cnt; t += U) {
            int cc[U];
            A vv[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                cc[u] = lane_read(c, gbase + t + u);
                vv[u] = lane_read(v, gbase + t + u);
            }
            A bv[U][VW];
#pragma unroll
            for (int u = 0; u < U; ++u) vec_load<TB, VW>::run(elem<OFF32>(B, cc[u], ldb, koff), bv[u]);
#pragma unroll
            for (int u = 0; u < U; ++u)
#pragma unroll
                for (int e = 0; e < VW; ++e) acc[e] = fma(vv[u], bv[u][e], acc[e]);
        }
    }
}

template <typename A, int VW>
__device__ __forceinline__ void zero(A *acc) {
#pragma unroll
    for (int e = 0; e < VW; ++e) acc[e] = A(0);
}

template <typename TB, typename TV, int VW, int LANES, bool OFF32>
__global__ __launch_bounds__(kBlock) void spmm_rows_kernel(int64_t m, int K, const int32_t *__restrict__ rp,
                                                           const int32_t *__restrict__ ci,
                                                           const TV *__restrict__ vals,
                                                           const int32_t *__restrict__ vperm,
                                                           const TB *__restrict__ B, int64_t ldb,
                                                           typename acc_of<TB>::type *__restrict__ C,
                                                           int64_t ldc) {
    using A = typename acc_of<TB>::type;
    constexpr int GPB = kBlock / LANES;
    const int lig = threadIdx.x & (LANES - 1);
    const int gbase = (threadIdx.x & (kWave - 1)) & ~(LANES - 1);
    const int64_t blk = xcd_block(blockIdx.x, gridDim.x);
    const int64_t row = blk * GPB + threadIdx.x / LANES;
    if (row >= m) return;  // the whole group leaves together
    const int k0 = blockIdx.y * (LANES * VW) + lig * VW;
    const bool kvalid = k0 < K;
    A acc[VW];
    zero<A, VW>(acc);
    accumulate_entries<TB, TV, VW, LANES, OFF32>(rp[row], rp[row + 1], ci, vals, vperm, B, ldb, kvalid ? k0 : 0,
                                                 gbase, lig, acc);
    if (kvalid) vec_store<A, VW>::run(C + row * ldc + k0, acc);
}

// Slab s of a SLAB SpMM: entries of row i with columns in slab s are
// [bnd(s, i), bnd(s+1, i)), where bnd(0, i) = row_ptr[i], bnd(S, i) =
// row_ptr[i+1] and interior boundaries come from slab_bounds_kernel.
// Slab 0 writes C; later slabs add to it.
template <typename TB, typename TV, int VW, int LANES, bool OFF32>
__global__ __launch_bounds__(kBlock) void spmm_slab_kernel(int64_t m, int K, const int32_t *__restrict__ rp,
                                                           const int32_t *__restrict__ bnd, int nslabs, int s,
                                                           const int32_t *__restrict__ ci,
                                                           const TV *__restrict__ vals,
                                                           const int32_t *__restrict__ vperm,
                                                           const TB *__restrict__ B, int64_t ldb,
                                                           typename acc_of<TB>::type *__restrict__ C,
                                                           int64_t ldc) {
    using A = typename acc_of<TB>::type;
    constexpr int GPB = kBlock / LANES;
    const int lig = threadIdx.x & (LANES - 1);
    const int gbase = (threadIdx.x & (kWave - 1)) & ~(LANES - 1);
    const int64_t blk = xcd_block(blockIdx.x, gridDim.x);
    const int64_t row = blk * GPB + threadIdx.x / LANES;
    if (row >= m) return;
    const int k0 = blockIdx.y * (LANES * VW) + lig * VW;
    const bool kvalid = k0 < K;
    const int64_t a = s == 0 ? rp[row] : bnd[(s - 1) * m + row];
    const int64_t b = s == nslabs - 1 ? rp[row + 1] : bnd[s * m + row];
    A acc[VW];
    zero<A, VW>(acc);
    accumulate_entries<TB, TV, VW, LANES, OFF32>(a, b, ci, vals, vperm, B, ldb, kvalid ? k0 : 0, gbase, lig, acc);
    if (kvalid) {
        A *out = C + row * ldc + k0;
        if (s > 0) {
            A prev[VW];
#pragma unroll
            for (int e = 0; e < VW; ++e) prev[e] = out[e];
#pragma unroll
            for (int e = 0; e < VW; ++e) acc[e] = prev[e] + acc[e];
        }
        vec_store<A, VW>::run(out, acc);
    }
}

// TILE: a workgroup owns GPB*RPG consecutive rows (RPG per group) and walks
// the columns in slabs of W; each slab of B is staged once in LDS and every
// group gathers its rows' entries of that slab from LDS.  A staged row of B
// serves (rows per workgroup) x density entries on average, which cuts the
// L2 gather traffic by that factor for dense-ish matrices.  Entries within a
// row are sorted, so the entries of a row inside a slab are a prefix of the
// ones not yet consumed: a chunk of LANES entries is read, the count below
// the slab end found with a ballot, and the cursor advanced by it.
template <typename TB, typename TV, int VW, int LANES, int RPG>
__global__ __launch_bounds__(kBlock) void spmm_tile_kernel(int64_t m, int64_t n, int K, const int32_t *__restrict__ rp,
                                                           const int32_t *__restrict__ ci,
                                                           const TV *__restrict__ vals,
                                                           const int32_t *__restrict__ vperm,
                                                           const TB *__restrict__ B, int64_t ldb,
                                                           typename acc_of<TB>::type *__restrict__ C, int64_t ldc,
                                                           int W) {
    using A = typename acc_of<TB>::type;
    extern __shared__ __align__(16) unsigned char smem[];
    TB *Bs = reinterpret_cast<TB *>(smem);  // [W][K]
    constexpr int GPB = kBlock / LANES;
    constexpr int U = LANES < 8 ? LANES : 8;
    const int lane = threadIdx.x & (kWave - 1);
    const int lig = threadIdx.x & (LANES - 1);
    const int gbase = lane & ~(LANES - 1);
    const uint64_t gmask = LANES == 64 ? ~0ull : (((1ull << LANES) - 1) << gbase);
    const int64_t blk = xcd_block(blockIdx.x, gridDim.x);
    const int64_t row0 = (blk * GPB + threadIdx.x / LANES) * RPG;
    const int k0 = lig * VW;
    const bool kvalid = k0 < K;
    const int koff = kvalid ? k0 : 0;
    int64_t cur[RPG], end[RPG];
#pragma unroll
    for (int r = 0; r < RPG; ++r) {
        const int64_t row = row0 + r;
        cur[r] = row < m ? rp[row] : 0;
        end[r] = row < m ? rp[row + 1] : 0;
    }
    A acc[RPG][VW];
#pragma unroll
    for (int r = 0; r < RPG; ++r) zero<A, VW>(acc[r]);
    constexpr int SV = 16 / sizeof(TB);  // elements per 16-byte staging load
    for (int64_t c0 = 0; c0 < n; c0 += W) {
        const int w = static_cast<int>(n - c0 < W ? n - c0 : W);
        __syncthreads();  // the previous slab is consumed
        const int per_row = K / SV;  // K is a multiple of SV for this variant
        for (int idx = threadIdx.x; idx < w * per_row; idx += kBlock) {
            const int rr = idx / per_row, cc = (idx % per_row) * SV;
            *reinterpret_cast<uint4 *>(Bs + rr * K + cc) =
                *reinterpret_cast<const uint4 *>(B + (c0 + rr) * ldb + cc);
        }
        __syncthreads();
        const int32_t c1 = static_cast<int32_t>(c0 + w);
#pragma unroll
        for (int r = 0; r < RPG; ++r) {
            while (cur[r] < end[r]) {  // group-uniform
                const int64_t p = cur[r] + lig;
                int c = 0x7FFFFFFF;
                A v = A(0);
                if (p < end[r]) {
                    c = __builtin_nontemporal_load(ci + p);
                    if (vals) {
                        const int64_t pv = vperm ? static_cast<int64_t>(__builtin_nontemporal_load(vperm + p)) : p;
                        v = static_cast<A>(vals[pv]);
                    } else {
                        v = A(1);
                    }
                }
                const bool in = c < c1;
                const int cnt = __popcll(__ballot(in) & gmask);
                const int crel = in ? c - static_cast<int>(c0) : 0;
                for (int t = 0; t < cnt; t += U) {
                    int cc[U];
                    A vv[U];
#pragma unroll
                    for (int u = 0; u < U; ++u) {
                        cc[u] = lane_read(crel, gbase + t + u);
                        vv[u] = lane_read(in ? v : A(0), gbase + t + u);
                    }
                    A bv[U][VW];
#pragma unroll
                    for (int u = 0; u < U; ++u) vec_load<TB, VW>::run(Bs + cc[u] * K + koff, bv[u]);
#pragma unroll
                    for (int u = 0; u < U; ++u)
#pragma unroll
                        for (int e = 0; e < VW; ++e) acc[r][e] = fma(vv[u], bv[u][e], acc[r][e]);
                }
                cur[r] += cnt;
                if (cnt < LANES) break;  // the rest of the row lies beyond this slab
            }
        }
    }
    if (!kvalid) return;
#pragma unroll
    for (int r = 0; r < RPG; ++r) {
        const int64_t row = row0 + r;
        if (row < m) vec_store<A, VW>::run(C + row * ldc + k0, acc[r]);
    }
}

// Interior slab boundaries: bnd[(s-1)*m + i] = first entry of row i whose
// column is >= s*W, for s = 1 .. nslabs-1 (binary search in the sorted row).
__global__ void slab_bounds_kernel(int64_t m, const int32_t *__restrict__ rp, const int32_t *__restrict__ ci,
                                   int64_t width, int nslabs, int32_t *__restrict__ bnd) {
    const int64_t idx = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (idx >= m * (nslabs - 1)) return;
    const int64_t s = idx / m + 1, i = idx % m;
    int64_t lo = rp[i], hi = rp[i + 1];  // first position in [lo, hi) with col >= s*W
    const int64_t key = s * width;
    while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if (ci[mid] < key) lo = mid + 1; else hi = mid;
    }
    bnd[idx] = static_cast<int32_t>(lo);
}

hipError_t slab_bounds_launch(int64_t m, const int32_t *rp, const int32_t *ci, int64_t width, int64_t nslabs,
                              int32_t *bnd, hipStream_t s) {
    if (nslabs <= 1 || m == 0) return hipSuccess;
    const int64_t count = m * (nslabs - 1);
    hipLaunchKernelGGL(slab_bounds_kernel, dim3(static_cast<unsigned>((count + kBlock - 1) / kBlock)), dim3(kBlock), 0, s,
                       m, rp, ci, width, static_cast<int>(nslabs), bnd);
    return hipGetLastError();
}

// Start row of every merge-path share: part[g] = largest i in
// [max(0, d - nnz), min(d, m)] with row_ptr[i] + i <= d, d = min(g*items, m+nnz).
// The walk consumes an entry while the current row still has one and a row
// end otherwise, so after d steps it has finished exactly part[g] rows and
// consumed d - part[g] entries.
__global__ void merge_partition_kernel(int64_t m, int64_t nnz, const int32_t *__restrict__ rp,
                                       int64_t items, int64_t ngroups, int32_t *__restrict__ part) {
    const int64_t g = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (g > ngroups) return;
    const int64_t total = m + nnz;
    const int64_t d = g * items < total ? g * items : total;
    const int64_t lo = d - nnz > 0 ? d - nnz : 0;
    const int64_t hi = d < m ? d : m;
    part[g] = static_cast<int32_t>(last_at_most(lo, hi, d, [&](int64_t i) { return static_cast<int64_t>(rp[i]) + i; }));
}

template <typename TB, typename TV, int VW, int LANES, bool OFF32>
__global__ __launch_bounds__(kBlock) void spmm_merge_kernel(
    int64_t m, int64_t nnz, int K, const int32_t *__restrict__ rp, const int32_t *__restrict__ ci,
    const TV *__restrict__ vals, const int32_t *__restrict__ vperm, const TB *__restrict__ B, int64_t ldb,
    typename acc_of<TB>::type *__restrict__ C, int64_t ldc, const int32_t *__restrict__ part, int64_t items,
    int64_t ngroups, int32_t *__restrict__ carry_row, typename acc_of<TB>::type *__restrict__ carry_val) {
    using A = typename acc_of<TB>::type;
    constexpr int GPB = kBlock / LANES;
    const int lig = threadIdx.x & (LANES - 1);
    const int gbase = (threadIdx.x & (kWave - 1)) & ~(LANES - 1);
    const int64_t blk = xcd_block(blockIdx.x, gridDim.x);
    const int64_t g = blk * GPB + threadIdx.x / LANES;
    if (g >= ngroups) return;
    const int k0 = blockIdx.y * (LANES * VW) + lig * VW;
    const bool kvalid = k0 < K;
    const int koff = kvalid ? k0 : 0;
    const int64_t total = m + nnz;
    const int64_t d0 = g * items;
    const int64_t d1 = d0 + items < total ? d0 + items : total;
    const int64_t i0 = part[g], i1 = part[g + 1];
    const int64_t j1 = d1 - i1;
    int64_t j = d0 - i0;
    A acc[VW];
    for (int64_t r = i0; r < i1; ++r) {  // rows whose end lies in this share
        const int64_t e = rp[r + 1];
        zero<A, VW>(acc);
        accumulate_entries<TB, TV, VW, LANES, OFF32>(j, e, ci, vals, vperm, B, ldb, koff, gbase, lig, acc);
        if (kvalid) vec_store<A, VW>::run(C + r * ldc + k0, acc);
        j = e;
    }
    // Entries of row i1 inside this share: carried to the fix-up.
    const bool has_carry = j < j1;
    if (has_carry) {
        zero<A, VW>(acc);
        accumulate_entries<TB, TV, VW, LANES, OFF32>(j, j1, ci, vals, vperm, B, ldb, koff, gbase, lig, acc);
        if (kvalid) vec_store<A, VW>::run(carry_val + g * K + k0, acc);
    }
    if (lig == 0 && blockIdx.y == 0) carry_row[g] = has_carry ? static_cast<int32_t>(i1) : -1;
}

// One wave per share: the first share of each run of shares carrying the
// same row adds the run's carries, in share order, to that row of C.
template <typename A>
__global__ __launch_bounds__(kBlock) void merge_fixup_kernel(int64_t ngroups, int K, const int32_t *__restrict__ carry_row,
                                                             const A *__restrict__ carry_val, A *__restrict__ C,
                                                             int64_t ldc) {
    const int64_t g = static_cast<int64_t>(blockIdx.x) * (kBlock / kWave) + threadIdx.x / kWave;
    if (g >= ngroups) return;
    const int32_t r = carry_row[g];
    if (r < 0 || (g > 0 && carry_row[g - 1] == r)) return;
    int64_t g_end = g + 1;
    while (g_end < ngroups && carry_row[g_end] == r) ++g_end;
    for (int k = threadIdx.x & (kWave - 1); k < K; k += kWave) {
        A s = A(0);
        for (int64_t h = g; h < g_end; ++h) s += carry_val[h * K + k];
        C[static_cast<int64_t>(r) * ldc + k] += s;
    }
}

// -------------------------------------------------------------------------
// Host launchers
// -------------------------------------------------------------------------
static unsigned grid1(int64_t count, int per) { return static_cast<unsigned>((count + per - 1) / per); }

template <typename TB, typename TV, int VW, int LANES, bool OFF32>
static hipError_t launch_rows(const SpmmArgs &a, hipStream_t s) {
    constexpr int GPB = kBlock / LANES;
    const int64_t nb = (a.m + GPB - 1) / GPB;
    const int64_t ktiles = (a.K + LANES * VW - 1) / (LANES * VW);
    if (nb > 0x7FFFFFFF || ktiles > 65535) return hipErrorInvalidValue;
    hipLaunchKernelGGL((spmm_rows_kernel<TB, TV, VW, LANES, OFF32>), dim3(static_cast<unsigned>(nb), static_cast<unsigned>(ktiles)),
                       dim3(kBlock), 0, s, a.m, static_cast<int>(a.K), a.rp, a.ci, static_cast<const TV *>(a.vals),
                       a.vperm, static_cast<const TB *>(a.B), a.ldb,
                       static_cast<typename acc_of<TB>::type *>(a.C), a.ldc);
    return hipGetLastError();
}

template <typename TB, typename TV, int VW, int LANES, bool OFF32>
static hipError_t launch_slab(const SpmmArgs &a, hipStream_t s) {
    constexpr int GPB = kBlock / LANES;
    const SlabLayout L = slab_layout(a.m, a.n, a.chunk);
    int32_t *bnd = static_cast<int32_t *>(a.ws);
    hipError_t e0 = slab_bounds_launch(a.m, a.rp, a.ci, L.width, L.nslabs, bnd, s);
    if (e0 != hipSuccess) return e0;
    const int64_t nb = (a.m + GPB - 1) / GPB;
    const int64_t ktiles = (a.K + LANES * VW - 1) / (LANES * VW);
    if (nb > 0x7FFFFFFF || ktiles > 65535) return hipErrorInvalidValue;
    for (int sl = 0; sl < L.nslabs; ++sl) {
        hipLaunchKernelGGL((spmm_slab_kernel<TB, TV, VW, LANES, OFF32>),
                           dim3(static_cast<unsigned>(nb), static_cast<unsigned>(ktiles)), dim3(kBlock), 0, s, a.m,
                           static_cast<int>(a.K), a.rp, bnd, static_cast<int>(L.nslabs), sl, a.ci,
                           static_cast<const TV *>(a.vals), a.vperm, static_cast<const TB *>(a.B), a.ldb,
                           static_cast<typename acc_of<TB>::type *>(a.C), a.ldc);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

template <typename TB, typename TV, int VW, int LANES, bool OFF32>
static hipError_t launch_merge(const SpmmArgs &a, hipStream_t s) {
    using A = typename acc_of<TB>::type;
    constexpr int GPB = kBlock / LANES;
    const MergeLayout L = merge_layout(a.m, a.nnz, a.K, a.chunk, sizeof(A));
    char *ws = static_cast<char *>(a.ws);
    int32_t *part = reinterpret_cast<int32_t *>(ws + L.part_off);
    int32_t *carry_row = reinterpret_cast<int32_t *>(ws + L.row_off);
    A *carry_val = reinterpret_cast<A *>(ws + L.val_off);
    hipLaunchKernelGGL(merge_partition_kernel, dim3(grid1(L.ngroups + 1, kBlock)), dim3(kBlock), 0, s, a.m, a.nnz,
                       a.rp, L.items, L.ngroups, part);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int64_t nb = (L.ngroups + GPB - 1) / GPB;
    const int64_t ktiles = (a.K + LANES * VW - 1) / (LANES * VW);
    if (nb > 0x7FFFFFFF || ktiles > 65535) return hipErrorInvalidValue;
    hipLaunchKernelGGL((spmm_merge_kernel<TB, TV, VW, LANES, OFF32>), dim3(static_cast<unsigned>(nb), static_cast<unsigned>(ktiles)),
                       dim3(kBlock), 0, s, a.m, a.nnz, static_cast<int>(a.K), a.rp, a.ci,
                       static_cast<const TV *>(a.vals), a.vperm, static_cast<const TB *>(a.B), a.ldb,
                       static_cast<A *>(a.C), a.ldc, part, L.items, L.ngroups, carry_row, carry_val);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((merge_fixup_kernel<A>), dim3(grid1(L.ngroups, kBlock / kWave)), dim3(kBlock), 0, s, L.ngroups,
                       static_cast<int>(a.K), carry_row, carry_val, static_cast<A *>(a.C), a.ldc);
    return hipGetLastError();
}

template <typename TB, typename TV, int VW, int LANES>
static hipError_t launch_tile(const SpmmArgs &a, hipStream_t s) {
    if constexpr (VW != 4 || sizeof(TB) > 4) {
        return hipErrorInvalidValue;  // the API layer admits TILE only for 16-byte F32 / 8-byte BF16 lanes
    } else {
        constexpr int RPG = 4;
        constexpr int GPB = kBlock / LANES;
        const int64_t rows_per_block = GPB * RPG;
        const int64_t nb = (a.m + rows_per_block - 1) / rows_per_block;
        const size_t lds = static_cast<size_t>(a.chunk) * static_cast<size_t>(a.K) * sizeof(TB);
        if (nb > 0x7FFFFFFF || a.K > LANES * VW || lds > kTileLds) return hipErrorInvalidValue;
        hipLaunchKernelGGL((spmm_tile_kernel<TB, TV, VW, LANES, RPG>), dim3(static_cast<unsigned>(nb)), dim3(kBlock), lds,
                           s, a.m, a.n, static_cast<int>(a.K), a.rp, a.ci, static_cast<const TV *>(a.vals), a.vperm,
                           static_cast<const TB *>(a.B), a.ldb, static_cast<typename acc_of<TB>::type *>(a.C), a.ldc,
                           static_cast<int>(a.chunk));
        return hipGetLastError();
    }
}

template <typename TB, typename TV, int VW, bool OFF32>
static hipError_t dispatch_lanes(const SpmmArgs &a, hipStream_t s) {
    switch (a.lanes) {
#define SPK_CASE(L)                                                                   \
    case L:                                                                           \
        if (a.variant == SPK_VAR_MERGE) return launch_merge<TB, TV, VW, L, OFF32>(a, s); \
        if (a.variant == SPK_VAR_SLAB) return launch_slab<TB, TV, VW, L, OFF32>(a, s);   \
        if (a.variant == SPK_VAR_TILE) return launch_tile<TB, TV, VW, L>(a, s);          \
        return launch_rows<TB, TV, VW, L, OFF32>(a, s);
        SPK_CASE(4)
        SPK_CASE(8)
        SPK_CASE(16)
        SPK_CASE(32)
        SPK_CASE(64)
#undef SPK_CASE
    default: return hipErrorInvalidValue;
    }
}

template <typename TB, typename TV, int VW>
static hipError_t dispatch_off(const SpmmArgs &a, hipStream_t s) {
    // 32-bit element offsets when every element of B (n rows of ldb) is reachable.
    const bool off32 = static_cast<uint64_t>(a.n) * static_cast<uint64_t>(a.ldb) < (1ull << 32);
    return off32 ? dispatch_lanes<TB, TV, VW, true>(a, s) : dispatch_lanes<TB, TV, VW, false>(a, s);
}

hipError_t spmm_launch(const SpmmArgs &a, hipStream_t s) {
    switch (a.b_dtype) {
    case SPK_F32:
        return a.vec > 1 ? dispatch_off<float, float, 4>(a, s) : dispatch_off<float, float, 1>(a, s);
    case SPK_BF16:
        if (a.vec == 8) return dispatch_off<bf16, float, 8>(a, s);
        return a.vec > 1 ? dispatch_off<bf16, float, 4>(a, s) : dispatch_off<bf16, float, 1>(a, s);
    case SPK_F64:
        return a.vec > 1 ? dispatch_off<double, double, 2>(a, s) : dispatch_off<double, double, 1>(a, s);
    default: return hipErrorInvalidValue;
    }
}

// Zero-fill of an m x K block with leading dimension ld (nnz = 0 case).
template <typename A>
__global__ void fill_zero_kernel(int64_t m, int64_t K, A *__restrict__ C, int64_t ld) {
    const int64_t idx = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (idx >= m * K) return;
    C[(idx / K) * ld + idx % K] = A(0);
}

hipError_t zero_fill(void *C, int64_t m, int64_t K, int64_t ld, int32_t dtype, hipStream_t s) {
    const int64_t total = m * K;
    if (total == 0) return hipSuccess;
    const int64_t nb = (total + kBlock - 1) / kBlock;
    if (nb > 0x7FFFFFFF) return hipErrorInvalidValue;
    if (dtype == SPK_F64)
        hipLaunchKernelGGL((fill_zero_kernel<double>), dim3(static_cast<unsigned>(nb)), dim3(kBlock), 0, s, m, K,
                           static_cast<double *>(C), ld);
    else
        hipLaunchKernelGGL((fill_zero_kernel<float>), dim3(static_cast<unsigned>(nb)), dim3(kBlock), 0, s, m, K,
                           static_cast<float *>(C), ld);
    return hipGetLastError();
}

}  // namespace spk
