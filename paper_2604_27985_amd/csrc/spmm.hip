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
#include "tile.h"

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
// column for lanes beyond K (their results are never stored).  The column of
// entry p is cbase + ci[p] (CT = uint16_t: the slab form's 16-bit offsets)
// and its value vals[p + voff] (or vals[vperm[p]]).
template <typename TB, typename TV, int VW, int LANES, bool OFF32, typename CT = int32_t>
__device__ __forceinline__ void accumulate_entries(int64_t a, int64_t b, const CT *__restrict__ ci,
                                                   const TV *__restrict__ vals,
                                                   const int32_t *__restrict__ vperm,
                                                   const TB *__restrict__ B, int64_t ldb, int koff, int gbase,
                                                   int lig, typename acc_of<TB>::type *acc, int32_t cbase = 0,
                                                   int64_t voff = 0) {
    using A = typename acc_of<TB>::type;
    constexpr int U = LANES < 8 ? LANES : 8;
    for (int64_t p0 = a; p0 < b; p0 += LANES) {
        const int64_t p = p0 + lig;
        int c = 0;
        A v = A(0);
        if (p < b) {
            c = cbase + static_cast<int>(__builtin_nontemporal_load(ci + p));
            if (vals) {
                const int64_t pv = vperm ? static_cast<int64_t>(__builtin_nontemporal_load(vperm + p)) : p + voff;
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

// DCSR: group g takes row order[g] of the non-empty rows (g < nrows).
template <typename TB, typename TV, int VW, int LANES, bool OFF32>
__global__ __launch_bounds__(kBlock) void spmm_dcsr_kernel(int64_t nrows, int K, const int32_t *__restrict__ order,
                                                           const int32_t *__restrict__ rp,
                                                           const int32_t *__restrict__ ci,
                                                           const TV *__restrict__ vals, const TB *__restrict__ B,
                                                           int64_t ldb, typename acc_of<TB>::type *__restrict__ C,
                                                           int64_t ldc) {
    using A = typename acc_of<TB>::type;
    constexpr int GPB = kBlock / LANES;
    const int lig = threadIdx.x & (LANES - 1);
    const int gbase = (threadIdx.x & (kWave - 1)) & ~(LANES - 1);
    const int64_t blk = xcd_block(blockIdx.x, gridDim.x);
    const int64_t g = blk * GPB + threadIdx.x / LANES;
    if (g >= nrows) return;
    const int64_t row = order[g];
    const int k0 = blockIdx.y * (LANES * VW) + lig * VW;
    const bool kvalid = k0 < K;
    A acc[VW];
    zero<A, VW>(acc);
    accumulate_entries<TB, TV, VW, LANES, OFF32>(rp[row], rp[row + 1], ci, vals, nullptr, B, ldb, kvalid ? k0 : 0,
                                                 gbase, lig, acc);
    if (kvalid) vec_store<A, VW>::run(C + row * ldc + k0, acc);
}

// Zeros for rows order[0 .. count) (the empty rows of a DCSR order): one
// thread per VW-wide piece of a row, so consecutive threads fill a row with
// vector stores and a wave covers several rows.
template <typename A, int VW>
__global__ void zero_rows_kernel(int64_t count, int64_t pieces, const int32_t *__restrict__ order, A *__restrict__ C,
                                 int64_t ldc) {
    const int64_t idx = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (idx >= count * pieces) return;
    const int64_t g = idx / pieces, k = (idx - g * pieces) * VW;
    A z[VW];
#pragma unroll
    for (int e = 0; e < VW; ++e) z[e] = A(0);
    vec_store<A, VW>::run(C + static_cast<int64_t>(order[g]) * ldc + k, z);
}

// Slab s of the column-slab form (slab16.hip): group g takes run (s, g), whose
// entries are positions [seg[s m + g], seg[s m + g + 1]) of col16 (columns
// s W + col16) with values at A positions apos[s m + g] onward.  Slab 0 writes
// C; a later slab adds its run to C, and a row with an empty run there is
// left alone (no read or write of C).
template <typename TB, typename TV, int VW, int LANES, bool OFF32>
__global__ __launch_bounds__(kBlock) void spmm_s16_kernel(int64_t m, int K, const int32_t *__restrict__ seg,
                                                          const int32_t *__restrict__ apos,
                                                          const uint16_t *__restrict__ col16, int s, int32_t cbase,
                                                          const TV *__restrict__ vals, const TB *__restrict__ B,
                                                          int64_t ldb, typename acc_of<TB>::type *__restrict__ C,
                                                          int64_t ldc) {
    using A = typename acc_of<TB>::type;
    constexpr int GPB = kBlock / LANES;
    const int lig = threadIdx.x & (LANES - 1);
    const int gbase = (threadIdx.x & (kWave - 1)) & ~(LANES - 1);
    const int64_t blk = xcd_block(blockIdx.x, gridDim.x);
    const int64_t row = blk * GPB + threadIdx.x / LANES;
    if (row >= m) return;
    const int64_t run = static_cast<int64_t>(s) * m + row;
    const int64_t a = seg[run], b = seg[run + 1];
    if (s > 0 && a == b) return;  // group-uniform
    const int k0 = blockIdx.y * (LANES * VW) + lig * VW;
    const bool kvalid = k0 < K;
    A acc[VW];
    zero<A, VW>(acc);
    accumulate_entries<TB, TV, VW, LANES, OFF32, uint16_t>(a, b, col16, vals, nullptr, B, ldb, kvalid ? k0 : 0, gbase,
                                                           lig, acc, cbase, static_cast<int64_t>(apos[run]) - a);
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

// ------------------------------------------------------------------ TILE
// A workgroup owns GPB*RPG consecutive rows (RPG per lane group) and walks
// the columns in slabs of W; each slab of B is copied once to LDS and every
// group gathers its rows' entries of that slab from LDS.  A staged row of B
// serves (rows per workgroup) x density entries on average, which cuts the
// L2 gather traffic by that factor for dense-ish matrices.
//
// Memory waits are left to the compiler, which can count them exactly
// because every slab issues the same loads: the next slab's copy (NPT
// 16-byte pieces per thread, read into registers right after the barrier
// that opens a slab and written to the other LDS buffer at its end) and the
// column and value loads of every row's next chunk.  The copy's
// latency hides behind the gathers of the current slab; a chunk fetched in
// one slab is first used in the next.
// One pass for groups of fewer than 16 lanes (K <= 32): lane lig holds entry
// cursor + lig; the in-slab prefix (entries are sorted) is gathered with
// ds_bpermute broadcasts, the cursor advanced past it and the chunk at the
// new cursor fetched.  Returns the prefix length.
template <typename TB, typename TV, int VW, int LANES>
__device__ __forceinline__ int tile_pass(const TB *__restrict__ buf, int K, int koff, int32_t c0, int32_t c1,
                                         int gbase, uint64_t gmask, int lig, bool has_vals,
                                         const int32_t *__restrict__ ci, const TV *__restrict__ vsrc, int32_t last,
                                         int32_t &cur, int32_t end, int &c, TV &v, float (&acc)[VW]) {
    constexpr int U = LANES < 8 ? LANES : 8;
    const bool in = cur + lig < end && c < c1;
    const int cnt = __popcll(__ballot(in) & gmask);
    const int crel = in ? c - c0 : 0;
    const float vin = in ? (has_vals ? static_cast<float>(v) : 1.f) : 0.f;
    cur += cnt;  // the next chunk's fetch goes out before the gathers
    tile_fetch(cur + lig, last, ci, vsrc, c, v);
    for (int t = 0; t < cnt; t += U) {
        int cc[U];
        float vv[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            cc[u] = lane_read(crel, gbase + t + u);
            vv[u] = lane_read(vin, gbase + t + u);
        }
        float bv[U][VW];
#pragma unroll
        for (int u = 0; u < U; ++u) vec_load<TB, VW>::run(buf + cc[u] * K + koff, bv[u]);
#pragma unroll
        for (int u = 0; u < U; ++u)
#pragma unroll
            for (int e = 0; e < VW; ++e) acc[e] = fma(vv[u], bv[u][e], acc[e]);
    }
    return cnt;
}

// Entries N .. N+3 of the chunk: LDS row offset and weight broadcast from
// lanes N .. N+3 of each 16-lane row, four independent gathers, then the
// FMAs.
template <typename TB, int VW, int N>
__device__ __forceinline__ void tile_quad(const unsigned char *__restrict__ smem, uint32_t base, int offb, float w,
                                          float (&acc)[VW]) {
    const uint32_t a[4] = {row_bcast_add<N>(offb, base), row_bcast_add<N + 1>(offb, base),
                           row_bcast_add<N + 2>(offb, base), row_bcast_add<N + 3>(offb, base)};
    const float x[4] = {row_bcast<N>(w), row_bcast<N + 1>(w), row_bcast<N + 2>(w), row_bcast<N + 3>(w)};
    float bv[4][VW];
#pragma unroll
    for (int q = 0; q < 4; ++q) vec_load<TB, VW>::run(reinterpret_cast<const TB *>(smem + a[q]), bv[q]);
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
        for (int e = 0; e < VW; ++e) acc[e] = fma(x[q], bv[q][e], acc[e]);
}

// One pass for groups of 16 or more lanes: every 16-lane row of a group holds
// the same 16-entry chunk (lane r16 = lane mod 16 holds entry cursor + r16).
// The in-slab prefix is gathered by broadcasting entry u from lane u of the
// row, four entries at a time (group-divergent: a group runs only the quads
// its prefix reaches); the last quad adds zero-weight terms of a valid LDS row.
template <typename TB, typename TV, int VW>
__device__ __forceinline__ int tile_pass16(const TB *__restrict__ buf, int K, int koff, int32_t c0, int32_t c1,
                                           int r16, int gbase16, bool has_vals, const int32_t *__restrict__ ci,
                                           const TV *__restrict__ vsrc, int32_t last, int32_t &cur, int32_t end,
                                           int &c, TV &v, float (&acc)[VW]) {
    const bool in = cur + r16 < end && c < c1;
    const int cnt = count16(__ballot(in), gbase16);
    const int offb = in ? (c - c0) * K * static_cast<int>(sizeof(TB)) : 0;  // row offset in the slab, bytes
    const float w = in ? (has_vals ? static_cast<float>(v) : 1.f) : 0.f;
    // the next chunk's fetch goes out before the gathers (off and w hold what
    // they need of this one); a chunk with nothing in the slab is fetched again
    cur += cnt;
    tile_fetch(cur + r16, last, ci, vsrc, c, v);
    // LDS byte address of a gather: the buffer plus this lane's K offset plus
    // the broadcast row offset
    const unsigned char *smem = reinterpret_cast<const unsigned char *>(buf);
    const uint32_t base = static_cast<uint32_t>(koff * sizeof(TB));
    if (cnt > 0) tile_quad<TB, VW, 0>(smem, base, offb, w, acc);
    if (cnt > 4) tile_quad<TB, VW, 4>(smem, base, offb, w, acc);
    if (cnt > 8) tile_quad<TB, VW, 8>(smem, base, offb, w, acc);
    if (cnt > 12) tile_quad<TB, VW, 12>(smem, base, offb, w, acc);
    return cnt;
}

// The entries of one row inside the slab.  The first pass uses the chunk
// fetched during the previous slab; only a chunk wholly inside the slab needs
// the fresh chunk at once, and only that rarer loop waits for it.
template <typename TB, typename TV, int VW, int LANES>
__device__ __forceinline__ void tile_row(const TB *__restrict__ buf, int K, int koff, int32_t c0, int32_t c1,
                                         int gbase, uint64_t gmask, int lig, bool has_vals,
                                         const int32_t *__restrict__ ci, const TV *__restrict__ vsrc, int32_t last,
                                         int32_t &cur, int32_t end, int &c, TV &v, float (&acc)[VW]) {
    if constexpr (LANES >= 16) {
        const int r16 = lig & 15;
        if (tile_pass16<TB, TV, VW>(buf, K, koff, c0, c1, r16, gbase, has_vals, ci, vsrc, last, cur, end, c, v,
                                    acc) == 16) {
            while (tile_pass16<TB, TV, VW>(buf, K, koff, c0, c1, r16, gbase, has_vals, ci, vsrc, last, cur, end, c,
                                           v, acc) == 16) {
            }
        }
    } else {
        if (tile_pass<TB, TV, VW, LANES>(buf, K, koff, c0, c1, gbase, gmask, lig, has_vals, ci, vsrc, last, cur, end,
                                         c, v, acc) == LANES) {
            while (tile_pass<TB, TV, VW, LANES>(buf, K, koff, c0, c1, gbase, gmask, lig, has_vals, ci, vsrc, last,
                                                cur, end, c, v, acc) == LANES) {
            }
        }
    }
}

template <typename TB, typename TV, int VW, int LANES, int RPG, int NPT>
__global__ __launch_bounds__(kBlock) void spmm_tile_kernel(int64_t m, int64_t n, int64_t nnz, int K,
                                                           const int32_t *__restrict__ rp,
                                                           const int32_t *__restrict__ ci,
                                                           const TV *__restrict__ vals, const TB *__restrict__ B,
                                                           int64_t ldb, float *__restrict__ C, int64_t ldc, int W) {
    static_assert(sizeof(TV) == 4, "values are F32 on this path");
    extern __shared__ __align__(16) unsigned char smem[];
    TB *Bs = reinterpret_cast<TB *>(smem);  // two buffers of NPT * 4 KiB
    constexpr int buf_elems = NPT * kTilePiece / static_cast<int>(sizeof(TB));
    constexpr int GPB = kBlock / LANES;
    const int lane = threadIdx.x & (kWave - 1);
    const int lig = threadIdx.x & (LANES - 1);
    const int gbase = lane & ~(LANES - 1);
    const uint64_t gmask = LANES == 64 ? ~0ull : (((1ull << LANES) - 1) << gbase);
    const int64_t blk = xcd_block(blockIdx.x, gridDim.x);
    const int64_t row0 = (blk * GPB + threadIdx.x / LANES) * RPG;
    const int k0 = lig * VW;
    const bool kvalid = k0 < K;
    const int koff = kvalid ? k0 : 0;
    const int32_t last = static_cast<int32_t>(nnz - 1);  // row_ptr is int32: positions fit
    const bool has_vals = vals != nullptr;
    const TV *vsrc = has_vals ? vals : reinterpret_cast<const TV *>(ci);
    const int pos = LANES >= 16 ? (lig & 15) : lig;  // the lane's entry within a chunk
    const int per_row = K / kTileSV<TB>;              // K is a multiple of the 16-byte width
    int32_t cur[RPG], end[RPG];
#pragma unroll
    for (int r = 0; r < RPG; ++r) {
        const int64_t row = row0 + r;
        cur[r] = row < m ? rp[row] : 0;
        end[r] = row < m ? rp[row + 1] : 0;
    }
    u32x4 stg[NPT];
    TileCopy<TB, NPT> copy;
    copy.layout(static_cast<int>(n < W ? n : W), per_row, ldb);
    copy.load(B, ldb, 0, stg);
    tile_store<TB, NPT>(Bs, stg);
    int pc[RPG];
    TV pv[RPG];
    float acc[RPG][VW];
#pragma unroll
    for (int r = 0; r < RPG; ++r) {
        zero<float, VW>(acc[r]);
        tile_fetch(cur[r] + pos, last, ci, vsrc, pc[r], pv[r]);
    }
    int sl = 0;
    for (int32_t c0 = 0; c0 < n; c0 += W, ++sl) {
        const int32_t c1 = static_cast<int32_t>(n - c0 < W ? n : c0 + W);
        __syncthreads();  // slab sl is in LDS; every group is done with the other buffer
        // The next slab's copy into registers; the last slab reads itself
        // again so that every slab issues the same loads.
        const int32_t nx = c1 < n ? c1 : c0;
        if (n - nx < W) copy.layout(static_cast<int>(n - nx), per_row, ldb);  // a narrower last slab
        copy.load(B, ldb, nx, stg);
        const TB *buf = Bs + (sl & 1) * buf_elems;
#pragma unroll
        for (int r = 0; r < RPG; ++r)
            tile_row<TB, TV, VW, LANES>(buf, K, koff, c0, c1, gbase, gmask, lig, has_vals, ci, vsrc, last, cur[r],
                                        end[r], pc[r], pv[r], acc[r]);
        tile_store<TB, NPT>(Bs + ((sl + 1) & 1) * buf_elems, stg);
    }
    if (!kvalid) return;
#pragma unroll
    for (int r = 0; r < RPG; ++r) {
        const int64_t row = row0 + r;
        if (row < m) vec_store<float, VW>::run(C + row * ldc + k0, acc[r]);
    }
}

// TILE with one entry per 4-lane quad (16-lane groups, rows of B of 128, 256
// or 512 bytes).  The same slabs and chunks as above; inside a group the four
// quads take four entries at once and each lane covers a quarter of the row
// (NP pieces of 16 bytes), so an entry costs its FMAs, one address and one
// weight broadcast per quad instead of per lane.  A chunk is fetched so that
// lane 4q + j holds entry 4j + q: in step s quad q adds entry 4s + q, whose
// row offset and weight sit on lane 4q + s (quad_perm broadcasts).  In read i
// of a step quad q reads the 64-byte group quad_group(i, q) of its row
// ((i + q) mod NP, rotated within halves for NP = 8), so the four quads of a
// group hit different bank groups.  Each quad thus accumulates every group of
// the row in a rotated order.  At the end lane (q, j) gathers groups q + 4h
// from quad (q - k) mod 4 with row_ror:4k (DPP 0x120 + 4k, lane l reads lane
// l - 4k of its row): that quad holds group q + 4h in acc[(4h + k) mod NP].
template <typename TB, int NP, int S>
__device__ __forceinline__ void spmm_qstep(const unsigned char *__restrict__ smem, const uint32_t (&pb)[NP],
                                           int offb, float w, float (&acc)[NP][kTileSV<TB>]) {
    constexpr int SV = kTileSV<TB>;
    const float x = quad_bcast<S>(w);
    float bv[NP][SV];
#pragma unroll
    for (int i = 0; i < NP; ++i)
        vec_load<TB, SV>::run(reinterpret_cast<const TB *>(smem + quad_bcast_add<S>(offb, pb[i])), bv[i]);
#pragma unroll
    for (int i = 0; i < NP; ++i)
#pragma unroll
        for (int e = 0; e < SV; ++e) acc[i][e] = fma(x, bv[i][e], acc[i][e]);
}

template <typename TB, typename TV, int NP>
__device__ __forceinline__ int spmm_tileq_pass(const unsigned char *__restrict__ smem, int32_t c0, int32_t c1,
                                               int slot, int gbase16, bool has_vals, const int32_t *__restrict__ ci,
                                               const TV *__restrict__ vsrc, int32_t last, int32_t &cur, int32_t end,
                                               int &c, TV &v, const uint32_t (&pb)[NP],
                                               float (&acc)[NP][kTileSV<TB>]) {
    constexpr int kRowShift = NP == 2 ? 7 : NP == 4 ? 8 : 9;  // log2 of a row's bytes
    const bool in = cur + slot < end && c < c1;
    const int cnt = count16(__builtin_amdgcn_ballot_w64(in), gbase16);
    const int offb = in ? (c - c0) << kRowShift : 0;
    // entries past the in-slab prefix are added with weight zero (valid row 0)
    const float w = in ? (has_vals ? static_cast<float>(v) : 1.f) : 0.f;
    cur += cnt;
    tile_fetch(cur + slot, last, ci, vsrc, c, v);
    if (cnt > 0) spmm_qstep<TB, NP, 0>(smem, pb, offb, w, acc);
    if (cnt > 4) spmm_qstep<TB, NP, 1>(smem, pb, offb, w, acc);
    if (cnt > 8) spmm_qstep<TB, NP, 2>(smem, pb, offb, w, acc);
    if (cnt > 12) spmm_qstep<TB, NP, 3>(smem, pb, offb, w, acc);
    return cnt;
}

template <int CTRL>
__device__ __forceinline__ float dpp_move(float v) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xF, 0xF, true));
}

template <typename TB, typename TV, int NP, int RPG, int NPT, int BS>
__global__ __launch_bounds__(BS, BS > kBlock ? 4 : 1) void spmm_tileq_kernel(int64_t m, int64_t n, int64_t nnz,
                                                            const int32_t *__restrict__ rp,
                                                            const int32_t *__restrict__ ci,
                                                            const TV *__restrict__ vals, const TB *__restrict__ B,
                                                            int64_t ldb, float *__restrict__ C, int64_t ldc, int W) {
    static_assert(sizeof(TV) == 4, "values are F32 on this path");
    constexpr int SV = kTileSV<TB>;
    constexpr int per_row = 4 * NP;
    constexpr int buf_bytes = NPT * BS * 16;
    extern __shared__ __align__(16) unsigned char smem[];
    constexpr int GPB = BS / 16;
    const int lane = threadIdx.x & (kWave - 1);
    const int lig = threadIdx.x & 15;
    const int q = lig >> 2, j = lig & 3;
    const int slot = 4 * j + q;
    const int gbase = lane & ~15;
    const int64_t blk = xcd_block(blockIdx.x, gridDim.x);
    const int64_t row0 = (blk * GPB + threadIdx.x / 16) * RPG;
    const int32_t last = static_cast<int32_t>(nnz - 1);  // row_ptr is int32: positions fit
    const bool has_vals = vals != nullptr;
    const TV *vsrc = has_vals ? vals : reinterpret_cast<const TV *>(ci);
    uint32_t pb[NP];  // byte offset in a row of piece j of group quad_group(i, q)
#pragma unroll
    for (int i = 0; i < NP; ++i) pb[i] = static_cast<uint32_t>((quad_group<NP>(i, q) * 4 + j) * 16);
    int32_t cur[RPG], end[RPG];
#pragma unroll
    for (int r = 0; r < RPG; ++r) {
        const int64_t row = row0 + r;
        cur[r] = row < m ? rp[row] : 0;
        end[r] = row < m ? rp[row + 1] : 0;
    }
    u32x4 stg[NPT];
    TileCopy<TB, NPT, BS> copy;
    copy.layout(static_cast<int>(n < W ? n : W), per_row, ldb);
    copy.load(B, ldb, 0, stg);
    tile_store<TB, NPT, BS>(reinterpret_cast<TB *>(smem), stg);
    int pc[RPG];
    TV pv[RPG];
    float acc[RPG][NP][SV];
#pragma unroll
    for (int r = 0; r < RPG; ++r) {
#pragma unroll
        for (int i = 0; i < NP; ++i) zero<float, SV>(acc[r][i]);
        tile_fetch(cur[r] + slot, last, ci, vsrc, pc[r], pv[r]);
    }
    int sl = 0;
    for (int32_t c0 = 0; c0 < n; c0 += W, ++sl) {
        const int32_t c1 = static_cast<int32_t>(n - c0 < W ? n : c0 + W);
        __syncthreads();  // slab sl is in LDS; every group is done with the other buffer
        const int32_t nx = c1 < n ? c1 : c0;  // the last slab reads itself again: same loads every slab
        if (n - nx < W) copy.layout(static_cast<int>(n - nx), per_row, ldb);
        copy.load(B, ldb, nx, stg);
        const unsigned char *buf = smem + (sl & 1) * buf_bytes;
#pragma unroll
        for (int r = 0; r < RPG; ++r) {
            if (spmm_tileq_pass<TB, TV, NP>(buf, c0, c1, slot, gbase, has_vals, ci, vsrc, last, cur[r], end[r],
                                                 pc[r], pv[r], pb, acc[r]) == 16) {
                while (spmm_tileq_pass<TB, TV, NP>(buf, c0, c1, slot, gbase, has_vals, ci, vsrc, last, cur[r],
                                                        end[r], pc[r], pv[r], pb, acc[r]) == 16) {
                }
            }
        }
        tile_store<TB, NPT, BS>(reinterpret_cast<TB *>(smem + ((sl + 1) & 1) * buf_bytes), stg);
    }
    // lane (q, j) sums groups g = q + 4h of each row over the four quads and,
    // for g < NP, stores piece j of it: elements (4g + j) * SV .. + SV
    constexpr int H = NP > 4 ? NP / 4 : 1;
#pragma unroll
    for (int r = 0; r < RPG; ++r) {
        const int64_t row = row0 + r;
#pragma unroll
        for (int h = 0; h < H; ++h) {
            float out[SV];
#pragma unroll
            for (int e = 0; e < SV; ++e) {
                float t = acc[r][(4 * h) % NP][e];
                t += dpp_move<0x124>(acc[r][(4 * h + 1) % NP][e]);
                t += dpp_move<0x128>(acc[r][(4 * h + 2) % NP][e]);
                t += dpp_move<0x12C>(acc[r][(4 * h + 3) % NP][e]);
                out[e] = t;
            }
            const int g = q + 4 * h;
            if (row < m && g < NP) vec_store<float, SV>::run(C + row * ldc + (4 * g + j) * SV, out);
        }
    }
}

template <typename TB, typename TV, int NP, int RPG, int NPT, int BS>
static hipError_t launch_tileq_npt(const SpmmArgs &a, const TV *vals, hipStream_t s) {
    constexpr int GPB = BS / 16;
    const int64_t nb = (a.m + GPB * RPG - 1) / (GPB * RPG);
    const size_t lds = 2 * static_cast<size_t>(NPT) * BS * 16;  // two slab buffers
    if (lds > 65536) {  // beyond the default dynamic LDS limit (gfx950 has 160 KiB per CU)
        const hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void *>(&spmm_tileq_kernel<TB, TV, NP, RPG, NPT, BS>),
                                                 hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(lds));
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL((spmm_tileq_kernel<TB, TV, NP, RPG, NPT, BS>), dim3(static_cast<unsigned>(nb)), dim3(BS), lds,
                       s, a.m, a.n, a.nnz, a.rp, a.ci, vals, static_cast<const TB *>(a.B), a.ldb,
                       static_cast<float *>(a.C), a.ldc, static_cast<int>(a.chunk));
    return hipGetLastError();
}

// BS threads per workgroup: a copy round moves BS * 16 bytes, so a slab of
// up to 32 KiB takes 2, 4 or 8 rounds.
template <typename TB, typename TV, int NP, int RPG, int BS = kBlock>
static hipError_t launch_tileq_rpg(const SpmmArgs &a, const TV *vals, hipStream_t s) {
    constexpr int GPB = BS / 16;
    constexpr int64_t round = BS * 16;
    const int64_t nb = (a.m + GPB * RPG - 1) / (GPB * RPG);
    const int64_t slab_bytes = a.chunk * a.K * static_cast<int64_t>(sizeof(TB));
    if (!grid_fits(nb, BS)) return kGridTooLarge;
    if (a.K * static_cast<int64_t>(sizeof(TB)) != 64 * NP || a.chunk < 1 ||
        2 * slab_bytes > (BS == 1024 ? 2 : 1) * static_cast<int64_t>(kTileLds) || a.n > 0x7FFFFFFF)
        return hipErrorInvalidValue;
    if (slab_bytes <= 2 * round) return launch_tileq_npt<TB, TV, NP, RPG, 2, BS>(a, vals, s);
    if (slab_bytes <= 4 * round) return launch_tileq_npt<TB, TV, NP, RPG, 4, BS>(a, vals, s);
    if constexpr (BS == kBlock) return launch_tileq_npt<TB, TV, NP, RPG, 8, BS>(a, vals, s);
    return hipErrorInvalidValue;
}

// Rows of 128 bytes (NP = 2), 256 bytes (NP = 4) or 512 bytes (NP = 8, F32
// only).  A row of 32 accumulators per lane (F32 rows of 512 bytes, BF16 rows
// of 256) keeps 4 rows per group whatever the plan asks: 8 would not fit the
// registers.
template <typename TB, typename TV>
static hipError_t launch_tileq(const SpmmArgs &a, const TV *vals, hipStream_t s) {
    const bool r8 = a.rows_per_group == 8;
    if (a.rows_per_group == 2) {
        // wide plans: 512 threads with two rows per group for slabs up to
        // 32 KiB, else 1024 threads with one row per group
        const bool big = a.chunk * a.K * static_cast<int64_t>(sizeof(TB)) > kTileLds / 2;
        switch (a.K * static_cast<int64_t>(sizeof(TB))) {
        case 128: return big ? launch_tileq_rpg<TB, TV, 2, 1, 1024>(a, vals, s) : launch_tileq_rpg<TB, TV, 2, 2, 512>(a, vals, s);
        case 256: return big ? launch_tileq_rpg<TB, TV, 4, 1, 1024>(a, vals, s) : launch_tileq_rpg<TB, TV, 4, 2, 512>(a, vals, s);
        case 512:  // 32 accumulators per lane and row: 1024 threads, one row per group
            if constexpr (sizeof(TB) == 4) return launch_tileq_rpg<TB, TV, 8, 1, 1024>(a, vals, s);
            return hipErrorInvalidValue;
        default: return hipErrorInvalidValue;
        }
    }
    switch (a.K * static_cast<int64_t>(sizeof(TB))) {
    case 128: return r8 ? launch_tileq_rpg<TB, TV, 2, 8>(a, vals, s) : launch_tileq_rpg<TB, TV, 2, 4>(a, vals, s);
    case 256:
        if constexpr (sizeof(TB) == 4)
            if (r8) return launch_tileq_rpg<TB, TV, 4, 8>(a, vals, s);
        return launch_tileq_rpg<TB, TV, 4, 4>(a, vals, s);
    case 512:
        if constexpr (sizeof(TB) == 4) return launch_tileq_rpg<TB, TV, 8, 4>(a, vals, s);
        return hipErrorInvalidValue;  // BF16 rows of 256 elements: 64 accumulators per lane and row
    default: return hipErrorInvalidValue;
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

// A long run's carries for columns k0 + b * 64 (b < KB), D shares per batch,
// added in share order, so the sum is the same as one carry at a time.
template <typename A, int KB>
__device__ __forceinline__ void fixup_long_run(int64_t g, int64_t g_end, int K, int lane, int32_t r,
                                               const A *__restrict__ carry_val, A *__restrict__ C, int64_t ldc) {
    constexpr int D = 16;
    for (int k0 = lane; k0 < K; k0 += KB * kWave) {
        A s[KB];
#pragma unroll
        for (int b = 0; b < KB; ++b) s[b] = A(0);
        for (int64_t h = g; h < g_end; h += D) {
            A v[D][KB];
#pragma unroll
            for (int u = 0; u < D; ++u) {
                const int64_t hu = h + u < g_end ? h + u : g_end - 1;
#pragma unroll
                for (int b = 0; b < KB; ++b) {
                    const int k = k0 + b * kWave;
                    v[u][b] = carry_val[hu * K + (k < K ? k : 0)];
                }
            }
#pragma unroll
            for (int u = 0; u < D; ++u)
                if (h + u < g_end)  // wave-uniform condition
#pragma unroll
                    for (int b = 0; b < KB; ++b) s[b] += v[u][b];
        }
#pragma unroll
        for (int b = 0; b < KB; ++b) {
            const int k = k0 + b * kWave;
            if (k < K) C[static_cast<int64_t>(r) * ldc + k] += s[b];
        }
    }
}

// One wave per share: the first share of each run of shares carrying the
// same row adds the run's carries, in share order, to that row of C.  Loads
// go out from clamped indices with no branch around them, so that a batch is
// in flight at once: a hub row's run spans thousands of shares, and its chain
// of batches is the kernel's critical path.
template <typename A>
__global__ __launch_bounds__(kBlock) void merge_fixup_kernel(int64_t ngroups, int K, const int32_t *__restrict__ carry_row,
                                                             const A *__restrict__ carry_val, A *__restrict__ C,
                                                             int64_t ldc) {
    const int64_t g = static_cast<int64_t>(blockIdx.x) * (kBlock / kWave) + threadIdx.x / kWave;
    if (g >= ngroups) return;
    const int32_t r = carry_row[g];
    if (r < 0 || (g > 0 && carry_row[g - 1] == r)) return;
    // The run's end, 256 shares per probe: each lane tests four shares and the
    // first share that carries another row (or lies past the end) marks it.
    // The conditions above are uniform over the wave, so all 64 lanes take
    // part.
    const int lane = threadIdx.x & (kWave - 1);
    constexpr int E = 4;
    int64_t g_end = g + 1;
    for (bool found = false; !found; ) {
        int32_t cr[E];
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const int64_t h = g_end + e * kWave + lane;
            cr[e] = carry_row[h < ngroups ? h : ngroups - 1];
        }
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const int64_t h = g_end + e * kWave + lane;
            const uint64_t other = __ballot(!(h < ngroups && cr[e] == r));
            if (other) {
                g_end += e * kWave + __ffsll(static_cast<long long>(other)) - 1;
                found = true;
                break;
            }
        }
        if (!found) g_end += E * kWave;
    }
    if (g_end - g <= 4) {  // most runs: one share and its successor
        for (int k = lane; k < K; k += kWave) {
            A s = A(0);
            for (int64_t h = g; h < g_end; ++h) s += carry_val[h * K + k];
            C[static_cast<int64_t>(r) * ldc + k] += s;
        }
        return;
    }
    if (K <= kWave) fixup_long_run<A, 1>(g, g_end, K, lane, r, carry_val, C, ldc);
    else if (K <= 2 * kWave) fixup_long_run<A, 2>(g, g_end, K, lane, r, carry_val, C, ldc);
    else fixup_long_run<A, 4>(g, g_end, K, lane, r, carry_val, C, ldc);
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
    if (!grid_fits(nb, kBlock)) return kGridTooLarge;
    if (ktiles > 65535) return hipErrorInvalidValue;
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
    if (!grid_fits(nb, kBlock)) return kGridTooLarge;
    if (ktiles > 65535) return hipErrorInvalidValue;
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
static hipError_t launch_s16(const SpmmArgs &a, hipStream_t s) {
    constexpr int GPB = kBlock / LANES;
    const int64_t nb = (a.m + GPB - 1) / GPB;
    const int64_t ktiles = (a.K + LANES * VW - 1) / (LANES * VW);
    if (!grid_fits(nb, kBlock)) return kGridTooLarge;
    if (ktiles > 65535 || a.s16.nslabs < 1) return hipErrorInvalidValue;
    for (int64_t sl = 0; sl < a.s16.nslabs; ++sl) {
        hipLaunchKernelGGL((spmm_s16_kernel<TB, TV, VW, LANES, OFF32>),
                           dim3(static_cast<unsigned>(nb), static_cast<unsigned>(ktiles)), dim3(kBlock), 0, s, a.m,
                           static_cast<int>(a.K), a.s16.seg, a.s16.apos, a.s16.col16, static_cast<int>(sl),
                           static_cast<int32_t>(sl * a.s16.width), static_cast<const TV *>(a.vals),
                           static_cast<const TB *>(a.B), a.ldb, static_cast<typename acc_of<TB>::type *>(a.C), a.ldc);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

template <typename TB, typename TV, int VW, int LANES, bool OFF32>
static hipError_t launch_dcsr(const SpmmArgs &a, hipStream_t s) {
    using A = typename acc_of<TB>::type;
    constexpr int GPB = kBlock / LANES;
    const int64_t nr = a.hv.nrows;
    const int64_t ktiles = (a.K + LANES * VW - 1) / (LANES * VW);
    if (ktiles > 65535 || nr < 0 || nr > a.m) return hipErrorInvalidValue;
    if (nr > 0) {
        const int64_t nb = (nr + GPB - 1) / GPB;
        if (!grid_fits(nb, kBlock)) return kGridTooLarge;
        hipLaunchKernelGGL((spmm_dcsr_kernel<TB, TV, VW, LANES, OFF32>),
                           dim3(static_cast<unsigned>(nb), static_cast<unsigned>(ktiles)), dim3(kBlock), 0, s, nr,
                           static_cast<int>(a.K), a.hv.order, a.rp, a.ci, static_cast<const TV *>(a.vals),
                           static_cast<const TB *>(a.B), a.ldb, static_cast<A *>(a.C), a.ldc);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    const int64_t empty = a.m - nr;
    if (empty > 0) {
        // 16-byte stores when rows of C are 16-byte aligned pieces
        const bool v4 = sizeof(A) == 4 && a.K % 4 == 0 && a.ldc % 4 == 0 &&
                        reinterpret_cast<uintptr_t>(a.C) % 16 == 0;
        const int64_t pieces = v4 ? a.K / 4 : a.K;
        const int64_t total = empty * pieces;
        const int64_t nb = (total + kBlock - 1) / kBlock;
        if (!grid_fits(nb, kBlock)) return kGridTooLarge;
        if (v4)
            hipLaunchKernelGGL((zero_rows_kernel<A, 4>), dim3(static_cast<unsigned>(nb)), dim3(kBlock), 0, s, empty,
                               pieces, a.hv.order + nr, static_cast<A *>(a.C), a.ldc);
        else
            hipLaunchKernelGGL((zero_rows_kernel<A, 1>), dim3(static_cast<unsigned>(nb)), dim3(kBlock), 0, s, empty,
                               pieces, a.hv.order + nr, static_cast<A *>(a.C), a.ldc);
        return hipGetLastError();
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
    const int64_t nb = (L.ngroups + GPB - 1) / GPB;
    const int64_t ktiles = (a.K + LANES * VW - 1) / (LANES * VW);
    constexpr int kWpb = kBlock / kWave;  // fix-up: one wave per group
    if (!grid_fits(nb, kBlock) || !grid_fits((L.ngroups + kWpb - 1) / kWpb, kBlock)) return kGridTooLarge;
    if (ktiles > 65535) return hipErrorInvalidValue;
    hipLaunchKernelGGL(merge_partition_kernel, dim3(grid1(L.ngroups + 1, kBlock)), dim3(kBlock), 0, s, a.m, a.nnz,
                       a.rp, L.items, L.ngroups, part);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((spmm_merge_kernel<TB, TV, VW, LANES, OFF32>), dim3(static_cast<unsigned>(nb), static_cast<unsigned>(ktiles)),
                       dim3(kBlock), 0, s, a.m, a.nnz, static_cast<int>(a.K), a.rp, a.ci,
                       static_cast<const TV *>(a.vals), a.vperm, static_cast<const TB *>(a.B), a.ldb,
                       static_cast<A *>(a.C), a.ldc, part, L.items, L.ngroups, carry_row, carry_val);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((merge_fixup_kernel<A>), dim3(grid1(L.ngroups, kWpb)), dim3(kBlock), 0, s, L.ngroups,
                       static_cast<int>(a.K), carry_row, carry_val, static_cast<A *>(a.C), a.ldc);
    return hipGetLastError();
}

// Values of a permuted CSR (the transpose in the backward pass) in entry order.
template <typename TV>
__global__ void gather_vals_kernel(int64_t nnz, const TV *__restrict__ vals, const int32_t *__restrict__ vperm,
                                   TV *__restrict__ out) {
    const int64_t p = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (p < nnz) out[p] = vals[vperm[p]];
}

template <typename TB, typename TV, int VW, int LANES, int RPG, int NPT>
static hipError_t launch_tile_npt(const SpmmArgs &a, const TV *vals, hipStream_t s) {
    constexpr int GPB = kBlock / LANES;
    const int64_t rows_per_block = GPB * RPG;
    const int64_t nb = (a.m + rows_per_block - 1) / rows_per_block;
    const size_t lds = 2 * static_cast<size_t>(NPT) * kTilePiece;  // two slab buffers
    hipLaunchKernelGGL((spmm_tile_kernel<TB, TV, VW, LANES, RPG, NPT>), dim3(static_cast<unsigned>(nb)), dim3(kBlock),
                       lds, s, a.m, a.n, a.nnz, static_cast<int>(a.K), a.rp, a.ci, vals, static_cast<const TB *>(a.B),
                       a.ldb, static_cast<float *>(a.C), a.ldc, static_cast<int>(a.chunk));
    return hipGetLastError();
}

template <typename TB, typename TV, int VW, int LANES, int RPG>
static hipError_t launch_tile_rpg(const SpmmArgs &a, const TV *vals, hipStream_t s) {
    const int64_t rows_per_block = (kBlock / LANES) * RPG;
    const int64_t nb = (a.m + rows_per_block - 1) / rows_per_block;
    const int64_t slab_bytes = a.chunk * a.K * static_cast<int64_t>(sizeof(TB));
    if (!grid_fits(nb, kBlock)) return kGridTooLarge;
    if (a.K > LANES * VW || a.chunk < 1 || 2 * slab_bytes > kTileLds || a.n > 0x7FFFFFFF)
        return hipErrorInvalidValue;
    // copy rounds per slab: 2, 4 or 8 (a buffer of 8, 16 or 32 KiB)
    if (slab_bytes <= 2 * kTilePiece) return launch_tile_npt<TB, TV, VW, LANES, RPG, 2>(a, vals, s);
    if (slab_bytes <= 4 * kTilePiece) return launch_tile_npt<TB, TV, VW, LANES, RPG, 4>(a, vals, s);
    return launch_tile_npt<TB, TV, VW, LANES, RPG, 8>(a, vals, s);
}

template <typename TB, typename TV, int VW, int LANES>
static hipError_t launch_tile(const SpmmArgs &a, hipStream_t s) {
    if constexpr (VW != 4 || sizeof(TB) > 4) {
        return hipErrorInvalidValue;  // the API layer admits TILE only for 16-byte F32 / 8-byte BF16 lanes
    } else {
        const TV *vals = static_cast<const TV *>(a.vals);
        if (vals && a.vperm) {
            if (!a.ws) return hipErrorInvalidValue;
            TV *dense = static_cast<TV *>(a.ws);
            hipLaunchKernelGGL((gather_vals_kernel<TV>), dim3(grid1(a.nnz, kBlock)), dim3(kBlock), 0, s, a.nnz, vals,
                               a.vperm, dense);
            const hipError_t e = hipGetLastError();
            if (e != hipSuccess) return e;
            vals = dense;
        }
        if (a.quad_split) return launch_tileq<TB, TV>(a, vals, s);
        return a.rows_per_group == 8 ? launch_tile_rpg<TB, TV, VW, LANES, 8>(a, vals, s)
                                     : launch_tile_rpg<TB, TV, VW, LANES, 4>(a, vals, s);
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
        if (a.variant == SPK_VAR_SLAB16) return launch_s16<TB, TV, VW, L, OFF32>(a, s);  \
        if (a.variant == SPK_VAR_DCSR) return launch_dcsr<TB, TV, VW, L, OFF32>(a, s);   \
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
    if (!grid_fits(nb, kBlock)) return kGridTooLarge;
    if (dtype == SPK_F64)
        hipLaunchKernelGGL((fill_zero_kernel<double>), dim3(static_cast<unsigned>(nb)), dim3(kBlock), 0, s, m, K,
                           static_cast<double *>(C), ld);
    else
        hipLaunchKernelGGL((fill_zero_kernel<float>), dim3(static_cast<unsigned>(nb)), dim3(kBlock), 0, s, m, K,
                           static_cast<float *>(C), ld);
    return hipGetLastError();
}

}  // namespace spk
