// sddmm.hip - SDDMM S = A (.) (U V^T) (Section II-A, Eq. (2)) for gfx950.
//
// Only stored entries of A are computed (the dense product is never formed):
// S[p] = a_p * <U[row(p), :], V[col(p), :]>.
//
// A group of LANES lanes works on one row at a time.  Each lane holds an
// NS x VW slice of the row of U in registers; per step the group takes up to
// R entries of the row, reads their column indices with one coalesced load,
// shares them with ds_bpermute, gathers all R slices of V's rows (no
// exec-mask branches: surplus entries re-read a valid row), and forms R
// partial dot products per lane.  The R dot products are then reduced
// together with a transposing butterfly: at each halving step a lane keeps
// half of its values and receives the partner's matching half, so R values
// over R lanes cost R-1 exchanges instead of R log2(R).  Lane q of the group
// ends holding entry q's total.
//
// Three ways to hand rows to groups:
//   MERGE  (default) groups take equal runs of `chunk` entries regardless of
//          rows (binary search for the first row), so power-law rows cost no
//          imbalance;
//   ROWS   group g takes row g;
//   SLAB   one launch per slab of W columns, group g takes the entries of row
//          g in that slab, so the rows of V being gathered stay in L2;
//   TILE   a workgroup owns a block of rows and walks the columns in slabs
//          of V staged in LDS (the SpMM TILE scheme, tile.h).
#include "common.h"
#include "internal.h"
#include "tile.h"

namespace spk {

template <bool OFF32, typename T>
__device__ __forceinline__ const T *row_elem(const T *base, int32_t row, int64_t ld, int32_t col) {
    if constexpr (OFF32)
        return base + (static_cast<uint32_t>(row) * static_cast<uint32_t>(ld) + static_cast<uint32_t>(col));
    else
        return base + (static_cast<int64_t>(row) * ld + col);
}

// Lane exchanges as DPP moves (VALU, no LDS crossbar).  dpp_ctrl values:
// quad_perm [1,0,3,2] = 0xB1 (partner lane ^ 1), quad_perm [2,3,0,1] = 0x4E
// (lane ^ 2), row_half_mirror = 0x141 (7 - lane within 8), row_mirror =
// 0x140 (15 - lane within 16), row_ror:8 = 0x128 (lane ^ 8 within 16).  In
// each of them every lane has a valid source and all lanes are written; with
// bound_ctrl set the move needs no prior value, and the compiler folds a move
// whose only use is an add into that add (v_add_f32_dpp).
template <int CTRL>
__device__ __forceinline__ float dpp(float v) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xF, 0xF, true));
}
template <int CTRL>
__device__ __forceinline__ double dpp(double v) {
    const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, 0xF, 0xF, true);
    const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, 0xF, 0xF, true);
    return __hiloint2double(hi, lo);
}

// Partner value for a halving step of stride H: any lane whose bit H differs
// works, because both partners hold the same entries at that point (mirror
// pairs do for H = 4 and 8).
template <int H, typename T>
__device__ __forceinline__ T halving_partner(T v, int lane) {
    if constexpr (H == 1) return dpp<0xB1>(v);
    else if constexpr (H == 2) return dpp<0x4E>(v);
    else if constexpr (H == 4) return dpp<0x141>(v);
    else if constexpr (H == 8) return dpp<0x140>(v);
    else return lane_read(v, lane ^ H);
}

// Partner holding the same entry, exactly lane ^ S.
template <int S, typename T>
__device__ __forceinline__ T xor_partner(T v, int lane) {
    if constexpr (S == 1) return dpp<0xB1>(v);
    else if constexpr (S == 2) return dpp<0x4E>(v);
    else if constexpr (S == 8) return dpp<0x128>(v);
    else return lane_read(v, lane ^ S);
}

template <int H, int R, typename T>
__device__ __forceinline__ void halving_steps(T (&x)[R], int lane) {
    if constexpr (H >= 1) {
        const bool upper = (lane & H) != 0;
#pragma unroll
        for (int i = 0; i < H; ++i) {
            const T send = upper ? x[i] : x[i + H];
            const T keep = upper ? x[i + H] : x[i];
            x[i] = keep + halving_partner<H>(send, lane);
        }
        halving_steps<H / 2, R>(x, lane);
    }
}

template <int S, int LANES, typename T>
__device__ __forceinline__ T across_subgroups(T v, int lane) {
    if constexpr (S < LANES) return across_subgroups<S * 2, LANES>(v + xor_partner<S>(v, lane), lane);
    else return v;
}

// On return, lane l of each LANES-lane group holds the group-wide total of
// x[l mod R] (R and LANES powers of two, R <= LANES): halving steps leave
// lane l with entry l mod R summed over its R-lane subgroup, then the
// subgroups are added.
template <int R, int LANES, typename T>
__device__ __forceinline__ T reduce_scatter(T (&x)[R], int lane) {
    halving_steps<R / 2, R>(x, lane);
    return across_subgroups<R, LANES>(x[0], lane);
}

template <typename TUV, int VW, int LANES, int NS>
struct URow {
    using A = typename acc_of<TUV>::type;
    A u[NS][VW];
    // Slice s of lane lig covers columns s*LANES*VW + lig*VW .. +VW; slices
    // beyond K are zero (their gathers read column 0 and add nothing).
    __device__ __forceinline__ void load(const TUV *U, int64_t row, int64_t ldu, int K, int lig) {
#pragma unroll
        for (int s = 0; s < NS; ++s) {
            const int k = s * LANES * VW + lig * VW;
            if (k < K) vec_load<TUV, VW>::run(U + row * ldu + k, u[s]);
            else
#pragma unroll
                for (int e = 0; e < VW; ++e) u[s][e] = A(0);
        }
    }
};

// One step: entries pb .. pb+cnt-1 (1 <= cnt <= R) of one row.  load()
// issues the column-index read, the lane exchanges and all R x NS gathers;
// dots() forms the R partial dot products with the row of U; finish()
// reduces them across the group and stores.  Callers issue the next step's
// load() between dots() and finish(), so its gathers are in flight while the
// current step reduces.
template <typename TUV, int VW, int LANES, int NS, int R, bool OFF32>
struct Step {
    using A = typename acc_of<TUV>::type;
    int64_t pb;
    int cnt;
    A vrow[R][NS][VW];

    // Column of entry p: cbase + ci[p] (CT = uint16_t: the slab form's offsets).
    template <typename CT>
    __device__ __forceinline__ void load(int64_t pb_, int cnt_, const CT *__restrict__ ci,
                                         const TUV *__restrict__ V, int64_t ldv, int K, int gbase, int lig,
                                         int32_t cbase = 0) {
        pb = pb_;
        cnt = cnt_;
        const int mine = lig < cnt ? lig : cnt - 1;
        const int c_mine = cbase + static_cast<int>(__builtin_nontemporal_load(ci + pb + mine));
        int cc[R];
#pragma unroll
        for (int q = 0; q < R; ++q) cc[q] = lane_read(c_mine, gbase + q);
#pragma unroll
        for (int q = 0; q < R; ++q)
#pragma unroll
            for (int s = 0; s < NS; ++s) {
                const int k = s * LANES * VW + lig * VW;
                vec_load<TUV, VW>::run(row_elem<OFF32>(V, cc[q], ldv, k < K ? k : 0), vrow[q][s]);
            }
    }

    __device__ __forceinline__ void dots(const URow<TUV, VW, LANES, NS> &ur, A (&part)[R]) const {
#pragma unroll
        for (int q = 0; q < R; ++q) {
            A acc = A(0);
#pragma unroll
            for (int s = 0; s < NS; ++s)
#pragma unroll
                for (int e = 0; e < VW; ++e) acc = fma(ur.u[s][e], vrow[q][s][e], acc);
            part[q] = acc;
        }
    }
};

template <int R, int LANES, typename A, typename TV>
__device__ __forceinline__ void finish(int64_t pb, int cnt, A (&part)[R], const TV *__restrict__ vals,
                                       A *__restrict__ S, int lig, int lane) {
    const A tot = reduce_scatter<R, LANES>(part, lane);
    if (lig < cnt && lig < R) {
        const int64_t p = pb + lig;
        const A a = vals ? static_cast<A>(__builtin_nontemporal_load(vals + p)) : A(1);
        S[p] = a * tot;  // cached store: a group writes R consecutive outputs per step
    }
}

// MERGE: group g takes entries [g*chunk, (g+1)*chunk).
template <typename TUV, typename TV, int VW, int LANES, int NS, bool OFF32>
__global__ __launch_bounds__(kBlock) void sddmm_split_kernel(int64_t m, int64_t nnz, int K, const int32_t *__restrict__ rp,
                                                             const int32_t *__restrict__ ci,
                                                             const TV *__restrict__ vals,
                                                             const TUV *__restrict__ U, int64_t ldu,
                                                             const TUV *__restrict__ V, int64_t ldv,
                                                             typename acc_of<TUV>::type *__restrict__ S,
                                                             int64_t chunk, int64_t ngroups) {
    constexpr int GPB = kBlock / LANES;
    constexpr int R = LANES < 8 ? LANES : 8;
    const int lane = threadIdx.x & (kWave - 1);
    const int lig = threadIdx.x & (LANES - 1);
    const int gbase = lane & ~(LANES - 1);
    const int64_t blk = xcd_block(blockIdx.x, gridDim.x);
    const int64_t g = blk * GPB + threadIdx.x / LANES;
    if (g >= ngroups) return;
    const int64_t p0 = g * chunk;
    const int64_t p1 = p0 + chunk < nnz ? p0 + chunk : nnz;
    // Row holding entry p0: largest r in [0, m-1] with row_ptr[r] <= p0.
    int64_t r = last_at_most(0, m - 1, p0, [&](int64_t i) { return static_cast<int64_t>(rp[i]); });
    int64_t next = rp[r + 1];
    int64_t pb = p0;
    // the step starting at pb never crosses a row end, so one row of U serves it
    auto step_len = [&]() {
        while (pb >= next) {  // group-uniform; also skips empty rows
            ++r;
            next = rp[r + 1];
        }
        const int64_t lim = p1 < next ? p1 : next;
        return static_cast<int>(lim - pb < R ? lim - pb : R);
    };
    URow<TUV, VW, LANES, NS> ur;
    Step<TUV, VW, LANES, NS, R, OFF32> st;
    int cnt = step_len();
    ur.load(U, r, ldu, K, lig);
    int64_t loaded = r;
    st.load(pb, cnt, ci, V, ldv, K, gbase, lig);
    while (true) {
        typename acc_of<TUV>::type part[R];
        st.dots(ur, part);
        const int64_t pb_cur = st.pb;
        const int cnt_cur = st.cnt;
        pb = pb_cur + cnt_cur;
        const bool more = pb < p1;
        if (more) {  // next step's gathers go out before this step's reduction
            cnt = step_len();
            if (r != loaded) {
                ur.load(U, r, ldu, K, lig);
                loaded = r;
            }
            st.load(pb, cnt, ci, V, ldv, K, gbase, lig);
        }
        finish<R, LANES>(pb_cur, cnt_cur, part, vals, S, lig, lane);
        if (!more) break;
    }
}

// ROWS / SLAB: group g takes the entries of row g in slab s
// ([bnd(s, g), bnd(s+1, g)) with bnd(0, .) = row_ptr, bnd(nslabs, .) = row_ptr[+1]).
template <typename TUV, typename TV, int VW, int LANES, int NS, bool OFF32>
__global__ __launch_bounds__(kBlock) void sddmm_rows_kernel(int64_t m, int K, const int32_t *__restrict__ rp,
                                                            const int32_t *__restrict__ bnd, int nslabs, int s,
                                                            const int32_t *__restrict__ ci,
                                                            const TV *__restrict__ vals,
                                                            const TUV *__restrict__ U, int64_t ldu,
                                                            const TUV *__restrict__ V, int64_t ldv,
                                                            typename acc_of<TUV>::type *__restrict__ S) {
    constexpr int GPB = kBlock / LANES;
    constexpr int R = LANES < 8 ? LANES : 8;
    const int lane = threadIdx.x & (kWave - 1);
    const int lig = threadIdx.x & (LANES - 1);
    const int gbase = lane & ~(LANES - 1);
    const int64_t blk = xcd_block(blockIdx.x, gridDim.x);
    const int64_t row = blk * GPB + threadIdx.x / LANES;
    if (row >= m) return;
    const int64_t a = s == 0 ? rp[row] : bnd[(s - 1) * m + row];
    const int64_t b = s == nslabs - 1 ? rp[row + 1] : bnd[s * m + row];
    if (a >= b) return;
    URow<TUV, VW, LANES, NS> ur;
    ur.load(U, row, ldu, K, lig);
    Step<TUV, VW, LANES, NS, R, OFF32> st;
    st.load(a, static_cast<int>(b - a < R ? b - a : R), ci, V, ldv, K, gbase, lig);
    while (true) {
        typename acc_of<TUV>::type part[R];
        st.dots(ur, part);
        const int64_t pb_cur = st.pb;
        const int cnt_cur = st.cnt;
        const int64_t pb = pb_cur + cnt_cur;
        const bool more = pb < b;
        if (more) st.load(pb, static_cast<int>(b - pb < R ? b - pb : R), ci, V, ldv, K, gbase, lig);
        finish<R, LANES>(pb_cur, cnt_cur, part, vals, S, lig, lane);
        if (!more) break;
    }
}

// DCSR: group g takes row order[g] of the non-empty rows (g < nrows).
template <typename TUV, typename TV, int VW, int LANES, int NS, bool OFF32>
__global__ __launch_bounds__(kBlock) void sddmm_dcsr_kernel(int64_t nrows, int K, const int32_t *__restrict__ order,
                                                            const int32_t *__restrict__ rp,
                                                            const int32_t *__restrict__ ci,
                                                            const TV *__restrict__ vals,
                                                            const TUV *__restrict__ U, int64_t ldu,
                                                            const TUV *__restrict__ V, int64_t ldv,
                                                            typename acc_of<TUV>::type *__restrict__ S) {
    constexpr int GPB = kBlock / LANES;
    constexpr int R = LANES < 8 ? LANES : 8;
    const int lane = threadIdx.x & (kWave - 1);
    const int lig = threadIdx.x & (LANES - 1);
    const int gbase = lane & ~(LANES - 1);
    const int64_t blk = xcd_block(blockIdx.x, gridDim.x);
    const int64_t g = blk * GPB + threadIdx.x / LANES;
    if (g >= nrows) return;
    const int64_t row = order[g];
    const int64_t a = rp[row], b = rp[row + 1];
    URow<TUV, VW, LANES, NS> ur;
    ur.load(U, row, ldu, K, lig);
    Step<TUV, VW, LANES, NS, R, OFF32> st;
    st.load(a, static_cast<int>(b - a < R ? b - a : R), ci, V, ldv, K, gbase, lig);
    while (true) {
        typename acc_of<TUV>::type part[R];
        st.dots(ur, part);
        const int64_t pb_cur = st.pb;
        const int cnt_cur = st.cnt;
        const int64_t pb = pb_cur + cnt_cur;
        const bool more = pb < b;
        if (more) st.load(pb, static_cast<int>(b - pb < R ? b - pb : R), ci, V, ldv, K, gbase, lig);
        finish<R, LANES>(pb_cur, cnt_cur, part, vals, S, lig, lane);
        if (!more) break;
    }
}

// COO: group g takes entries [g*chunk, (g+1)*chunk), R at a time, whatever
// their rows: each entry's row comes from rowidx and its slice of U is
// gathered like V's (consecutive entries of a row hit the same cached row).
template <typename TUV, typename TV, int VW, int LANES, int NS, bool OFF32>
__global__ __launch_bounds__(kBlock) void sddmm_coo_kernel(int64_t nnz, int K, const int32_t *__restrict__ rowidx,
                                                           const int32_t *__restrict__ ci,
                                                           const TV *__restrict__ vals,
                                                           const TUV *__restrict__ U, int64_t ldu,
                                                           const TUV *__restrict__ V, int64_t ldv,
                                                           typename acc_of<TUV>::type *__restrict__ S, int64_t chunk,
                                                           int64_t ngroups) {
    using A = typename acc_of<TUV>::type;
    constexpr int GPB = kBlock / LANES;
    constexpr int R = LANES < 8 ? LANES : 8;
    const int lane = threadIdx.x & (kWave - 1);
    const int lig = threadIdx.x & (LANES - 1);
    const int gbase = lane & ~(LANES - 1);
    const int64_t blk = xcd_block(blockIdx.x, gridDim.x);
    const int64_t g = blk * GPB + threadIdx.x / LANES;
    if (g >= ngroups) return;
    const int64_t p0 = g * chunk;
    const int64_t p1 = p0 + chunk < nnz ? p0 + chunk : nnz;
    for (int64_t pb = p0; pb < p1; pb += R) {
        const int cnt = static_cast<int>(p1 - pb < R ? p1 - pb : R);
        const int mine = lig < cnt ? lig : cnt - 1;
        const int r_mine = __builtin_nontemporal_load(rowidx + pb + mine);
        const int c_mine = __builtin_nontemporal_load(ci + pb + mine);
        A part[R];
#pragma unroll
        for (int q = 0; q < R; ++q) {
            const int rq = lane_read(r_mine, gbase + q), cq = lane_read(c_mine, gbase + q);
            A acc = A(0);
#pragma unroll
            for (int sl = 0; sl < NS; ++sl) {
                const int k = sl * LANES * VW + lig * VW;
                const int kk = k < K ? k : 0;
                A uu[VW], vv[VW];
                vec_load<TUV, VW>::run(U + static_cast<int64_t>(rq) * ldu + kk, uu);
                vec_load<TUV, VW>::run(row_elem<OFF32>(V, cq, ldv, kk), vv);
                if (k < K)
#pragma unroll
                    for (int e = 0; e < VW; ++e) acc = fma(uu[e], vv[e], acc);
            }
            part[q] = acc;
        }
        finish<R, LANES>(pb, cnt, part, vals, S, lig, lane);
    }
}

// SLAB16: group g of a block takes run (s, row) of the column-slab form
// (slab16.hip): its entries are positions [seg[s m + row], seg[s m + row + 1])
// of col16 (columns s W + col16), and entry k sits at A position
// apos[s m + row] + k, where its value is read and its output written (the
// runs of a row cover its entries once, so every output is written by one
// group).  One launch covers every (slab, row block) item in slab-major
// order (or several launches of whole slabs, each from item blk0, where the
// items pass a grid's work-item count), renumbered so that each XCD takes a
// contiguous range of it: an XCD works through one slab (or part of one) at a
// time, and the rows of V it gathers come from that slab alone, which its own
// 4 MiB L2 holds when the slab fits (2 MiB: 4096 columns of 512-byte rows).
// Outputs are per entry, so items running at once on different XCDs never
// share one.
template <typename TUV, typename TV, int VW, int LANES, int NS, bool OFF32>
__global__ __launch_bounds__(kBlock) void sddmm_s16_kernel(int64_t m, int K, const int32_t *__restrict__ seg,
                                                           const int32_t *__restrict__ apos,
                                                           const uint16_t *__restrict__ col16, int64_t nbr,
                                                           int64_t blk0, int32_t width, const TV *__restrict__ vals,
                                                           const TUV *__restrict__ U, int64_t ldu,
                                                           const TUV *__restrict__ V, int64_t ldv,
                                                           typename acc_of<TUV>::type *__restrict__ S) {
    constexpr int GPB = kBlock / LANES;
    constexpr int R = LANES < 8 ? LANES : 8;
    const int lane = threadIdx.x & (kWave - 1);
    const int lig = threadIdx.x & (LANES - 1);
    const int gbase = lane & ~(LANES - 1);
    const int64_t blk = blk0 + xcd_block(blockIdx.x, gridDim.x);
    const int64_t s = blk / nbr;
    const int64_t row = (blk - s * nbr) * GPB + threadIdx.x / LANES;
    if (row >= m) return;
    const int32_t cbase = static_cast<int32_t>(s * width);
    const int64_t run = s * m + row;
    const int64_t a = seg[run], b = seg[run + 1];
    if (a >= b) return;
    const int64_t voff = static_cast<int64_t>(apos[run]) - a;
    URow<TUV, VW, LANES, NS> ur;
    ur.load(U, row, ldu, K, lig);
    Step<TUV, VW, LANES, NS, R, OFF32> st;
    st.load(a, static_cast<int>(b - a < R ? b - a : R), col16, V, ldv, K, gbase, lig, cbase);
    while (true) {
        typename acc_of<TUV>::type part[R];
        st.dots(ur, part);
        const int64_t pb_cur = st.pb;
        const int cnt_cur = st.cnt;
        const int64_t pb = pb_cur + cnt_cur;
        const bool more = pb < b;
        if (more) st.load(pb, static_cast<int>(b - pb < R ? b - pb : R), col16, V, ldv, K, gbase, lig, cbase);
        finish<R, LANES>(pb_cur + voff, cnt_cur, part, vals, S, lig, lane);
        if (!more) break;
    }
}

// ------------------------------------------------------------------ TILE
// A workgroup owns GPB*RPG consecutive rows (RPG per group of LANES >= 16
// lanes) and walks the columns in slabs of W rows of V, each copied once to
// LDS (double-buffered, the copy of the next slab in flight during the
// current one).  A group keeps its rows' slices of U in registers and reads
// each row's entries in chunks of 16 (every 16-lane row of the group holds
// the same chunk); the in-slab prefix of a chunk is processed four entries at
// a time: the four rows of V come from LDS, each lane forms four partial dot
// products, and one transposing reduction over the group sums all four.

// Sum over a 16-lane row of four partial dot products: on return lane l holds
// entry (l mod 4)'s total.  Two halving steps (partners lane ^ 2, lane ^ 1)
// leave each lane with one entry summed over its 4-lane subgroup; the four
// subgroups then hold the same entries in the same lane order and are added
// with rotations of the row by 4 and 8 lanes (row_ror:4 = 0x124, row_ror:8 =
// 0x128).
__device__ __forceinline__ float reduce4_row(float (&x)[4], int lane) {
    halving_steps<2, 4>(x, lane);
    float t = x[0];
    t += dpp<0x124>(t);
    t += dpp<0x128>(t);
    return t;
}

// Entries N .. N+3 of the chunk (valid while N < cnt): S[cur + N + j] for
// j = 0..3, written by lane j of the group (the reduction leaves entry j's
// total on lane j).
template <typename TUV, int VW, int LANES, int N>
__device__ __forceinline__ void sddmm_quad(const unsigned char *__restrict__ smem, uint32_t base, int offb, float w,
                                           const float (&u)[VW], int32_t cur, int cnt, float *__restrict__ S,
                                           int lig, int lane) {
    const uint32_t ad[4] = {row_bcast_add<N>(offb, base), row_bcast_add<N + 1>(offb, base),
                            row_bcast_add<N + 2>(offb, base), row_bcast_add<N + 3>(offb, base)};
    float vv[4][VW];
#pragma unroll
    for (int q = 0; q < 4; ++q) vec_load<TUV, VW>::run(reinterpret_cast<const TUV *>(smem + ad[q]), vv[q]);
    float part[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        float acc = 0.f;
#pragma unroll
        for (int e = 0; e < VW; ++e) acc = fma(u[e], vv[q][e], acc);
        part[q] = acc;
    }
    float tot = reduce4_row(part, lane);
    if constexpr (LANES >= 32) tot += lane_read(tot, lane ^ 16);
    if constexpr (LANES >= 64) tot += lane_read(tot, lane ^ 32);
    // lane j < 4 stores entry N + j, whose weight sits on lane N + j of the
    // row: row_shl:N (DPP 0x100 + N) moves it to lane j
    float a = w;
    if constexpr (N > 0) a = __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(w), 0x100 + N, 0xF, 0xF, true));
    if (lig < 4 && N + lig < cnt) S[static_cast<uint32_t>(cur + N + lig)] = a * tot;
}

template <typename TUV, typename TV, int VW, int LANES>
__device__ __forceinline__ int sddmm_tile_pass(const TUV *__restrict__ buf, int K, int koff, int32_t c0, int32_t c1,
                                               int lig, int lane, int gbase16, bool has_vals,
                                               const int32_t *__restrict__ ci, const TV *__restrict__ vsrc,
                                               int32_t last, int32_t &cur, int32_t end, int &c, TV &v,
                                               const float (&u)[VW], float *__restrict__ S) {
    const int r16 = lig & 15;
    const bool in = cur + r16 < end && c < c1;
    const int cnt = count16(__ballot(in), gbase16);
    const int offb = in ? (c - c0) * K * static_cast<int>(sizeof(TUV)) : 0;  // row offset in the slab, bytes
    const float w = in ? (has_vals ? static_cast<float>(v) : 1.f) : 0.f;
    // the next chunk's fetch goes out before the gathers (off and w hold what
    // they need of this one); a chunk with nothing in the slab is fetched again
    const int32_t p0 = cur;
    cur += cnt;
    tile_fetch(cur + r16, last, ci, vsrc, c, v);
    // LDS byte address of a gather: the buffer plus this lane's K offset plus
    // the broadcast row offset
    const unsigned char *smem = reinterpret_cast<const unsigned char *>(buf);
    const uint32_t base = static_cast<uint32_t>(koff * sizeof(TUV));
    if (cnt > 0) sddmm_quad<TUV, VW, LANES, 0>(smem, base, offb, w, u, p0, cnt, S, lig, lane);
    if (cnt > 4) sddmm_quad<TUV, VW, LANES, 4>(smem, base, offb, w, u, p0, cnt, S, lig, lane);
    if (cnt > 8) sddmm_quad<TUV, VW, LANES, 8>(smem, base, offb, w, u, p0, cnt, S, lig, lane);
    if (cnt > 12) sddmm_quad<TUV, VW, LANES, 12>(smem, base, offb, w, u, p0, cnt, S, lig, lane);
    return cnt;
}

template <typename TUV, typename TV, int VW, int LANES, int RPG, int NPT>
__global__ __launch_bounds__(kBlock) void sddmm_tile_kernel(int64_t m, int64_t n, int64_t nnz, int K,
                                                            const int32_t *__restrict__ rp,
                                                            const int32_t *__restrict__ ci,
                                                            const TV *__restrict__ vals,
                                                            const TUV *__restrict__ U, int64_t ldu,
                                                            const TUV *__restrict__ V, int64_t ldv,
                                                            float *__restrict__ S, int W) {
    static_assert(LANES >= 16 && sizeof(TV) == 4, "16-lane rows, F32 values");
    extern __shared__ __align__(16) unsigned char smem[];
    TUV *Vs = reinterpret_cast<TUV *>(smem);  // two buffers of NPT * 4 KiB
    constexpr int buf_elems = NPT * kTilePiece / static_cast<int>(sizeof(TUV));
    constexpr int GPB = kBlock / LANES;
    const int lane = threadIdx.x & (kWave - 1);
    const int lig = threadIdx.x & (LANES - 1);
    const int gbase = lane & ~(LANES - 1);
    const int64_t blk = xcd_block(blockIdx.x, gridDim.x);
    const int64_t row0 = (blk * GPB + threadIdx.x / LANES) * RPG;
    const int k0 = lig * VW;
    const bool kvalid = k0 < K;
    const int koff = kvalid ? k0 : 0;
    const int32_t last = static_cast<int32_t>(nnz - 1);  // row_ptr is int32: positions fit
    const bool has_vals = vals != nullptr;
    const TV *vsrc = has_vals ? vals : reinterpret_cast<const TV *>(ci);
    const int per_row = K / kTileSV<TUV>;  // K is a multiple of the 16-byte width
    int32_t cur[RPG], end[RPG];
    float u[RPG][VW];
#pragma unroll
    for (int r = 0; r < RPG; ++r) {
        const int64_t row = row0 + r;
        cur[r] = row < m ? rp[row] : 0;
        end[r] = row < m ? rp[row + 1] : 0;
        if (row < m && kvalid) vec_load<TUV, VW>::run(U + row * ldu + k0, u[r]);
        else
#pragma unroll
            for (int e = 0; e < VW; ++e) u[r][e] = 0.f;  // lanes past K add nothing
    }
    u32x4 stg[NPT];
    TileCopy<TUV, NPT> copy;
    copy.layout(static_cast<int>(n < W ? n : W), per_row, ldv);
    copy.load(V, ldv, 0, stg);
    tile_store<TUV, NPT>(Vs, stg);
    int pc[RPG];
    TV pv[RPG];
#pragma unroll
    for (int r = 0; r < RPG; ++r) tile_fetch(cur[r] + (lig & 15), last, ci, vsrc, pc[r], pv[r]);
    int sl = 0;
    for (int32_t c0 = 0; c0 < n; c0 += W, ++sl) {
        const int32_t c1 = static_cast<int32_t>(n - c0 < W ? n : c0 + W);
        __syncthreads();  // slab sl is in LDS; every group is done with the other buffer
        const int32_t nx = c1 < n ? c1 : c0;  // the last slab reads itself again: same loads every slab
        if (n - nx < W) copy.layout(static_cast<int>(n - nx), per_row, ldv);  // a narrower last slab
        copy.load(V, ldv, nx, stg);
        const TUV *buf = Vs + (sl & 1) * buf_elems;
#pragma unroll
        for (int r = 0; r < RPG; ++r) {
            // only a chunk wholly inside the slab needs the fresh chunk at once
            if (sddmm_tile_pass<TUV, TV, VW, LANES>(buf, K, koff, c0, c1, lig, lane, gbase, has_vals, ci, vsrc, last,
                                                    cur[r], end[r], pc[r], pv[r], u[r], S) == 16) {
                while (sddmm_tile_pass<TUV, TV, VW, LANES>(buf, K, koff, c0, c1, lig, lane, gbase, has_vals, ci,
                                                           vsrc, last, cur[r], end[r], pc[r], pv[r], u[r], S) == 16) {
                }
            }
        }
        tile_store<TUV, NPT>(Vs + ((sl + 1) & 1) * buf_elems, stg);
    }
}

// TILE with one entry per 4-lane quad.  The same slabs and chunks, another
// split of the work inside a 16-lane group: its four quads take four entries
// at once and each lane covers a quarter of the row (NP pieces of 16 bytes),
// so a dot product is summed with two quad exchanges instead of the
// transposing reduction over the group, at the price of four copies of the
// rows of U per group.  A chunk is fetched so that lane 4q + j holds entry
// 4j + q: in step s quad q works on entry 4s + q, whose row offset sits on
// lane 4q + s of the same quad (a quad_perm broadcast, DPP 0x55 * s), and the
// total of entry 4j + q ends on the lane that fetched it, which stores it
// with its own weight.  In read i of a step quad q reads the 64-byte group
// quad_group(i, q) of its row, piece j of it, so the four quads of a group
// read different bank groups although their rows are unrelated.
// Partial dot product of two 16-byte pieces of a row: four FMAs on F32, four
// two-element dot products (v_dot2c_f32_bf16: exact products, F32 sums) on
// BF16, so the BF16 rows need no unpacking.
template <typename TUV>
__device__ __forceinline__ float dot_piece(const u32x4 &a, const u32x4 &b, float acc);
template <>
__device__ __forceinline__ float dot_piece<float>(const u32x4 &a, const u32x4 &b, float acc) {
    acc = fma(__uint_as_float(a.x), __uint_as_float(b.x), acc);
    acc = fma(__uint_as_float(a.y), __uint_as_float(b.y), acc);
    acc = fma(__uint_as_float(a.z), __uint_as_float(b.z), acc);
    return fma(__uint_as_float(a.w), __uint_as_float(b.w), acc);
}
typedef __bf16 bf16x2_t __attribute__((ext_vector_type(2)));
__device__ __forceinline__ float dot2_bf16(uint32_t a, uint32_t b, float acc) {
    return __builtin_amdgcn_fdot2_f32_bf16(__builtin_bit_cast(bf16x2_t, a), __builtin_bit_cast(bf16x2_t, b), acc,
                                           false);
}
template <>
__device__ __forceinline__ float dot_piece<bf16>(const u32x4 &a, const u32x4 &b, float acc) {
    acc = dot2_bf16(a.x, b.x, acc);
    acc = dot2_bf16(a.y, b.y, acc);
    acc = dot2_bf16(a.z, b.z, acc);
    return dot2_bf16(a.w, b.w, acc);
}

template <typename TUV, int NP, int S>
__device__ __forceinline__ float sddmm_qstep(const unsigned char *__restrict__ smem, const uint32_t (&pb)[NP],
                                             int offb, const u32x4 (&u)[NP]) {
    u32x4 vv[NP];
#pragma unroll
    for (int i = 0; i < NP; ++i) vv[i] = *reinterpret_cast<const u32x4 *>(smem + quad_bcast_add<S>(offb, pb[i]));
    float acc = 0.f;
#pragma unroll
    for (int i = 0; i < NP; ++i) acc = dot_piece<TUV>(u[i], vv[i], acc);
    acc += dpp<0xB1>(acc);
    return acc + dpp<0x4E>(acc);
}

template <typename TUV, typename TV, int NP>
__device__ __forceinline__ int sddmm_tileq_pass(const unsigned char *__restrict__ smem, int32_t c0, int32_t c1,
                                                int slot, int j, int gbase16, bool has_vals,
                                                const int32_t *__restrict__ ci, const TV *__restrict__ vsrc,
                                                int32_t last, int32_t &cur, int32_t end, int &c, TV &v,
                                                const uint32_t (&pb)[NP], const u32x4 (&u)[NP],
                                                float *__restrict__ S) {
    constexpr int kRowShift = NP == 2 ? 7 : NP == 4 ? 8 : 9;  // log2 of a row's bytes
    const bool in = cur + slot < end && c < c1;
    const int cnt = count16(__builtin_amdgcn_ballot_w64(in), gbase16);
    const int offb = in ? (c - c0) << kRowShift : 0;
    const float w = pin(has_vals ? static_cast<float>(v) : 1.f);
    const int32_t p = cur + slot;
    cur += cnt;
    tile_fetch(cur + slot, last, ci, vsrc, c, v);
    float res = 0.f;
    if (cnt > 0) {
        const float t = sddmm_qstep<TUV, NP, 0>(smem, pb, offb, u);
        res = j == 0 ? t : res;
    }
    if (cnt > 4) {
        const float t = sddmm_qstep<TUV, NP, 1>(smem, pb, offb, u);
        res = j == 1 ? t : res;
    }
    if (cnt > 8) {
        const float t = sddmm_qstep<TUV, NP, 2>(smem, pb, offb, u);
        res = j == 2 ? t : res;
    }
    if (cnt > 12) {
        const float t = sddmm_qstep<TUV, NP, 3>(smem, pb, offb, u);
        res = j == 3 ? t : res;
    }
    if (in) S[static_cast<uint32_t>(p)] = w * res;
    return cnt;
}

template <typename TUV, typename TV, int NP, int RPG, int NPT, int BS>
__global__ __launch_bounds__(BS, BS > kBlock ? 4 : 1) void sddmm_tileq_kernel(int64_t m, int64_t n, int64_t nnz,
                                                             const int32_t *__restrict__ rp,
                                                             const int32_t *__restrict__ ci,
                                                             const TV *__restrict__ vals,
                                                             const TUV *__restrict__ U, int64_t ldu,
                                                             const TUV *__restrict__ V, int64_t ldv,
                                                             float *__restrict__ S, int W) {
    constexpr int SV = kTileSV<TUV>;
    constexpr int per_row = 4 * NP;  // 16-byte pieces in a row of U or V
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
    u32x4 u[RPG][NP];  // this lane's pieces of the rows of U, as stored
#pragma unroll
    for (int r = 0; r < RPG; ++r) {
        const int64_t row = row0 + r;
        cur[r] = row < m ? rp[row] : 0;
        end[r] = row < m ? rp[row + 1] : 0;
#pragma unroll
        for (int i = 0; i < NP; ++i)
            u[r][i] = row < m ? *reinterpret_cast<const u32x4 *>(U + row * ldu + (pb[i] / 16) * SV) : u32x4{0, 0, 0, 0};
    }
    u32x4 stg[NPT];
    TileCopy<TUV, NPT, BS> copy;
    copy.layout(static_cast<int>(n < W ? n : W), per_row, ldv);
    copy.load(V, ldv, 0, stg);
    tile_store<TUV, NPT, BS>(reinterpret_cast<TUV *>(smem), stg);
    int pc[RPG];
    TV pv[RPG];
#pragma unroll
    for (int r = 0; r < RPG; ++r) tile_fetch(cur[r] + slot, last, ci, vsrc, pc[r], pv[r]);
    int sl = 0;
    for (int32_t c0 = 0; c0 < n; c0 += W, ++sl) {
        const int32_t c1 = static_cast<int32_t>(n - c0 < W ? n : c0 + W);
        __syncthreads();  // slab sl is in LDS; every group is done with the other buffer
        const int32_t nx = c1 < n ? c1 : c0;  // the last slab reads itself again: same loads every slab
        if (n - nx < W) copy.layout(static_cast<int>(n - nx), per_row, ldv);
        copy.load(V, ldv, nx, stg);
        const unsigned char *buf = smem + (sl & 1) * buf_bytes;
#pragma unroll
        for (int r = 0; r < RPG; ++r) {
            if (sddmm_tileq_pass<TUV, TV, NP>(buf, c0, c1, slot, j, gbase, has_vals, ci, vsrc, last, cur[r],
                                                   end[r], pc[r], pv[r], pb, u[r], S) == 16) {
                while (sddmm_tileq_pass<TUV, TV, NP>(buf, c0, c1, slot, j, gbase, has_vals, ci, vsrc, last,
                                                          cur[r], end[r], pc[r], pv[r], pb, u[r], S) == 16) {
                }
            }
        }
        tile_store<TUV, NPT, BS>(reinterpret_cast<TUV *>(smem + ((sl + 1) & 1) * buf_bytes), stg);
    }
}

template <typename TUV, typename TV, int NP, int RPG, int NPT, int BS>
static hipError_t launch_tileq_npt(const SddmmArgs &a, hipStream_t s) {
    constexpr int GPB = BS / 16;
    const int64_t nb = (a.m + GPB * RPG - 1) / (GPB * RPG);
    const size_t lds = 2 * static_cast<size_t>(NPT) * BS * 16;  // two slab buffers
    if (lds > 65536) {  // beyond the default dynamic LDS limit (gfx950 has 160 KiB per CU)
        const hipError_t e = hipFuncSetAttribute(
            reinterpret_cast<const void *>(&sddmm_tileq_kernel<TUV, TV, NP, RPG, NPT, BS>),
            hipFuncAttributeMaxDynamicSharedMemorySize, static_cast<int>(lds));
        if (e != hipSuccess) return e;
    }
    hipLaunchKernelGGL((sddmm_tileq_kernel<TUV, TV, NP, RPG, NPT, BS>), dim3(static_cast<unsigned>(nb)), dim3(BS),
                       lds, s, a.m, a.n, a.nnz, a.rp, a.ci, static_cast<const TV *>(a.vals),
                       static_cast<const TUV *>(a.U), a.ldu, static_cast<const TUV *>(a.V), a.ldv,
                       static_cast<float *>(a.S), static_cast<int>(a.chunk));
    return hipGetLastError();
}

template <typename TUV, typename TV, int NP, int RPG, int BS = kBlock>
static hipError_t launch_tileq_rpg(const SddmmArgs &a, hipStream_t s) {
    constexpr int GPB = BS / 16;
    constexpr int64_t round = BS * 16;
    const int64_t nb = (a.m + GPB * RPG - 1) / (GPB * RPG);
    const int64_t slab_bytes = a.chunk * a.K * static_cast<int64_t>(sizeof(TUV));
    if (!grid_fits(nb, BS)) return kGridTooLarge;
    if (a.K * static_cast<int64_t>(sizeof(TUV)) != 64 * NP || a.chunk < 1 ||
        2 * slab_bytes > (BS == 1024 ? 2 : 1) * static_cast<int64_t>(kTileLds) || a.n > 0x7FFFFFFF)
        return hipErrorInvalidValue;
    if (slab_bytes <= 2 * round) return launch_tileq_npt<TUV, TV, NP, RPG, 2, BS>(a, s);
    if (slab_bytes <= 4 * round) return launch_tileq_npt<TUV, TV, NP, RPG, 4, BS>(a, s);
    if constexpr (BS == kBlock) return launch_tileq_npt<TUV, TV, NP, RPG, 8, BS>(a, s);
    return hipErrorInvalidValue;
}

template <typename TUV, typename TV>
static hipError_t launch_tileq(const SddmmArgs &a, hipStream_t s) {
    const bool r8 = a.rows_per_group == 8;
    if (a.rows_per_group == 2) {
        // wide plans: 512 threads with two rows per group for slabs up to
        // 32 KiB, else 1024 threads with one row per group
        const bool big = a.chunk * a.K * static_cast<int64_t>(sizeof(TUV)) > kTileLds / 2;
        switch (a.K * static_cast<int64_t>(sizeof(TUV))) {
        case 128: return big ? launch_tileq_rpg<TUV, TV, 2, 1, 1024>(a, s) : launch_tileq_rpg<TUV, TV, 2, 2, 512>(a, s);
        case 256: return big ? launch_tileq_rpg<TUV, TV, 4, 1, 1024>(a, s) : launch_tileq_rpg<TUV, TV, 4, 2, 512>(a, s);
        case 512: return launch_tileq_rpg<TUV, TV, 8, 1, 1024>(a, s);  // 1024 threads, one row per group
        default: return hipErrorInvalidValue;
        }
    }
    switch (a.K * static_cast<int64_t>(sizeof(TUV))) {
    case 128: return r8 ? launch_tileq_rpg<TUV, TV, 2, 8>(a, s) : launch_tileq_rpg<TUV, TV, 2, 4>(a, s);
    case 256: return r8 ? launch_tileq_rpg<TUV, TV, 4, 8>(a, s) : launch_tileq_rpg<TUV, TV, 4, 4>(a, s);
    case 512: return launch_tileq_rpg<TUV, TV, 8, 4>(a, s);  // 32 registers of U per row: 4 rows per group
    default: return hipErrorInvalidValue;
    }
}

template <typename TUV, typename TV, int LANES, int RPG, int NPT>
static hipError_t launch_tile_npt(const SddmmArgs &a, hipStream_t s) {
    constexpr int GPB = kBlock / LANES;
    const int64_t nb = (a.m + GPB * RPG - 1) / (GPB * RPG);
    const size_t lds = 2 * static_cast<size_t>(NPT) * kTilePiece;  // two slab buffers
    hipLaunchKernelGGL((sddmm_tile_kernel<TUV, TV, 4, LANES, RPG, NPT>), dim3(static_cast<unsigned>(nb)), dim3(kBlock),
                       lds, s, a.m, a.n, a.nnz, static_cast<int>(a.K), a.rp, a.ci, static_cast<const TV *>(a.vals),
                       static_cast<const TUV *>(a.U), a.ldu, static_cast<const TUV *>(a.V), a.ldv,
                       static_cast<float *>(a.S), static_cast<int>(a.chunk));
    return hipGetLastError();
}

template <typename TUV, typename TV, int LANES, int RPG>
static hipError_t launch_tile_rpg(const SddmmArgs &a, hipStream_t s) {
    constexpr int GPB = kBlock / LANES;
    const int64_t nb = (a.m + GPB * RPG - 1) / (GPB * RPG);
    const int64_t slab_bytes = a.chunk * a.K * static_cast<int64_t>(sizeof(TUV));
    if (!grid_fits(nb, kBlock)) return kGridTooLarge;
    if (a.K > LANES * 4 || a.chunk < 1 || 2 * slab_bytes > kTileLds || a.n > 0x7FFFFFFF)
        return hipErrorInvalidValue;
    if (slab_bytes <= 2 * kTilePiece) return launch_tile_npt<TUV, TV, LANES, RPG, 2>(a, s);
    if (slab_bytes <= 4 * kTilePiece) return launch_tile_npt<TUV, TV, LANES, RPG, 4>(a, s);
    return launch_tile_npt<TUV, TV, LANES, RPG, 8>(a, s);
}

template <typename TUV, typename TV>
static hipError_t launch_tile(const SddmmArgs &a, hipStream_t s) {
    const bool r8 = a.rows_per_group == 8;
    switch (a.lanes) {
    case 16: return r8 ? launch_tile_rpg<TUV, TV, 16, 8>(a, s) : launch_tile_rpg<TUV, TV, 16, 4>(a, s);
    case 32: return r8 ? launch_tile_rpg<TUV, TV, 32, 8>(a, s) : launch_tile_rpg<TUV, TV, 32, 4>(a, s);
    case 64: return r8 ? launch_tile_rpg<TUV, TV, 64, 8>(a, s) : launch_tile_rpg<TUV, TV, 64, 4>(a, s);
    default: return hipErrorInvalidValue;
    }
}

template <typename TUV, typename TV, int VW, int LANES, int NS, bool OFF32>
static hipError_t launch(const SddmmArgs &a, hipStream_t s) {
    constexpr int GPB = kBlock / LANES;
    using A = typename acc_of<TUV>::type;
    if (a.variant == SPK_VAR_MERGE) {
        const int64_t ngroups = (a.nnz + a.chunk - 1) / a.chunk;
        const int64_t nb = (ngroups + GPB - 1) / GPB;
        if (!grid_fits(nb, kBlock)) return kGridTooLarge;
        hipLaunchKernelGGL((sddmm_split_kernel<TUV, TV, VW, LANES, NS, OFF32>), dim3(static_cast<unsigned>(nb)),
                           dim3(kBlock), 0, s, a.m, a.nnz, static_cast<int>(a.K), a.rp, a.ci,
                           static_cast<const TV *>(a.vals), static_cast<const TUV *>(a.U), a.ldu,
                           static_cast<const TUV *>(a.V), a.ldv, static_cast<A *>(a.S), a.chunk, ngroups);
        return hipGetLastError();
    }
    if (a.variant == SPK_VAR_DCSR) {
        if (a.hv.nrows <= 0) return hipSuccess;
        const int64_t nb = (a.hv.nrows + GPB - 1) / GPB;
        if (!grid_fits(nb, kBlock)) return kGridTooLarge;
        if (a.hv.nrows > a.m) return hipErrorInvalidValue;
        hipLaunchKernelGGL((sddmm_dcsr_kernel<TUV, TV, VW, LANES, NS, OFF32>), dim3(static_cast<unsigned>(nb)),
                           dim3(kBlock), 0, s, a.hv.nrows, static_cast<int>(a.K), a.hv.order, a.rp, a.ci,
                           static_cast<const TV *>(a.vals), static_cast<const TUV *>(a.U), a.ldu,
                           static_cast<const TUV *>(a.V), a.ldv, static_cast<A *>(a.S));
        return hipGetLastError();
    }
    if (a.variant == SPK_VAR_COO) {
        const int64_t ngroups = (a.nnz + a.chunk - 1) / a.chunk;
        const int64_t nb = (ngroups + GPB - 1) / GPB;
        if (!grid_fits(nb, kBlock)) return kGridTooLarge;
        hipLaunchKernelGGL((sddmm_coo_kernel<TUV, TV, VW, LANES, NS, OFF32>), dim3(static_cast<unsigned>(nb)),
                           dim3(kBlock), 0, s, a.nnz, static_cast<int>(a.K), a.hv.rowidx, a.ci,
                           static_cast<const TV *>(a.vals), static_cast<const TUV *>(a.U), a.ldu,
                           static_cast<const TUV *>(a.V), a.ldv, static_cast<A *>(a.S), a.chunk, ngroups);
        return hipGetLastError();
    }
    if (a.variant == SPK_VAR_SLAB16) {
        const int64_t nbr = (a.m + GPB - 1) / GPB;  // row blocks per slab
        if (!grid_fits(nbr, kBlock)) return kGridTooLarge;
        if (a.s16.nslabs < 1 || a.s16.width > 65536) return hipErrorInvalidValue;
        // Whole slabs per launch, as many as the grid's work-item count holds.
        const int64_t per = (static_cast<int64_t>(0xFFFFFFFFu) / kBlock / nbr) * nbr;
        const int64_t nb = a.s16.nslabs * nbr;
        for (int64_t b0 = 0; b0 < nb; b0 += per) {
            const int64_t cnt = nb - b0 < per ? nb - b0 : per;
            hipLaunchKernelGGL((sddmm_s16_kernel<TUV, TV, VW, LANES, NS, OFF32>), dim3(static_cast<unsigned>(cnt)),
                               dim3(kBlock), 0, s, a.m, static_cast<int>(a.K), a.s16.seg, a.s16.apos, a.s16.col16,
                               nbr, b0, static_cast<int32_t>(a.s16.width), static_cast<const TV *>(a.vals),
                               static_cast<const TUV *>(a.U), a.ldu, static_cast<const TUV *>(a.V), a.ldv,
                               static_cast<A *>(a.S));
            const hipError_t e = hipGetLastError();
            if (e != hipSuccess) return e;
        }
        return hipSuccess;
    }
    int nslabs = 1;
    int64_t width = a.n > 0 ? a.n : 1;
    int32_t *bnd = static_cast<int32_t *>(a.ws);
    if (a.variant == SPK_VAR_SLAB) {
        const SlabLayout L = slab_layout(a.m, a.n, a.chunk);
        nslabs = static_cast<int>(L.nslabs);
        width = L.width;
    }
    if (nslabs > 1) {
        hipError_t e = slab_bounds_launch(a.m, a.rp, a.ci, width, nslabs, bnd, s);
        if (e != hipSuccess) return e;
    }
    const int64_t nb = (a.m + GPB - 1) / GPB;
    if (!grid_fits(nb, kBlock)) return kGridTooLarge;
    for (int sl = 0; sl < nslabs; ++sl) {
        hipLaunchKernelGGL((sddmm_rows_kernel<TUV, TV, VW, LANES, NS, OFF32>), dim3(static_cast<unsigned>(nb)),
                           dim3(kBlock), 0, s, a.m, static_cast<int>(a.K), a.rp, bnd, nslabs, sl, a.ci,
                           static_cast<const TV *>(a.vals), static_cast<const TUV *>(a.U), a.ldu,
                           static_cast<const TUV *>(a.V), a.ldv, static_cast<A *>(a.S));
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
    }
    return hipSuccess;
}

template <typename TUV, typename TV, int VW, int LANES, bool OFF32>
static hipError_t dispatch_ns(const SddmmArgs &a, hipStream_t s) {
    const int64_t ns = (a.K + LANES * VW - 1) / (LANES * VW);
    if (ns <= 1) return launch<TUV, TV, VW, LANES, 1, OFF32>(a, s);
    if (ns <= 2) return launch<TUV, TV, VW, LANES, 2, OFF32>(a, s);
    if (ns <= 4) return launch<TUV, TV, VW, LANES, 4, OFF32>(a, s);
    if (ns <= 8) return launch<TUV, TV, VW, LANES, 8, OFF32>(a, s);
    return hipErrorInvalidValue;
}

template <typename TUV, typename TV, int VW, bool OFF32>
static hipError_t dispatch_lanes(const SddmmArgs &a, hipStream_t s) {
    switch (a.lanes) {
    case 4: return dispatch_ns<TUV, TV, VW, 4, OFF32>(a, s);
    case 8: return dispatch_ns<TUV, TV, VW, 8, OFF32>(a, s);
    case 16: return dispatch_ns<TUV, TV, VW, 16, OFF32>(a, s);
    case 32: return dispatch_ns<TUV, TV, VW, 32, OFF32>(a, s);
    case 64: return dispatch_ns<TUV, TV, VW, 64, OFF32>(a, s);
    default: return hipErrorInvalidValue;
    }
}

template <typename TUV, typename TV, int VW>
static hipError_t dispatch_off(const SddmmArgs &a, hipStream_t s) {
    const bool off32 = static_cast<uint64_t>(a.n) * static_cast<uint64_t>(a.ldv) < (1ull << 32);
    return off32 ? dispatch_lanes<TUV, TV, VW, true>(a, s) : dispatch_lanes<TUV, TV, VW, false>(a, s);
}

hipError_t sddmm_launch(const SddmmArgs &a, hipStream_t s) {
    if (a.variant == SPK_VAR_TILE) {
        if (a.quad_split) {
            if (a.uv_dtype == SPK_F32) return launch_tileq<float, float>(a, s);
            if (a.uv_dtype == SPK_BF16) return launch_tileq<bf16, float>(a, s);
        }
        if (a.uv_dtype == SPK_F32) return launch_tile<float, float>(a, s);
        if (a.uv_dtype == SPK_BF16) return launch_tile<bf16, float>(a, s);
        return hipErrorInvalidValue;
    }
    switch (a.uv_dtype) {
    case SPK_F32: return a.vec > 1 ? dispatch_off<float, float, 4>(a, s) : dispatch_off<float, float, 1>(a, s);
    case SPK_BF16: return a.vec > 1 ? dispatch_off<bf16, float, 4>(a, s) : dispatch_off<bf16, float, 1>(a, s);
    case SPK_F64: return a.vec > 1 ? dispatch_off<double, double, 2>(a, s) : dispatch_off<double, double, 1>(a, s);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace spk
