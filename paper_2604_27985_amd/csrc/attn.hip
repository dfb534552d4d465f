// attn.hip - three back-to-back products on A's pattern with the
// intermediate kept on chip (the paper's future work on consecutive
// operations whose result stays resident, Section V):
//
//   S = A (.) (U V^T)        scores on A's stored entries (Eq. 2)
//   P = softmax of each row's stored scores
//   O = P B                  (Eq. 1 with P as the values)
//
// One group of LANES lanes owns a row and walks its entries R at a time: the
// R rows of V are gathered and dotted with the row of U held in registers,
// the partial dots are summed across the group (DPP within 16 lanes), and a
// running (online) softmax rescales the accumulated row of O whenever the
// running maximum grows, so P is never written: per entry the only HBM
// traffic is its column and value and the two gathered rows.  The row's
// entries are taken in storage order with fixed reductions: results do not
// vary from run to run.
//
// csr_row_softmax is the middle step alone (scores in, probabilities out, in
// place), for the unfused three-launch form of the same chain.
#include <math.h>

#include "common.h"
#include "internal.h"

namespace spk {

// Sum over an aligned group of G lanes, every lane ending with the total:
// partner exchanges lane ^ 1, lane ^ 2 (quad_perm), then the 8-lane and
// 16-lane mirrors (each pairs two halves that hold disjoint partial sums),
// then ds_bpermute beyond 16 lanes.
template <int CTRL>
__device__ __forceinline__ float dpp_f(float v) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xF, 0xF, true));
}

template <int G>
__device__ __forceinline__ float allsum(float v, int lane) {
    if constexpr (G >= 2) v += dpp_f<0xB1>(v);
    if constexpr (G >= 4) v += dpp_f<0x4E>(v);
    if constexpr (G >= 8) v += dpp_f<0x141>(v);
    if constexpr (G >= 16) v += dpp_f<0x140>(v);
    if constexpr (G >= 32) v += lane_read(v, lane ^ 16);
    if constexpr (G >= 64) v += lane_read(v, lane ^ 32);
    return v;
}

// Running softmax state of a run of one row's entries: maximum score mx, sum
// of exp(score - mx) l, and acc = sum of exp(score - mx) B[col] (this lane's
// slices of K2 columns).
template <int NS, int VW>
struct SoftState {
    float mx, l;
    float acc[NS][VW];

    __device__ __forceinline__ void clear() {
        mx = -INFINITY;
        l = 0.f;
#pragma unroll
        for (int s = 0; s < NS; ++s)
#pragma unroll
            for (int e = 0; e < VW; ++e) acc[s][e] = 0.f;
    }
};

// The lane's slices of U's row and the clamped column offsets of its slices
// (lanes past K read column 0, whose products are never used).
template <typename T, int VW, int LANES, int NS>
struct RowCtx {
    float u[NS][VW];
    int k1[NS], k2[NS];

    __device__ __forceinline__ void load(const T *__restrict__ U, int64_t row, int64_t ldu, int K1, int K2, int lig) {
#pragma unroll
        for (int s = 0; s < NS; ++s) {
            const int k = s * LANES * VW + lig * VW;
            if (k < K1) vec_load<T, VW>::run(U + row * ldu + k, u[s]);
            else
#pragma unroll
                for (int e = 0; e < VW; ++e) u[s][e] = 0.f;
            k1[s] = k < K1 ? k : 0;
            k2[s] = k < K2 ? k : 0;
        }
    }
};

// Adds entries [pa, pb) of one row to st, R at a time: R rows of V are
// gathered and dotted with U's row, the dots summed over the group, the
// state rescaled to the new maximum and R weighted rows of B added.
template <typename T, int VW, int LANES, int NS>
__device__ __forceinline__ void soft_run(int64_t pa, int64_t pb, const int32_t *__restrict__ ci,
                                         const float *__restrict__ vals, const T *__restrict__ V, int64_t ldv,
                                         const T *__restrict__ B, int64_t ldb, const RowCtx<T, VW, LANES, NS> &rc,
                                         SoftState<NS, VW> &st, int lig, int gbase, int lane) {
    constexpr int R = LANES < 8 ? LANES : 8;
    for (int64_t p0 = pa; p0 < pb; p0 += R) {
        const int cnt = static_cast<int>(pb - p0 < R ? pb - p0 : R);
        const int mine = lig < cnt ? lig : cnt - 1;
        const int c_mine = ci[p0 + mine];
        const float v_mine = vals ? vals[p0 + mine] : 1.f;
        int cq[R];
        float sc[R];
#pragma unroll
        for (int q = 0; q < R; ++q) cq[q] = lane_read(c_mine, gbase + q);
        // every gather of the step (R rows of V, then R rows of B) is issued
        // before any of them is used: the B rows are in flight while the
        // scores are formed
        float vr[R][NS][VW], br[R][NS][VW];
#pragma unroll
        for (int q = 0; q < R; ++q)
#pragma unroll
            for (int s = 0; s < NS; ++s) vec_load<T, VW>::run(V + static_cast<int64_t>(cq[q]) * ldv + rc.k1[s], vr[q][s]);
#pragma unroll
        for (int q = 0; q < R; ++q)
#pragma unroll
            for (int s = 0; s < NS; ++s) vec_load<T, VW>::run(B + static_cast<int64_t>(cq[q]) * ldb + rc.k2[s], br[q][s]);
#pragma unroll
        for (int q = 0; q < R; ++q) {
            float part = 0.f;
#pragma unroll
            for (int s = 0; s < NS; ++s)
#pragma unroll
                for (int e = 0; e < VW; ++e) part = fma(rc.u[s][e], vr[q][s][e], part);
            sc[q] = allsum<LANES>(part, lane) * lane_read(v_mine, gbase + q);
        }
        float mstep = sc[0];
#pragma unroll
        for (int q = 1; q < R; ++q)
            if (q < cnt) mstep = fmaxf(mstep, sc[q]);
        const float mnew = fmaxf(st.mx, mstep);
        const float scale = __expf(st.mx - mnew);  // 0 while the state is empty (mx = -inf)
        float w[R];
        float wsum = 0.f;
#pragma unroll
        for (int q = 0; q < R; ++q) {
            w[q] = q < cnt ? __expf(sc[q] - mnew) : 0.f;
            wsum += w[q];
        }
        st.l = st.l * scale + wsum;
        st.mx = mnew;
#pragma unroll
        for (int s = 0; s < NS; ++s)
#pragma unroll
            for (int e = 0; e < VW; ++e) st.acc[s][e] *= scale;
#pragma unroll
        for (int q = 0; q < R; ++q)
#pragma unroll
            for (int s = 0; s < NS; ++s)
#pragma unroll
                for (int e = 0; e < VW; ++e) st.acc[s][e] = fma(w[q], br[q][s][e], st.acc[s][e]);
    }
}

// O's row (acc / l; zeros for a row without entries) and lse.
template <int VW, int LANES, int NS>
__device__ __forceinline__ void soft_store(const SoftState<NS, VW> &st, bool any, int64_t row, float *__restrict__ O,
                                           int64_t ldo, float *__restrict__ lse, int K2, int lig) {
    const float inv = any ? 1.f / st.l : 0.f;
#pragma unroll
    for (int s = 0; s < NS; ++s) {
        const int k = s * LANES * VW + lig * VW;
        if (k < K2) {
            float o[VW];
#pragma unroll
            for (int e = 0; e < VW; ++e) o[e] = st.acc[s][e] * inv;
            vec_store<float, VW>::run(O + row * ldo + k, o);
        }
    }
    if (lse && lig == 0) lse[row] = any ? st.mx + logf(st.l) : -INFINITY;
}

// ROWS: one group per row.
template <typename T, int VW, int LANES, int NS>
__global__ __launch_bounds__(kBlock) void attn_rows_kernel(int64_t m, int K1, int K2, const int32_t *__restrict__ rp,
                                                           const int32_t *__restrict__ ci,
                                                           const float *__restrict__ vals, const T *__restrict__ U,
                                                           int64_t ldu, const T *__restrict__ V, int64_t ldv,
                                                           const T *__restrict__ B, int64_t ldb,
                                                           float *__restrict__ O, int64_t ldo,
                                                           float *__restrict__ lse) {
    constexpr int GPB = kBlock / LANES;
    const int lane = threadIdx.x & (kWave - 1);
    const int lig = threadIdx.x & (LANES - 1);
    const int gbase = lane & ~(LANES - 1);
    const int64_t blk = xcd_block(blockIdx.x, gridDim.x);
    const int64_t row = blk * GPB + threadIdx.x / LANES;
    if (row >= m) return;
    RowCtx<T, VW, LANES, NS> rc;
    rc.load(U, row, ldu, K1, K2, lig);
    SoftState<NS, VW> st;
    st.clear();
    const int64_t a = rp[row], b = rp[row + 1];
    soft_run<T, VW, LANES, NS>(a, b, ci, vals, V, ldv, B, ldb, rc, st, lig, gbase, lane);
    soft_store<VW, LANES, NS>(st, b > a, row, O, ldo, lse, K2, lig);
}

// MERGE: group g takes entries [g*items, (g+1)*items).  A row lying wholly
// inside the run is finished here.  A row cut by the run's ends leaves a
// partial state: its first piece in slot 1 of the group, every later piece
// (the last one, and middle pieces when the row spans several runs) in
// slot 0.  Slot rows are -1 when unused.  attn_fixup_kernel combines the
// pieces of every cut row in run order.
template <typename T, int VW, int LANES, int NS>
__global__ __launch_bounds__(kBlock) void attn_split_kernel(int64_t m, int64_t nnz, int K1, int K2,
                                                            const int32_t *__restrict__ rp,
                                                            const int32_t *__restrict__ ci,
                                                            const float *__restrict__ vals, const T *__restrict__ U,
                                                            int64_t ldu, const T *__restrict__ V, int64_t ldv,
                                                            const T *__restrict__ B, int64_t ldb,
                                                            float *__restrict__ O, int64_t ldo,
                                                            float *__restrict__ lse, int64_t items, int64_t ngroups,
                                                            int32_t *__restrict__ slot_row,
                                                            float *__restrict__ slot_ml,
                                                            float *__restrict__ slot_acc) {
    constexpr int GPB = kBlock / LANES;
    const int lane = threadIdx.x & (kWave - 1);
    const int lig = threadIdx.x & (LANES - 1);
    const int gbase = lane & ~(LANES - 1);
    const int64_t blk = xcd_block(blockIdx.x, gridDim.x);
    const int64_t g = blk * GPB + threadIdx.x / LANES;
    if (g >= ngroups) return;
    const int64_t p0 = g * items;
    const int64_t p1 = p0 + items < nnz ? p0 + items : nnz;
    int32_t used0 = -1, used1 = -1;
    // row holding entry p0: largest r with row_ptr[r] <= p0
    int64_t r = last_at_most(0, m - 1, p0, [&](int64_t i) { return static_cast<int64_t>(rp[i]); });
    for (; r < m; ++r) {
        const int64_t ra = rp[r], rb = rp[r + 1];
        if (ra >= p1) break;
        const int64_t a = ra > p0 ? ra : p0, b = rb < p1 ? rb : p1;
        if (a >= b) continue;  // empty row (written by attn_empty_kernel)
        RowCtx<T, VW, LANES, NS> rc;
        rc.load(U, r, ldu, K1, K2, lig);
        SoftState<NS, VW> st;
        st.clear();
        soft_run<T, VW, LANES, NS>(a, b, ci, vals, V, ldv, B, ldb, rc, st, lig, gbase, lane);
        if (ra >= p0 && rb <= p1) {
            soft_store<VW, LANES, NS>(st, true, r, O, ldo, lse, K2, lig);
            continue;
        }
        const int64_t slot = 2 * g + (ra >= p0 ? 1 : 0);  // first piece: slot 1; later pieces: slot 0
        if (ra >= p0) used1 = static_cast<int32_t>(r);
        else used0 = static_cast<int32_t>(r);
        if (lig == 0) {
            slot_ml[2 * slot] = st.mx;
            slot_ml[2 * slot + 1] = st.l;
        }
#pragma unroll
        for (int s = 0; s < NS; ++s) {
            const int k = s * LANES * VW + lig * VW;
            if (k < K2) vec_store<float, VW>::run(slot_acc + slot * K2 + k, st.acc[s]);
        }
    }
    if (lig == 0) {
        slot_row[2 * g] = used0;
        slot_row[2 * g + 1] = used1;
    }
}

// Partial softmax states (maximum, normaliser, K2 weighted sums) are
// combined in a fixed order.  states_max_sum: state t (t < count) sits at
// slot slot_of(t) of ml; lane j combines states j, j + 64, ... in order,
// loading four at a time from clamped indices (no branch around the loads,
// so they are in flight together), then the 64 lane states are combined by
// a butterfly whose two partners compute the same (commutative) expression,
// so every lane ends with the same bits.
template <typename SlotOf>
__device__ __forceinline__ void states_max_sum(int64_t count, SlotOf slot_of, const float *__restrict__ ml, int lane,
                                               float &mx, float &l) {
    mx = -INFINITY;
    l = 0.f;
    constexpr int E = 4;
    for (int64_t t0 = lane; t0 < count; t0 += E * kWave) {
        float mb[E], lb[E];
#pragma unroll
        for (int e = 0; e < E; ++e) {
            const int64_t t = t0 + e * kWave;
            const int64_t sl = slot_of(t < count ? t : count - 1);
            mb[e] = ml[2 * sl];
            lb[e] = ml[2 * sl + 1];
        }
#pragma unroll
        for (int e = 0; e < E; ++e) {
            if (t0 + e * kWave >= count) break;
            const float mn = fmaxf(mx, mb[e]);
            l = l * __expf(mx - mn) + lb[e] * __expf(mb[e] - mn);
            mx = mn;
        }
    }
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) {
        const float m2 = lane_read(mx, lane ^ d), l2 = lane_read(l, lane ^ d);
        const float mn = fmaxf(mx, m2);
        // an empty lane state (mx = -inf, l = 0) adds nothing
        const float ea = mx == -INFINITY ? 0.f : l * __expf(mx - mn);
        const float eb = m2 == -INFINITY ? 0.f : l2 * __expf(m2 - mn);
        l = ea + eb;
        mx = mn;
    }
}

// Column k of the states' sums rescaled to the maximum mx and added in state
// order, 16 states' loads in flight at a time (clamped indices).
template <typename SlotOf>
__device__ __forceinline__ float states_weighted(int64_t count, SlotOf slot_of, const float *__restrict__ ml,
                                                 const float *__restrict__ acc, int K2, int k, float mx) {
    constexpr int D = 16;
    float a = 0.f;
    for (int64_t h = 0; h < count; h += D) {
        float v[D], w[D];
#pragma unroll
        for (int u = 0; u < D; ++u) {
            const int64_t sl = slot_of(h + u < count ? h + u : count - 1);
            v[u] = acc[sl * K2 + k];
            w[u] = ml[2 * sl];
        }
#pragma unroll
        for (int u = 0; u < D; ++u)
            if (h + u < count) a = fma(v[u], __expf(w[u] - mx), a);  // wave-uniform condition
    }
    return a;
}

// Pieces per first-level fold of a long row.
constexpr int64_t kFold = 64;

// First level for rows cut into more than kFold pieces: one wave per run; a
// run holding piece t0 of such a row with t0 a multiple of kFold (the first
// piece in slot 1, later ones in slot 0) combines pieces t0 .. t0 + kFold - 1
// into the fold slot of that piece.  A hub row's chain of loads is then
// kFold pieces long here and count / kFold folds long in the fix-up.
__global__ __launch_bounds__(kBlock) void attn_fold_kernel(int64_t ngroups, int64_t items, int K2,
                                                           const int32_t *__restrict__ rp,
                                                           const int32_t *__restrict__ slot_row,
                                                           const float *__restrict__ slot_ml,
                                                           const float *__restrict__ slot_acc,
                                                           float *__restrict__ fold_ml, float *__restrict__ fold_acc) {
    const int64_t h = static_cast<int64_t>(blockIdx.x) * (kBlock / kWave) + threadIdx.x / kWave;
    const int lane = threadIdx.x & (kWave - 1);
    if (h >= ngroups) return;
    for (int slot = 0; slot < 2; ++slot) {
        const int32_t r = slot_row[2 * h + slot];
        if (r < 0) continue;
        const int64_t g0 = static_cast<int64_t>(rp[r]) / items;  // the run of the row's first piece
        const int64_t np = (static_cast<int64_t>(rp[r + 1]) - 1) / items + 1 - g0;
        const int64_t t0 = h - g0;
        if (np <= kFold || t0 % kFold != 0) continue;
        const int64_t count = np - t0 < kFold ? np - t0 : kFold;
        auto slot_of = [&](int64_t t) { return t0 + t == 0 ? 2 * g0 + 1 : 2 * (g0 + t0 + t); };
        float mx, l;
        states_max_sum(count, slot_of, slot_ml, lane, mx, l);
        const int64_t fs = 2 * h + slot;
        for (int k = lane; k < K2; k += kWave)
            fold_acc[fs * K2 + k] = states_weighted(count, slot_of, slot_ml, slot_acc, K2, k, mx);
        if (lane == 0) {
            fold_ml[2 * fs] = mx;
            fold_ml[2 * fs + 1] = l;
        }
    }
}

// One wave per run: a run whose slot 1 holds a row's first piece combines the
// row's pieces (at most kFold of them) or the first level's folds of them, in
// run order, and writes the row of O and lse.  The row's last run follows
// from its end in row_ptr.
__global__ __launch_bounds__(kBlock) void attn_fixup_kernel(int64_t ngroups, int64_t items, int K2,
                                                            const int32_t *__restrict__ rp,
                                                            const int32_t *__restrict__ slot_row,
                                                            const float *__restrict__ slot_ml,
                                                            const float *__restrict__ slot_acc,
                                                            const float *__restrict__ fold_ml,
                                                            const float *__restrict__ fold_acc,
                                                            float *__restrict__ O, int64_t ldo,
                                                            float *__restrict__ lse) {
    const int64_t g = static_cast<int64_t>(blockIdx.x) * (kBlock / kWave) + threadIdx.x / kWave;
    const int lane = threadIdx.x & (kWave - 1);
    if (g >= ngroups) return;
    const int32_t r = slot_row[2 * g + 1];
    if (r < 0) return;
    // runs g .. h_end - 1 hold the row: the last is the run of its last entry
    const int64_t np = (static_cast<int64_t>(rp[r + 1]) - 1) / items + 1 - g;
    const bool folded = np > kFold;
    const int64_t count = folded ? (np + kFold - 1) / kFold : np;
    // piece t: slot 1 of run g for t = 0, else slot 0 of run g + t; fold b:
    // the slot of piece b * kFold
    auto slot_of = [&](int64_t t) {
        const int64_t piece = folded ? t * kFold : t;
        return piece == 0 ? 2 * g + 1 : 2 * (g + piece);
    };
    const float *ml = folded ? fold_ml : slot_ml;
    const float *acc = folded ? fold_acc : slot_acc;
    float mx, l;
    states_max_sum(count, slot_of, ml, lane, mx, l);
    const float inv = 1.f / l;
    for (int k = lane; k < K2; k += kWave)
        O[static_cast<int64_t>(r) * ldo + k] = states_weighted(count, slot_of, ml, acc, K2, k, mx) * inv;
    if (lse && lane == 0) lse[r] = mx + logf(l);
}

// Rows without stored entries: zeros and -inf (the entry-split kernel never
// visits them).
__global__ void attn_empty_kernel(int64_t m, int K2, const int32_t *__restrict__ rp, float *__restrict__ O, int64_t ldo,
                                  float *__restrict__ lse) {
    const int64_t idx = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (idx >= m) return;
    if (rp[idx] != rp[idx + 1]) return;
    for (int k = 0; k < K2; ++k) O[idx * ldo + k] = 0.f;
    if (lse) lse[idx] = -INFINITY;
}

template <typename T, int VW, int LANES, int NS>
static hipError_t launch_attn(const AttnArgs &a, hipStream_t s) {
    constexpr int GPB = kBlock / LANES;
    if (a.variant == SPK_VAR_MERGE) {
        const AttnLayout L = attn_layout(a.nnz, a.K2, a.items, true);
        char *ws = static_cast<char *>(a.ws);
        int32_t *slot_row = reinterpret_cast<int32_t *>(ws + L.row_off);
        float *slot_ml = reinterpret_cast<float *>(ws + L.ml_off);
        float *slot_acc = reinterpret_cast<float *>(ws + L.acc_off);
        float *fold_ml = reinterpret_cast<float *>(ws + L.fold_ml_off);
        float *fold_acc = reinterpret_cast<float *>(ws + L.fold_acc_off);
        if (a.m > 0) {
            hipLaunchKernelGGL(attn_empty_kernel, dim3(static_cast<unsigned>((a.m + kBlock - 1) / kBlock)), dim3(kBlock),
                               0, s, a.m, static_cast<int>(a.K2), a.rp, a.O, a.ldo, a.lse);
            hipError_t e = hipGetLastError();
            if (e != hipSuccess) return e;
        }
        if (L.ngroups == 0) return hipSuccess;
        const int64_t nb = (L.ngroups + GPB - 1) / GPB;
        if (!grid_fits(nb, kBlock)) return kGridTooLarge;
        hipLaunchKernelGGL((attn_split_kernel<T, VW, LANES, NS>), dim3(static_cast<unsigned>(nb)), dim3(kBlock), 0, s,
                           a.m, a.nnz, static_cast<int>(a.K1), static_cast<int>(a.K2), a.rp, a.ci, a.vals,
                           static_cast<const T *>(a.U), a.ldu, static_cast<const T *>(a.V), a.ldv,
                           static_cast<const T *>(a.B), a.ldb, a.O, a.ldo, a.lse, L.items, L.ngroups, slot_row,
                           slot_ml, slot_acc);
        hipError_t e = hipGetLastError();
        if (e != hipSuccess) return e;
        constexpr int wpb = kBlock / kWave;
        const dim3 grid(static_cast<unsigned>((L.ngroups + wpb - 1) / wpb));
        hipLaunchKernelGGL(attn_fold_kernel, grid, dim3(kBlock), 0, s, L.ngroups, L.items, static_cast<int>(a.K2), a.rp,
                           slot_row, slot_ml, slot_acc, fold_ml, fold_acc);
        if ((e = hipGetLastError()) != hipSuccess) return e;
        hipLaunchKernelGGL(attn_fixup_kernel, grid, dim3(kBlock), 0, s, L.ngroups, L.items, static_cast<int>(a.K2), a.rp,
                           slot_row, slot_ml, slot_acc, fold_ml, fold_acc, a.O, a.ldo, a.lse);
        return hipGetLastError();
    }
    const int64_t nb = (a.m + GPB - 1) / GPB;
    if (!grid_fits(nb, kBlock)) return kGridTooLarge;
    hipLaunchKernelGGL((attn_rows_kernel<T, VW, LANES, NS>), dim3(static_cast<unsigned>(nb)), dim3(kBlock), 0, s, a.m,
                       static_cast<int>(a.K1), static_cast<int>(a.K2), a.rp, a.ci, a.vals,
                       static_cast<const T *>(a.U), a.ldu, static_cast<const T *>(a.V), a.ldv,
                       static_cast<const T *>(a.B), a.ldb, a.O, a.ldo, a.lse);
    return hipGetLastError();
}

template <typename T, int VW, int LANES>
static hipError_t attn_ns(const AttnArgs &a, hipStream_t s) {
    const int64_t kmax = a.K1 > a.K2 ? a.K1 : a.K2;
    const int64_t ns = (kmax + LANES * VW - 1) / (LANES * VW);
    if (ns <= 1) return launch_attn<T, VW, LANES, 1>(a, s);
    if (ns <= 2) return launch_attn<T, VW, LANES, 2>(a, s);
    if (ns <= 4) return launch_attn<T, VW, LANES, 4>(a, s);
    if (ns <= 8) return launch_attn<T, VW, LANES, 8>(a, s);
    return hipErrorInvalidValue;
}

template <typename T, int VW>
static hipError_t attn_lanes(const AttnArgs &a, hipStream_t s) {
    switch (a.lanes) {
    case 4: return attn_ns<T, VW, 4>(a, s);
    case 8: return attn_ns<T, VW, 8>(a, s);
    case 16: return attn_ns<T, VW, 16>(a, s);
    case 32: return attn_ns<T, VW, 32>(a, s);
    case 64: return attn_ns<T, VW, 64>(a, s);
    default: return hipErrorInvalidValue;
    }
}

hipError_t attn_launch(const AttnArgs &a, hipStream_t s) {
    if (a.dtype == SPK_F32) return a.vec == 4 ? attn_lanes<float, 4>(a, s) : attn_lanes<float, 1>(a, s);
    if (a.dtype == SPK_BF16) return a.vec == 4 ? attn_lanes<bf16, 4>(a, s) : attn_lanes<bf16, 1>(a, s);
    return hipErrorInvalidValue;
}

// Row softmax of stored scores in place, balanced over entries: one wave per
// run of `items` entries (the same runs and piece slots as the entry-split
// attention).  Pass 1 finds each row piece's maximum and sum of exponentials
// (a row wholly inside the run is finished into rowml), pass 2 combines the
// pieces of cut rows in run order, pass 3 rewrites every score as its
// probability.  Reductions are deterministic: inside each 16-lane row by
// DPP moves (lane ^ 1, lane ^ 2, then the 8- and 16-lane mirrors; the two
// lanes of every pair compute the same commutative expression), then the
// four rows' values read back with readlane and combined in a fixed order,
// so every lane ends with the same bits.  No LDS round trip: a row of a few
// entries costs a handful of VALU moves instead of six ds_bpermute waits.
__device__ __forceinline__ float lane_value(float v, int src) {
    return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), src));
}
__device__ __forceinline__ float wave_max(float v) {
    v = fmaxf(v, dpp_f<0xB1>(v));
    v = fmaxf(v, dpp_f<0x4E>(v));
    v = fmaxf(v, dpp_f<0x141>(v));
    v = fmaxf(v, dpp_f<0x140>(v));
    return fmaxf(fmaxf(lane_value(v, 0), lane_value(v, 16)), fmaxf(lane_value(v, 32), lane_value(v, 48)));
}
__device__ __forceinline__ float wave_sum(float v) {
    v += dpp_f<0xB1>(v);
    v += dpp_f<0x4E>(v);
    v += dpp_f<0x141>(v);
    v += dpp_f<0x140>(v);
    return (lane_value(v, 0) + lane_value(v, 16)) + (lane_value(v, 32) + lane_value(v, 48));
}

// A wave's run of scores, staged in LDS with coalesced loads (lane l holds
// slot j * 64 + l), and the ends of the run's rows, 64 at a time in a
// register of each lane (read back with readlane): the walk over the run's
// rows then waits on no global load per row.
constexpr int kSoftmaxWaves = kBlock / kWave;
static_assert(kSoftmaxItems % kWave == 0, "a run fills whole slots of the wave");

__device__ __forceinline__ void stage_run(const float *__restrict__ S, int64_t p0, int64_t p1, float *xs, int lane) {
#pragma unroll 4
    for (int j = 0; j < kSoftmaxItems / kWave; ++j) {
        const int64_t p = p0 + j * kWave + lane;
        xs[j * kWave + lane] = S[p < p1 ? p : p1 - 1];
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

__global__ __launch_bounds__(kBlock) void softmax_stats_kernel(int64_t m, int64_t nnz, const int32_t *__restrict__ rp,
                                                               const float *__restrict__ S, int64_t items,
                                                               int64_t ngroups, float *__restrict__ rowml,
                                                               int32_t *__restrict__ slot_row,
                                                               float *__restrict__ slot_ml) {
    __shared__ float xs_all[kSoftmaxWaves][kSoftmaxItems];
    const int64_t g = static_cast<int64_t>(blockIdx.x) * kSoftmaxWaves + threadIdx.x / kWave;
    const int lane = threadIdx.x & (kWave - 1);
    if (g >= ngroups) return;
    float *xs = xs_all[threadIdx.x / kWave];
    const int64_t p0 = g * items;
    const int64_t p1 = p0 + items < nnz ? p0 + items : nnz;
    stage_run(S, p0, p1, xs, lane);
    int32_t used0 = -1, used1 = -1;
    int64_t r = last_at_most(0, m - 1, p0, [&](int64_t i) { return static_cast<int64_t>(rp[i]); });
    int64_t ra = rp[r];
    for (bool more = true; more && r < m;) {
        // ends of rows r .. r + 63 (clamped past the last row)
        const int32_t ends = rp[(r + 1 + lane) < m ? r + 1 + lane : m];
        for (int k = 0; k < kWave && r < m; ++k, ++r) {
            const int64_t rb = __builtin_amdgcn_readlane(ends, k);
            if (ra >= p1) {
                more = false;
                break;
            }
            const int64_t a = ra > p0 ? ra : p0, b = rb < p1 ? rb : p1;
            const int64_t row_start = ra;
            ra = rb;
            if (a >= b) continue;
            float mx = -INFINITY;
            for (int64_t p = a + lane; p < b; p += kWave) mx = fmaxf(mx, xs[p - p0]);
            mx = wave_max(mx);
            float l = 0.f;
            for (int64_t p = a + lane; p < b; p += kWave) l += __expf(xs[p - p0] - mx);
            l = wave_sum(l);
            if (row_start >= p0 && rb <= p1) {
                if (lane == 0) {
                    rowml[2 * r] = mx;
                    rowml[2 * r + 1] = l;
                }
                continue;
            }
            const int64_t slot = 2 * g + (row_start >= p0 ? 1 : 0);
            if (row_start >= p0) used1 = static_cast<int32_t>(r);
            else used0 = static_cast<int32_t>(r);
            if (lane == 0) {
                slot_ml[2 * slot] = mx;
                slot_ml[2 * slot + 1] = l;
            }
        }
    }
    if (lane == 0) {
        slot_row[2 * g] = used0;
        slot_row[2 * g + 1] = used1;
    }
}

__global__ __launch_bounds__(kBlock) void softmax_fixup_kernel(int64_t ngroups, int64_t items,
                                                               const int32_t *__restrict__ rp,
                                                               const int32_t *__restrict__ slot_row,
                                                               const float *__restrict__ slot_ml,
                                                               float *__restrict__ rowml) {
    const int64_t g = static_cast<int64_t>(blockIdx.x) * (kBlock / kWave) + threadIdx.x / kWave;
    const int lane = threadIdx.x & (kWave - 1);
    if (g >= ngroups) return;
    const int32_t r = slot_row[2 * g + 1];
    if (r < 0) return;
    // runs g .. the run of the row's last entry hold its pieces
    const int64_t npieces = (static_cast<int64_t>(rp[r + 1]) - 1) / items + 1 - g;
    auto slot_of = [&](int64_t t) { return t == 0 ? 2 * g + 1 : 2 * (g + t); };
    float mx, l;
    states_max_sum(npieces, slot_of, slot_ml, lane, mx, l);
    if (lane == 0) {
        rowml[2 * r] = mx;
        rowml[2 * r + 1] = l;
    }
}

__global__ __launch_bounds__(kBlock) void softmax_apply_kernel(int64_t m, int64_t nnz, const int32_t *__restrict__ rp,
                                                               float *__restrict__ S, int64_t items, int64_t ngroups,
                                                               const float *__restrict__ rowml,
                                                               float *__restrict__ lse) {
    __shared__ float xs_all[kSoftmaxWaves][kSoftmaxItems];
    const int64_t g = static_cast<int64_t>(blockIdx.x) * kSoftmaxWaves + threadIdx.x / kWave;
    const int lane = threadIdx.x & (kWave - 1);
    if (g >= ngroups) return;
    float *xs = xs_all[threadIdx.x / kWave];
    const int64_t p0 = g * items;
    const int64_t p1 = p0 + items < nnz ? p0 + items : nnz;
    stage_run(S, p0, p1, xs, lane);
    int64_t r = last_at_most(0, m - 1, p0, [&](int64_t i) { return static_cast<int64_t>(rp[i]); });
    int64_t ra = rp[r];
    for (bool more = true; more && r < m;) {
        // ends, maxima and normalisers of rows r .. r + 63
        const int64_t rl = (r + lane) < m ? r + lane : m - 1;
        const int32_t ends = rp[rl + 1];
        const float mxs = rowml[2 * rl], ls = rowml[2 * rl + 1];
        for (int k = 0; k < kWave && r < m; ++k, ++r) {
            const int64_t rb = __builtin_amdgcn_readlane(ends, k);
            if (ra >= p1) {
                more = false;
                break;
            }
            const int64_t a = ra > p0 ? ra : p0, b = rb < p1 ? rb : p1;
            const bool first = ra >= p0;
            ra = rb;
            if (a >= b) continue;
            const float mx = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(mxs), k));
            const float lr = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(ls), k));
            const float inv = 1.f / lr;
            for (int64_t p = a + lane; p < b; p += kWave) xs[p - p0] = __expf(xs[p - p0] - mx) * inv;
            if (lse && lane == 0 && first) lse[r] = mx + logf(lr);
        }
    }
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
#pragma unroll 4
    for (int j = 0; j < kSoftmaxItems / kWave; ++j) {
        const int64_t p = p0 + j * kWave + lane;
        if (p < p1) S[p] = xs[j * kWave + lane];
    }
}

__global__ void softmax_empty_kernel(int64_t m, const int32_t *__restrict__ rp, float *__restrict__ lse) {
    const int64_t idx = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (idx < m && rp[idx] == rp[idx + 1]) lse[idx] = -INFINITY;
}

size_t row_softmax_ws_bytes(int64_t m, int64_t nnz) {
    const AttnLayout L = attn_layout(nnz, 0, kSoftmaxItems);
    return align_up(sizeof(float) * 2 * static_cast<size_t>(m)) + L.total;
}

hipError_t row_softmax_launch(int64_t m, int64_t nnz, const int32_t *rp, float *S, float *lse, void *ws_, hipStream_t s) {
    if (m == 0) return hipSuccess;
    hipError_t e;
    if (lse) {
        hipLaunchKernelGGL(softmax_empty_kernel, dim3(static_cast<unsigned>((m + kBlock - 1) / kBlock)), dim3(kBlock), 0, s,
                           m, rp, lse);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    const AttnLayout L = attn_layout(nnz, 0, kSoftmaxItems);
    if (L.ngroups == 0) return hipSuccess;
    char *ws = static_cast<char *>(ws_);
    float *rowml = reinterpret_cast<float *>(ws);
    char *slots = ws + align_up(sizeof(float) * 2 * static_cast<size_t>(m));
    int32_t *slot_row = reinterpret_cast<int32_t *>(slots + L.row_off);
    float *slot_ml = reinterpret_cast<float *>(slots + L.ml_off);
    constexpr int wpb = kBlock / kWave;
    const unsigned nb = static_cast<unsigned>((L.ngroups + wpb - 1) / wpb);
    hipLaunchKernelGGL(softmax_stats_kernel, dim3(nb), dim3(kBlock), 0, s, m, nnz, rp, S, L.items, L.ngroups, rowml,
                       slot_row, slot_ml);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(softmax_fixup_kernel, dim3(nb), dim3(kBlock), 0, s, L.ngroups, L.items, rp, slot_row, slot_ml,
                       rowml);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(softmax_apply_kernel, dim3(nb), dim3(kBlock), 0, s, m, nnz, rp, S, L.items, L.ngroups, rowml, lse);
    return hipGetLastError();
}

}  // namespace spk
