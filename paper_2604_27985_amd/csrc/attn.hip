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

template <typename T, int VW, int LANES, int NS>
__global__ __launch_bounds__(kBlock) void attn_rows_kernel(int64_t m, int K1, int K2, const int32_t *__restrict__ rp,
                                                           const int32_t *__restrict__ ci,
                                                           const float *__restrict__ vals, const T *__restrict__ U,
                                                           int64_t ldu, const T *__restrict__ V, int64_t ldv,
                                                           const T *__restrict__ B, int64_t ldb,
                                                           float *__restrict__ O, int64_t ldo,
                                                           float *__restrict__ lse) {
    constexpr int GPB = kBlock / LANES;
    constexpr int R = LANES < 8 ? LANES : 8;
    const int lane = threadIdx.x & (kWave - 1);
    const int lig = threadIdx.x & (LANES - 1);
    const int gbase = lane & ~(LANES - 1);
    const int64_t blk = xcd_block(blockIdx.x, gridDim.x);
    const int64_t row = blk * GPB + threadIdx.x / LANES;
    if (row >= m) return;
    // slice s of this lane: columns s * LANES * VW + lig * VW .. + VW
    float u[NS][VW], acc[NS][VW];
#pragma unroll
    for (int s = 0; s < NS; ++s) {
        const int k = s * LANES * VW + lig * VW;
        if (k < K1) vec_load<T, VW>::run(U + row * ldu + k, u[s]);
        else
#pragma unroll
            for (int e = 0; e < VW; ++e) u[s][e] = 0.f;
#pragma unroll
        for (int e = 0; e < VW; ++e) acc[s][e] = 0.f;
    }
    int k1[NS], k2[NS];  // clamped column offsets: lanes past K read column 0 (never used)
#pragma unroll
    for (int s = 0; s < NS; ++s) {
        const int k = s * LANES * VW + lig * VW;
        k1[s] = k < K1 ? k : 0;
        k2[s] = k < K2 ? k : 0;
    }
    float mrun = -INFINITY, lrun = 0.f;
    const int64_t a = rp[row], b = rp[row + 1];
    for (int64_t pb = a; pb < b; pb += R) {
        const int cnt = static_cast<int>(b - pb < R ? b - pb : R);
        const int mine = lig < cnt ? lig : cnt - 1;
        const int c_mine = ci[pb + mine];
        const float v_mine = vals ? vals[pb + mine] : 1.f;
        int cq[R];
        float sc[R];
#pragma unroll
        for (int q = 0; q < R; ++q) cq[q] = lane_read(c_mine, gbase + q);
        // scores: R gathered rows of V against the row of U
#pragma unroll
        for (int q = 0; q < R; ++q) {
            float part = 0.f;
#pragma unroll
            for (int s = 0; s < NS; ++s) {
                float vr[VW];
                vec_load<T, VW>::run(V + static_cast<int64_t>(cq[q]) * ldv + k1[s], vr);
#pragma unroll
                for (int e = 0; e < VW; ++e) part = fma(u[s][e], vr[e], part);
            }
            sc[q] = allsum<LANES>(part, lane) * lane_read(v_mine, gbase + q);
        }
        // online softmax: the accumulated row is rescaled to the new maximum
        float mstep = sc[0];
#pragma unroll
        for (int q = 1; q < R; ++q)
            if (q < cnt) mstep = fmaxf(mstep, sc[q]);
        const float mnew = fmaxf(mrun, mstep);
        const float scale = __expf(mrun - mnew);  // 0 on the first step (mrun = -inf)
        float w[R];
        float wsum = 0.f;
#pragma unroll
        for (int q = 0; q < R; ++q) {
            w[q] = q < cnt ? __expf(sc[q] - mnew) : 0.f;
            wsum += w[q];
        }
        lrun = lrun * scale + wsum;
        mrun = mnew;
#pragma unroll
        for (int s = 0; s < NS; ++s)
#pragma unroll
            for (int e = 0; e < VW; ++e) acc[s][e] *= scale;
#pragma unroll
        for (int q = 0; q < R; ++q) {
#pragma unroll
            for (int s = 0; s < NS; ++s) {
                float br[VW];
                vec_load<T, VW>::run(B + static_cast<int64_t>(cq[q]) * ldb + k2[s], br);
#pragma unroll
                for (int e = 0; e < VW; ++e) acc[s][e] = fma(w[q], br[e], acc[s][e]);
            }
        }
    }
    const float inv = b > a ? 1.f / lrun : 0.f;
#pragma unroll
    for (int s = 0; s < NS; ++s) {
        const int k = s * LANES * VW + lig * VW;
        if (k < K2) {
            float o[VW];
#pragma unroll
            for (int e = 0; e < VW; ++e) o[e] = acc[s][e] * inv;
            vec_store<float, VW>::run(O + row * ldo + k, o);
        }
    }
    if (lse && lig == 0) lse[row] = b > a ? mrun + logf(lrun) : -INFINITY;
}

template <typename T, int VW, int LANES, int NS>
static hipError_t launch_attn(const AttnArgs &a, hipStream_t s) {
    constexpr int GPB = kBlock / LANES;
    const int64_t nb = (a.m + GPB - 1) / GPB;
    if (nb > 0x7FFFFFFF) return hipErrorInvalidValue;
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

// Row softmax of stored scores in place: a wave per row, three passes
// (maximum, sum of exponentials, normalisation), fixed reduction order.
__global__ __launch_bounds__(kBlock) void row_softmax_kernel(int64_t m, const int32_t *__restrict__ rp,
                                                             float *__restrict__ S, float *__restrict__ lse) {
    const int64_t row = static_cast<int64_t>(blockIdx.x) * (kBlock / kWave) + threadIdx.x / kWave;
    const int lane = threadIdx.x & (kWave - 1);
    if (row >= m) return;
    const int64_t a = rp[row], b = rp[row + 1];
    float mx = -INFINITY;
    for (int64_t p = a + lane; p < b; p += kWave) mx = fmaxf(mx, S[p]);
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) mx = fmaxf(mx, lane_read(mx, lane ^ d));
    float sum = 0.f;
    for (int64_t p = a + lane; p < b; p += kWave) sum += __expf(S[p] - mx);
#pragma unroll
    for (int d = 1; d < kWave; d <<= 1) sum += lane_read(sum, lane ^ d);
    const float inv = 1.f / sum;
    for (int64_t p = a + lane; p < b; p += kWave) S[p] = __expf(S[p] - mx) * inv;
    if (lse && lane == 0) lse[row] = b > a ? mx + logf(sum) : -INFINITY;
}

hipError_t row_softmax_launch(int64_t m, const int32_t *rp, float *S, float *lse, hipStream_t s) {
    if (m == 0) return hipSuccess;
    constexpr int rows_per_block = kBlock / kWave;
    hipLaunchKernelGGL(row_softmax_kernel, dim3(static_cast<unsigned>((m + rows_per_block - 1) / rows_per_block)),
                       dim3(kBlock), 0, s, m, rp, S, lse);
    return hipGetLastError();
}

}  // namespace spk
