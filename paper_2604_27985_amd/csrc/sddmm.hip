// sddmm.hip - SDDMM S = A (.) (U V^T) (Section II-A, Eq. (2)) for gfx950.
//
// Only stored entries of A are computed (the dense product is never formed):
// S[p] = a_p * <U[row(p), :], V[col(p), :]>.
//
// Work is split by entries, not rows: group g of LANES lanes takes entries
// [g*chunk, (g+1)*chunk), finds the row of its first entry by binary search in
// row_ptr and walks forward, so power-law rows cost no imbalance.  Each lane
// holds an NS x VW slice of the current U row in registers (reloaded only
// when the row changes), gathers the matching slice of V's row with 8/16-byte
// loads, and the group's partial dot products are summed with a butterfly
// over the LANES lanes (ds_bpermute exchanges).  Up to eight entries of one
// row are processed per step: their column indices are read with one
// coalesced load and shared across the group, and all their V gathers are
// issued before any arithmetic.
#include "common.h"
#include "internal.h"

namespace spk {

template <typename TUV, typename TV, int VW, int LANES, int NS>
__global__ __launch_bounds__(kBlock) void sddmm_kernel(int64_t m, int64_t nnz, int K, const int32_t *__restrict__ rp,
                                                       const int32_t *__restrict__ ci,
                                                       const TV *__restrict__ vals,
                                                       const TUV *__restrict__ U, int64_t ldu,
                                                       const TUV *__restrict__ V, int64_t ldv,
                                                       typename acc_of<TUV>::type *__restrict__ S,
                                                       int64_t chunk, int64_t ngroups) {
    using A = typename acc_of<TUV>::type;
    constexpr int GPB = kBlock / LANES;
    constexpr int KT = LANES * VW;             // columns per slice
    constexpr int R = LANES < 8 ? LANES : 8;   // entries per step (<= LANES)
    const int lig = threadIdx.x & (LANES - 1);
    const int gbase = (threadIdx.x & (kWave - 1)) & ~(LANES - 1);
    const int64_t blk = xcd_block(blockIdx.x, gridDim.x);
    const int64_t g = blk * GPB + threadIdx.x / LANES;
    if (g >= ngroups) return;
    const int64_t p0 = g * chunk;
    const int64_t p1 = p0 + chunk < nnz ? p0 + chunk : nnz;

    // Row holding entry p0: largest r in [0, m-1] with row_ptr[r] <= p0.
    int64_t r = last_at_most(0, m - 1, p0, [&](int64_t i) { return static_cast<int64_t>(rp[i]); });
    int64_t next = rp[r + 1];
    int64_t loaded = -1;
    A u[NS][VW];

    for (int64_t pb = p0; pb < p1;) {
        while (pb >= next) {  // group-uniform; also skips empty rows
            ++r;
            next = rp[r + 1];
        }
        if (r != loaded) {
#pragma unroll
            for (int s = 0; s < NS; ++s) {
                const int k = s * KT + lig * VW;
                if (k < K) vec_load<TUV, VW>::run(U + r * ldu + k, u[s]);
                else
#pragma unroll
                    for (int e = 0; e < VW; ++e) u[s][e] = A(0);
            }
            loaded = r;
        }
        // A step never crosses a row end, so one U row serves all of it.
        int64_t lim = p1 < next ? p1 : next;
        const int cnt = static_cast<int>(lim - pb < R ? lim - pb : R);
        const int c_mine = lig < cnt ? ci[pb + lig] : 0;
        A vrow[R][NS][VW];
#pragma unroll
        for (int q = 0; q < R; ++q) {
            const int64_t c = lane_read(c_mine, gbase + q);
#pragma unroll
            for (int s = 0; s < NS; ++s) {
                const int k = s * KT + lig * VW;
                if (q < cnt && k < K) vec_load<TUV, VW>::run(V + c * ldv + k, vrow[q][s]);
                else
#pragma unroll
                    for (int e = 0; e < VW; ++e) vrow[q][s][e] = A(0);
            }
        }
        A part[R];
#pragma unroll
        for (int q = 0; q < R; ++q) {
            part[q] = A(0);
#pragma unroll
            for (int s = 0; s < NS; ++s)
#pragma unroll
                for (int e = 0; e < VW; ++e) part[q] = fma(u[s][e], vrow[q][s][e], part[q]);
            part[q] = group_sum<LANES>(part[q]);
        }
        if (lig < cnt) {  // lane q of the group writes entry pb + q
            A mine = part[0];
#pragma unroll
            for (int q = 1; q < R; ++q) mine = (lig == q) ? part[q] : mine;
            const int64_t p = pb + lig;
            const A a = vals ? static_cast<A>(vals[p]) : A(1);
            S[p] = a * mine;
        }
        pb += cnt;
    }
}

template <typename TUV, typename TV, int VW, int LANES, int NS>
static hipError_t launch_sddmm(const SddmmArgs &a, hipStream_t s) {
    constexpr int GPB = kBlock / LANES;
    const int64_t ngroups = (a.nnz + a.chunk - 1) / a.chunk;
    const int64_t nb = (ngroups + GPB - 1) / GPB;
    if (nb > 0x7FFFFFFF) return hipErrorInvalidValue;
    hipLaunchKernelGGL((sddmm_kernel<TUV, TV, VW, LANES, NS>), dim3(static_cast<unsigned>(nb)), dim3(kBlock), 0, s,
                       a.m, a.nnz, static_cast<int>(a.K), a.rp, a.ci, static_cast<const TV *>(a.vals),
                       static_cast<const TUV *>(a.U), a.ldu, static_cast<const TUV *>(a.V), a.ldv,
                       static_cast<typename acc_of<TUV>::type *>(a.S), a.chunk, ngroups);
    return hipGetLastError();
}

template <typename TUV, typename TV, int VW, int LANES>
static hipError_t dispatch_ns(const SddmmArgs &a, hipStream_t s) {
    const int64_t ns = (a.K + LANES * VW - 1) / (LANES * VW);
    if (ns <= 1) return launch_sddmm<TUV, TV, VW, LANES, 1>(a, s);
    if (ns <= 2) return launch_sddmm<TUV, TV, VW, LANES, 2>(a, s);
    if (ns <= 4) return launch_sddmm<TUV, TV, VW, LANES, 4>(a, s);
    if (ns <= 8) return launch_sddmm<TUV, TV, VW, LANES, 8>(a, s);
    return hipErrorInvalidValue;
}

template <typename TUV, typename TV, int VW>
static hipError_t dispatch_lanes(const SddmmArgs &a, hipStream_t s) {
    switch (a.lanes) {
    case 4: return dispatch_ns<TUV, TV, VW, 4>(a, s);
    case 8: return dispatch_ns<TUV, TV, VW, 8>(a, s);
    case 16: return dispatch_ns<TUV, TV, VW, 16>(a, s);
    case 32: return dispatch_ns<TUV, TV, VW, 32>(a, s);
    case 64: return dispatch_ns<TUV, TV, VW, 64>(a, s);
    default: return hipErrorInvalidValue;
    }
}

hipError_t sddmm_launch(const SddmmArgs &a, hipStream_t s) {
    switch (a.uv_dtype) {
    case SPK_F32: return a.vec > 1 ? dispatch_lanes<float, float, 4>(a, s) : dispatch_lanes<float, float, 1>(a, s);
    case SPK_BF16: return a.vec > 1 ? dispatch_lanes<bf16, float, 4>(a, s) : dispatch_lanes<bf16, float, 1>(a, s);
    case SPK_F64: return a.vec > 1 ? dispatch_lanes<double, double, 2>(a, s) : dispatch_lanes<double, double, 1>(a, s);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace spk
