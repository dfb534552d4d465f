// bsr.hip - 4x4 block-sparse SpMM on matrix cores (gfx950), and the CSR ->
// 4x4-block conversion it needs.
//
// Where A really holds dense 4x4 tiles, C = A B is a sum of dense 4x4 x 4xK
// products: C[4I:4I+4, :] += A_IJ B[4J:4J+4, :].  One wave owns a block row
// (four rows of C) and a slice of 64*VW columns.  For each block and each of
// its four columns k, v_mfma_f32_4x4x1_16b_f32 (16 independent 4x4x1 outer
// products) adds A_IJ[:, k] (x) B[4J+k, cols] for 64 columns at once: in MFMA
// block b, row i is block-row row i and column j is dense column 4b + j.  Each
// element of B that is read feeds four output rows, so the gather traffic per
// stored value is a quarter of the CSR kernels', and the products run on the
// matrix cores.  With VW = 4 each lane reads 16 bytes of a B row and feeds four
// MFMAs (one per component), covering 256 columns per wave.
//
// Values stay FP32 (BF16 dense operands are widened exactly in registers), so
// the precision matches the CSR kernels.
#include "common.h"
#include "internal.h"

namespace spk {

typedef float f32x4 __attribute__((ext_vector_type(4)));

// ---------------------------------------------------------------- conversion
// One thread per block row merges the (up to four) sorted rows by block
// column.  Count pass (b_col == nullptr): number of distinct block columns.
// Fill pass: block columns ascending, and the 4x4 value tiles (zeros where A
// has no entry; F32 values or ones in pattern mode).
template <bool FILL>
__global__ void bsr4_merge_kernel(int64_t m, int64_t mb, const int32_t *__restrict__ rp, const int32_t *__restrict__ ci,
                                  const float *__restrict__ vals, const int32_t *__restrict__ b_rp,
                                  int32_t *__restrict__ counts, int32_t *__restrict__ b_col, float *__restrict__ b_vals) {
    const int64_t I = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (I >= mb) return;
    int64_t cur[4], end[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int64_t row = I * 4 + r;
        cur[r] = row < m ? rp[row] : 0;
        end[r] = row < m ? rp[row + 1] : 0;
    }
    int64_t q = FILL ? b_rp[I] : 0;
    int32_t cnt = 0;
    while (true) {
        int32_t J = 0x7FFFFFFF;
#pragma unroll
        for (int r = 0; r < 4; ++r)
            if (cur[r] < end[r]) J = min(J, ci[cur[r]] >> 2);
        if (J == 0x7FFFFFFF) break;
        if (FILL) {
            float tile[16];
#pragma unroll
            for (int e = 0; e < 16; ++e) tile[e] = 0.f;
#pragma unroll
            for (int r = 0; r < 4; ++r)
                while (cur[r] < end[r] && (ci[cur[r]] >> 2) == J) {
                    tile[r * 4 + (ci[cur[r]] & 3)] = vals ? vals[cur[r]] : 1.f;
                    ++cur[r];
                }
            b_col[q] = J;
#pragma unroll
            for (int e = 0; e < 16; ++e) b_vals[q * 16 + e] = tile[e];
            ++q;
        } else {
#pragma unroll
            for (int r = 0; r < 4; ++r)
                while (cur[r] < end[r] && (ci[cur[r]] >> 2) == J) ++cur[r];
        }
        ++cnt;
    }
    if (!FILL) counts[I] = cnt;
}

// ---------------------------------------------------------------- SpMM
template <typename TB, int VW>
__global__ __launch_bounds__(kBlock) void spmm_bsr4_kernel(int64_t m, int64_t n, int64_t mb, int K,
                                                           const int32_t *__restrict__ b_rp,
                                                           const int32_t *__restrict__ b_col,
                                                           const float *__restrict__ b_vals,
                                                           const TB *__restrict__ B, int64_t ldb,
                                                           float *__restrict__ C, int64_t ldc) {
    constexpr int WPB = kBlock / kWave;
    const int lane = threadIdx.x & (kWave - 1);
    const int64_t blk = xcd_block(blockIdx.x, gridDim.x);
    const int64_t I = blk * WPB + threadIdx.x / kWave;  // block row of this wave
    if (I >= mb) return;
    const int kcol = blockIdx.y * (kWave * VW) + lane * VW;  // first dense column of this lane
    const bool kvalid = kcol < K;
    const int koff = kvalid ? kcol : 0;
    const int i = lane & 3;  // row of the 4x4 tile this lane supplies to the A operand
    f32x4 acc[VW];
#pragma unroll
    for (int t = 0; t < VW; ++t) acc[t] = f32x4{0.f, 0.f, 0.f, 0.f};
    const int64_t q0 = b_rp[I], q1 = b_rp[I + 1];
    for (int64_t q = q0; q < q1; ++q) {
        const int64_t J = b_col[q];  // wave-uniform
        const float4 arow = *reinterpret_cast<const float4 *>(b_vals + q * 16 + i * 4);
        const float a[4] = {arow.x, arow.y, arow.z, arow.w};
        float bv[4][VW];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            // rows past n only meet zero tile entries; read a valid row instead
            const int64_t brow = J * 4 + k < n ? J * 4 + k : n - 1;
            vec_load<TB, VW>::run(B + brow * ldb + koff, bv[k]);
        }
#pragma unroll
        for (int k = 0; k < 4; ++k)
#pragma unroll
            for (int t = 0; t < VW; ++t) acc[t] = __builtin_amdgcn_mfma_f32_4x4x1f32(a[k], bv[k][t], acc[t], 0, 0, 0);
    }
    if (!kvalid) return;
    // acc[t][r] holds C[4I + r][kcol + t]
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        const int64_t row = I * 4 + r;
        if (row >= m) break;
        float out[VW];
#pragma unroll
        for (int t = 0; t < VW; ++t) out[t] = acc[t][r];
        vec_store<float, VW>::run(C + row * ldc + kcol, out);
    }
}

// ---------------------------------------------------------------- launchers
static unsigned grid1(int64_t count, int per) { return static_cast<unsigned>((count + per - 1) / per); }

hipError_t bsr4_count_launch(int64_t m, const int32_t *rp, const int32_t *ci, int32_t *counts, hipStream_t s) {
    const int64_t mb = (m + 3) / 4;
    if (mb == 0) return hipSuccess;
    hipLaunchKernelGGL((bsr4_merge_kernel<false>), dim3(grid1(mb, 128)), dim3(128), 0, s, m, mb, rp, ci, nullptr,
                       nullptr, counts, nullptr, nullptr);
    return hipGetLastError();
}

hipError_t bsr4_fill_launch(int64_t m, const int32_t *rp, const int32_t *ci, const float *vals, const int32_t *b_rp,
                            int32_t *b_col, float *b_vals, hipStream_t s) {
    const int64_t mb = (m + 3) / 4;
    if (mb == 0) return hipSuccess;
    hipLaunchKernelGGL((bsr4_merge_kernel<true>), dim3(grid1(mb, 128)), dim3(128), 0, s, m, mb, rp, ci, vals, b_rp,
                       nullptr, b_col, b_vals);
    return hipGetLastError();
}

template <typename TB, int VW>
static hipError_t launch_bsr(const Bsr4Args &a, hipStream_t s) {
    const int64_t mb = (a.m + 3) / 4;
    const int64_t nb = (mb + (kBlock / kWave) - 1) / (kBlock / kWave);
    const int64_t ktiles = (a.K + kWave * VW - 1) / (kWave * VW);
    if (!grid_fits(nb, kBlock)) return kGridTooLarge;
    if (ktiles > 65535) return hipErrorInvalidValue;
    hipLaunchKernelGGL((spmm_bsr4_kernel<TB, VW>), dim3(static_cast<unsigned>(nb), static_cast<unsigned>(ktiles)),
                       dim3(kBlock), 0, s, a.m, a.n, mb, static_cast<int>(a.K), a.b_rp, a.b_col, a.b_vals,
                       static_cast<const TB *>(a.B), a.ldb, a.C, a.ldc);
    return hipGetLastError();
}

hipError_t bsr4_spmm_launch(const Bsr4Args &a, hipStream_t s) {
    if (a.b_dtype == SPK_BF16) return a.vec == 4 ? launch_bsr<bf16, 4>(a, s) : launch_bsr<bf16, 1>(a, s);
    return a.vec == 4 ? launch_bsr<float, 4>(a, s) : launch_bsr<float, 1>(a, s);
}

}  // namespace spk
