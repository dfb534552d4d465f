// selector.hip - learned plan selection on the GPU (gfx950).
//
//   features   integer structural counts of a CSR pattern (row-length
//              histogram, lengths, bandwidth, 4x4-block count)
//   inputs     33 scaled inputs from the features, the dense width K and dtype
//   MLP        three affine layers with ReLU between them; one output per
//              plan of the op's plan list, predicting log(time / best time)
//   select     argmin of the outputs over the plans valid for K and dtype
//   training   batched forward, hand-derived backward of the masked mean
//              squared error, and Adam; every reduction runs in a fixed order,
//              so gradients are reproducible bit for bit
//
// The trained weights live in a small static device table per op (loaded by
// selector_load): plan_select allocates nothing.
#include <math.h>

#include "common.h"
#include "internal.h"

namespace spk {

constexpr int kNFeat = 28;
constexpr int kNIn = 33;
// 192 hidden units: room for the average of three 64-unit networks stacked
// into one (selector.merge_tables).
constexpr int kMaxIn = 64, kMaxHidden = 192, kMaxOut = 32;
constexpr int kTable = 2 * kMaxIn + kMaxHidden * kMaxIn + kMaxHidden + kMaxHidden * kMaxHidden + kMaxHidden +
                       kMaxOut * kMaxHidden + kMaxOut;

// Per op (SpMM, SDDMM): standardisation (mean, scale) of the inputs, then the
// MLP parameters in the order W1[H][F], b1[H], W2[H][H], b2[H], W3[P][H], b3[P].
__device__ float g_table[2][kTable];

struct Dims {
    int F, H, P;
};

__device__ __forceinline__ int params_count(Dims d) { return d.H * d.F + d.H + d.H * d.H + d.H + d.P * d.H + d.P; }

// ---------------------------------------------------------------- features
// f: 0 m, 1 n, 2 nnz, 3..22 row-length histogram (bin 0 empty rows, bin b =
// [2^(b-1), 2^b), bin 19 >= 2^18), 23 max length, 24 sum of squared lengths,
// 25 max |i - j|, 26 sum |i - j|, 27 nonempty 4x4 blocks.
// Grid-stride: a wave per row, rows t, t + stride, ...; each workgroup sums
// into LDS and adds to f once (a few thousand global atomics in all).
__global__ __launch_bounds__(kBlock) void features_rows_kernel(int64_t m, const int32_t *__restrict__ rp,
                                                               const int32_t *__restrict__ ci,
                                                               unsigned long long *__restrict__ f) {
    __shared__ unsigned long long acc[kNFeat];
    if (threadIdx.x < kNFeat) acc[threadIdx.x] = 0;
    __syncthreads();
    const int lane = threadIdx.x & (kWave - 1);
    const int64_t stride = static_cast<int64_t>(gridDim.x) * (kBlock / kWave);
    for (int64_t row = static_cast<int64_t>(blockIdx.x) * (kBlock / kWave) + threadIdx.x / kWave; row < m;
         row += stride) {
        const int64_t a = rp[row], b = rp[row + 1];
        unsigned long long bw = 0;
        for (int64_t p = a + lane; p < b; p += kWave) {
            const int64_t d = row - ci[p];
            bw += static_cast<unsigned long long>(d < 0 ? -d : d);
        }
#pragma unroll
        for (int s = kWave / 2; s >= 1; s >>= 1) bw += __shfl_xor(bw, s, kWave);
        if (lane == 0) {
            const int64_t L = b - a;
            int bin = 0;
            if (L > 0) {
                bin = 1;
                while (bin < 19 && L >= (int64_t(1) << bin)) ++bin;
            }
            atomicAdd(&acc[3 + bin], 1ull);
            atomicMax(&acc[23], static_cast<unsigned long long>(L));
            atomicAdd(&acc[24], static_cast<unsigned long long>(L * L));
            if (L > 0) {  // sorted columns: the extremes of |i - j| are at the row's ends
                const int64_t d0 = row - ci[a], d1 = row - ci[b - 1];
                const int64_t mx = max(d0 < 0 ? -d0 : d0, d1 < 0 ? -d1 : d1);
                atomicMax(&acc[25], static_cast<unsigned long long>(mx));
            }
            atomicAdd(&acc[26], bw);
        }
    }
    __syncthreads();
    if (threadIdx.x >= 3 && threadIdx.x < 27) {
        const int k = threadIdx.x;
        if (k == 23 || k == 25) atomicMax(&f[k], acc[k]);
        else atomicAdd(&f[k], acc[k]);
    }
}

__global__ void features_init_kernel(int64_t m, int64_t n, int64_t nnz, unsigned long long *__restrict__ f) {
    const int k = threadIdx.x;
    if (k >= kNFeat) return;
    f[k] = k == 0 ? static_cast<unsigned long long>(m) : k == 1 ? static_cast<unsigned long long>(n)
           : k == 2 ? static_cast<unsigned long long>(nnz) : 0ull;
}

// Number of nonempty 4x4 blocks into f[27].  Entry (i, j) opens block
// (i/4, j/4) when it is the first entry of row i in block column j/4 and no
// earlier row of the same block row holds a column in [4(j/4), 4(j/4)+4)
// (a binary search in each such row).  One wave per row (grid-stride),
// lanes over entries.
__global__ __launch_bounds__(kBlock) void features_blocks_kernel(int64_t m, const int32_t *__restrict__ rp,
                                                                 const int32_t *__restrict__ ci,
                                                                 unsigned long long *__restrict__ f) {
    __shared__ unsigned long long part[kBlock / kWave];
    const int lane = threadIdx.x & (kWave - 1);
    const int64_t stride = static_cast<int64_t>(gridDim.x) * (kBlock / kWave);
    unsigned long long s = 0;
    for (int64_t row = static_cast<int64_t>(blockIdx.x) * (kBlock / kWave) + threadIdx.x / kWave; row < m;
         row += stride) {
        const int64_t a = rp[row], b = rp[row + 1];
        const int64_t first_row = row & ~int64_t(3);
        for (int64_t p = a + lane; p < b; p += kWave) {
            const int32_t J = ci[p] >> 2;
            if (p > a && (ci[p - 1] >> 2) == J) continue;
            bool seen = false;
            for (int64_t r = first_row; r < row && !seen; ++r) {
                int64_t lo = rp[r], hi = rp[r + 1];  // first column >= 4J in row r
                while (lo < hi) {
                    const int64_t mid = (lo + hi) >> 1;
                    if (ci[mid] < 4 * J) lo = mid + 1; else hi = mid;
                }
                seen = lo < rp[r + 1] && ci[lo] < 4 * J + 4;
            }
            s += seen ? 0ull : 1ull;
        }
    }
#pragma unroll
    for (int o = kWave / 2; o >= 1; o >>= 1) s += __shfl_xor(s, o, kWave);
    if (lane == 0) part[threadIdx.x / kWave] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long t = 0;
        for (int w = 0; w < kBlock / kWave; ++w) t += part[w];
        atomicAdd(&f[27], t);
    }
}

// The same count with a bitmap of block columns in LDS: one workgroup per
// block row sets bit j/4 for every entry (i, j) of its four rows, then counts
// the set bits.  Used while the bitmap of n/4 bits fits kBitmapLds.
constexpr int64_t kBitmapLds = 65536;

__global__ __launch_bounds__(kBlock) void features_blocks_lds_kernel(int64_t m, int64_t n,
                                                                     const int32_t *__restrict__ rp,
                                                                     const int32_t *__restrict__ ci,
                                                                     unsigned long long *__restrict__ f) {
    extern __shared__ unsigned int bm[];
    __shared__ unsigned long long part[kBlock / kWave];
    const int64_t nwords = (n + 127) / 128;
    const int64_t nbr = (m + 3) / 4;
    unsigned long long s = 0;
    for (int64_t br = blockIdx.x; br < nbr; br += gridDim.x) {  // workgroup-uniform
        const int64_t r0 = br * 4;
        const int64_t r1 = r0 + 4 < m ? r0 + 4 : m;
        const int64_t a = rp[r0], b = rp[r1];
        if (a == b) continue;  // an empty block row has no blocks
        for (int64_t w = threadIdx.x; w < nwords; w += kBlock) bm[w] = 0u;
        __syncthreads();
        for (int64_t p = a + threadIdx.x; p < b; p += kBlock) {
            const uint32_t J = static_cast<uint32_t>(ci[p]) >> 2;
            atomicOr(&bm[J >> 5], 1u << (J & 31));
        }
        __syncthreads();
        for (int64_t w = threadIdx.x; w < nwords; w += kBlock) s += __popc(bm[w]);
        __syncthreads();  // the next block row clears the bitmap
    }
    const int lane = threadIdx.x & (kWave - 1);
#pragma unroll
    for (int o = kWave / 2; o >= 1; o >>= 1) s += __shfl_xor(s, o, kWave);
    if (lane == 0) part[threadIdx.x / kWave] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        unsigned long long t = 0;
        for (int w = 0; w < kBlock / kWave; ++w) t += part[w];
        atomicAdd(&f[27], t);
    }
}

// ---------------------------------------------------------------- inputs
__device__ void inputs_of(const long long *f, int64_t K, int32_t dtype, float *x) {
    const float m = static_cast<float>(f[0]), n = static_cast<float>(f[1]), nnz = static_cast<float>(f[2]);
    const float md = m > 0 ? m : 1.f, nd = n > 0 ? n : 1.f, zd = nnz > 0 ? nnz : 1.f;
    x[0] = log2f(1.f + m) / 20.f;
    x[1] = log2f(1.f + n) / 20.f;
    x[2] = log2f(1.f + nnz) / 30.f;
    for (int b = 0; b < 20; ++b) x[3 + b] = static_cast<float>(f[3 + b]) / md;
    const float mean = nnz / md;
    x[23] = log2f(1.f + static_cast<float>(f[23])) / 20.f;
    x[24] = log2f(1.f + mean) / 20.f;
    const float var = static_cast<float>(f[24]) / md - mean * mean;
    const float cv = mean > 0 ? sqrtf(var > 0 ? var : 0.f) / mean : 0.f;
    x[25] = log2f(1.f + cv) / 4.f;
    x[26] = log2f(1.f + static_cast<float>(f[25])) / 20.f;
    x[27] = (static_cast<float>(f[26]) / zd) / nd;
    x[28] = nnz / (16.f * (f[27] > 0 ? static_cast<float>(f[27]) : 1.f));
    x[29] = log2f(static_cast<float>(K > 0 ? K : 1)) / 8.f;
    const float dens = nnz / (md * nd);
    x[30] = 1.f + log10f(dens > 1e-12f ? dens : 1e-12f) / 5.f;
    x[31] = 1.f;
    x[32] = dtype == SPK_BF16 ? 1.f : 0.f;
}

__global__ void inputs_kernel(const long long *__restrict__ f, int64_t K, int32_t dtype, float *__restrict__ x) {
    if (threadIdx.x == 0) {
        float t[kNIn];
        inputs_of(f, K, dtype, t);
        for (int i = 0; i < kNIn; ++i) x[i] = t[i];
    }
}

// ---------------------------------------------------------------- MLP
// One workgroup of kMaxHidden threads evaluates one sample: x (F values in
// LDS) -> y (P values in LDS).  Affine sums run over inputs in index order.
__device__ void mlp_eval(const float *__restrict__ p, Dims d, const float *x, float *a1, float *a2, float *y) {
    const float *W1 = p, *b1 = W1 + d.H * d.F, *W2 = b1 + d.H, *b2 = W2 + d.H * d.H, *W3 = b2 + d.H;
    const float *b3 = W3 + d.P * d.H;
    const int t = threadIdx.x;
    if (t < d.H) {
        float z = b1[t];
        for (int i = 0; i < d.F; ++i) z = fmaf(W1[t * d.F + i], x[i], z);
        a1[t] = z > 0.f ? z : 0.f;
    }
    __syncthreads();
    if (t < d.H) {
        float z = b2[t];
        for (int i = 0; i < d.H; ++i) z = fmaf(W2[t * d.H + i], a1[i], z);
        a2[t] = z > 0.f ? z : 0.f;
    }
    __syncthreads();
    if (t < d.P) {
        float z = b3[t];
        for (int i = 0; i < d.H; ++i) z = fmaf(W3[t * d.H + i], a2[i], z);
        y[t] = z;
    }
    __syncthreads();
}

// Plans of an op that suit width K and dense dtype (mirrors the plan lists
// of plan_of_index in api.hip).
__device__ __host__ inline bool quad_fits(int32_t op, int64_t K, int32_t dtype) {
    const int64_t row = K * (dtype == SPK_BF16 ? 2 : 4);
    return row == 128 || row == 256 || (row == 512 && (op == SPK_OP_SDDMM || dtype == SPK_F32));
}

__device__ __host__ inline bool plan_valid(int32_t op, int idx, int64_t K, int32_t dtype) {
    const bool tile_ok = K >= 8 && K <= 256 && K % 8 == 0;  // LDS slabs: 16-byte pieces of F32 and BF16 rows
    if (dtype == SPK_F64 && idx >= 15) return false;  // block, slab, compressed forms: F32 and BF16 only
    if (op == SPK_OP_SPMM) {
        if (idx == 15) return true;                   // 4x4 blocks on matrix cores
        if (idx >= 16 && idx <= 24) return tile_ok;   // TILE (24: wide, 32 KiB slabs)
        if (idx == 25) return tile_ok && quad_fits(op, K, dtype);  // wide, 64 KiB slabs
        if (idx >= 26) return true;                   // column-slab form, doubly compressed rows
        const int lanes = 4 << (idx % 5);
        int64_t cap = 16;
        while (cap < K) cap <<= 1;
        return lanes == 4 || lanes * 4 <= 2 * cap;
    }
    if (idx >= 15 && idx <= 23) return tile_ok;  // TILE of V (23: wide, 32 KiB slabs)
    if (idx == 24) return tile_ok && quad_fits(op, K, dtype);
    if (idx >= 25 && idx <= 27) return true;  // column-slab form, doubly compressed rows
    if (idx == 28) return K <= 512;           // COO entries, 16 lanes: at most 8 slices of 64 columns
    const int lanes = 4 << (idx % 5);
    const int64_t ns = (K + lanes * 4 - 1) / (lanes * 4);
    return ns <= 8 && (lanes == 4 || lanes * 4 <= 2 * (K > 4 ? K : 4));
}

__global__ __launch_bounds__(kMaxHidden) void select_kernel(int32_t op, const long long *__restrict__ f, int64_t K,
                                                            int32_t dtype, Dims d, int32_t *__restrict__ out) {
    __shared__ float x[kMaxIn], a1[kMaxHidden], a2[kMaxHidden], y[kMaxOut];
    const float *tab = g_table[op];
    if (threadIdx.x == 0) {
        float t[kNIn];
        inputs_of(f, K, dtype, t);
        for (int i = 0; i < d.F; ++i) x[i] = (i < kNIn ? t[i] : 0.f);
    }
    __syncthreads();
    if (threadIdx.x < d.F) x[threadIdx.x] = (x[threadIdx.x] - tab[threadIdx.x]) / tab[kMaxIn + threadIdx.x];
    __syncthreads();
    mlp_eval(tab + 2 * kMaxIn, d, x, a1, a2, y);
    if (threadIdx.x == 0) {
        // the plans valid for K in ascending predicted time (ties: lower
        // index first), -1 after the last
        bool taken[kMaxOut];
        for (int p = 0; p < kMaxOut; ++p) taken[p] = false;
        for (int r = 0; r < kMaxOut; ++r) {
            int best = -1;
            for (int p = 0; p < d.P; ++p)
                if (!taken[p] && plan_valid(op, p, K, dtype) && (best < 0 || y[p] < y[best])) best = p;
            out[r] = best;
            if (best >= 0) taken[best] = true;
        }
    }
}

__global__ __launch_bounds__(kMaxHidden) void mlp_forward_kernel(const float *__restrict__ params, Dims d,
                                                                 const float *__restrict__ X, int64_t batch,
                                                                 float *__restrict__ Y) {
    __shared__ float x[kMaxIn], a1[kMaxHidden], a2[kMaxHidden], y[kMaxOut];
    const int64_t s = blockIdx.x;
    if (threadIdx.x < d.F) x[threadIdx.x] = X[s * d.F + threadIdx.x];
    __syncthreads();
    mlp_eval(params, d, x, a1, a2, y);
    if (threadIdx.x < d.P) Y[s * d.P + threadIdx.x] = y[threadIdx.x];
}

// ---------------------------------------------------------------- training
// Per-sample scratch: a1[H], a2[H], d1[H], d2[H], dy[P], loss term.
struct TrainLayout {
    int64_t stride;  // floats per sample
    int64_t a1, a2, d1, d2, dy, ls;
};
__host__ __device__ inline TrainLayout train_layout(Dims d) {
    TrainLayout L;
    L.a1 = 0;
    L.a2 = L.a1 + d.H;
    L.d1 = L.a2 + d.H;
    L.d2 = L.d1 + d.H;
    L.dy = L.d2 + d.H;
    L.ls = L.dy + d.P;
    L.stride = L.ls + 1;
    return L;
}

// Number of nonzero mask entries, summed in a fixed order (one workgroup).
__global__ __launch_bounds__(kBlock) void mask_count_kernel(const float *__restrict__ mask, int64_t count,
                                                            float *__restrict__ out) {
    __shared__ float part[kBlock];
    float s = 0.f;
    for (int64_t i = threadIdx.x; i < count; i += kBlock) s += mask[i] != 0.f ? 1.f : 0.f;
    part[threadIdx.x] = s;
    __syncthreads();
    for (int w = kBlock / 2; w >= 1; w >>= 1) {
        if (threadIdx.x < w) part[threadIdx.x] += part[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[0] = part[0];
}

// Forward and the backward deltas of one sample per workgroup.
__global__ __launch_bounds__(kMaxHidden) void mlp_delta_kernel(const float *__restrict__ params, Dims d,
                                                               const float *__restrict__ X, const float *__restrict__ T,
                                                               const float *__restrict__ mask,
                                                               const float *__restrict__ count,
                                                               float *__restrict__ scratch) {
    __shared__ float x[kMaxIn], a1[kMaxHidden], a2[kMaxHidden], y[kMaxOut], dy[kMaxOut], d2[kMaxHidden];
    const int64_t s = blockIdx.x;
    const TrainLayout L = train_layout(d);
    float *sc = scratch + s * L.stride;
    const float *W1 = params, *b1 = W1 + d.H * d.F, *W2 = b1 + d.H, *b2 = W2 + d.H * d.H, *W3 = b2 + d.H;
    (void)b2;
    const int t = threadIdx.x;
    if (t < d.F) x[t] = X[s * d.F + t];
    __syncthreads();
    mlp_eval(params, d, x, a1, a2, y);
    const float cnt = count[0];
    if (t < d.P) {
        const float w = mask[s * d.P + t];  // the mask's value weighs the term
        const float e = y[t] - T[s * d.P + t];
        dy[t] = cnt > 0.f ? w * e / cnt : 0.f;
        sc[L.dy + t] = dy[t];
    }
    __syncthreads();
    if (t == 0) {
        float l = 0.f;
        for (int p = 0; p < d.P; ++p) {
            const float w = mask[s * d.P + p];
            const float e = y[p] - T[s * d.P + p];
            l = fmaf(w * e, e, l);
        }
        sc[L.ls] = l;
    }
    if (t < d.H) {  // through layer 3, then ReLU of layer 2 (a2 > 0 iff z2 > 0)
        float g = 0.f;
        for (int p = 0; p < d.P; ++p) g = fmaf(W3[p * d.H + t], dy[p], g);
        d2[t] = a2[t] > 0.f ? g : 0.f;
        sc[L.a1 + t] = a1[t];
        sc[L.a2 + t] = a2[t];
        sc[L.d2 + t] = d2[t];
    }
    __syncthreads();
    if (t < d.H) {  // through layer 2, then ReLU of layer 1
        float g = 0.f;
        for (int o = 0; o < d.H; ++o) g = fmaf(W2[o * d.H + t], d2[o], g);
        sc[L.d1 + t] = a1[t] > 0.f ? g : 0.f;
    }
    (void)W1;
}

// One thread per parameter: its gradient summed over samples in order.
__global__ __launch_bounds__(kBlock) void mlp_grad_kernel(Dims d, const float *__restrict__ X, int64_t batch,
                                                          const float *__restrict__ scratch, float *__restrict__ grads) {
    const int64_t idx = static_cast<int64_t>(blockIdx.x) * kBlock + threadIdx.x;
    const TrainLayout L = train_layout(d);
    const int64_t nW1 = d.H * d.F, nW2 = d.H * d.H, nW3 = d.P * d.H;
    int64_t delta_off, in_off = -1;  // in_off < 0: bias, -2: input from X
    int o, i;
    int64_t r = idx;
    if (r < nW1) { o = r / d.F; i = r % d.F; delta_off = L.d1 + o; in_off = -2; }
    else if ((r -= nW1) < d.H) { o = r; i = 0; delta_off = L.d1 + o; }
    else if ((r -= d.H) < nW2) { o = r / d.H; i = r % d.H; delta_off = L.d2 + o; in_off = L.a1 + i; }
    else if ((r -= nW2) < d.H) { o = r; i = 0; delta_off = L.d2 + o; }
    else if ((r -= d.H) < nW3) { o = r / d.H; i = r % d.H; delta_off = L.dy + o; in_off = L.a2 + i; }
    else if ((r -= nW3) < d.P) { o = r; i = 0; delta_off = L.dy + o; }
    else return;
    float g = 0.f;
    for (int64_t s = 0; s < batch; ++s) {
        const float *sc = scratch + s * L.stride;
        const float in = in_off == -1 ? 1.f : in_off == -2 ? X[s * d.F + i] : sc[in_off];
        g = fmaf(sc[delta_off], in, g);
    }
    grads[idx] = g;
}

__global__ __launch_bounds__(kBlock) void mlp_loss_kernel(Dims d, int64_t batch, const float *__restrict__ scratch,
                                                          const float *__restrict__ count, float *__restrict__ loss) {
    __shared__ float part[kBlock];
    const TrainLayout L = train_layout(d);
    float s = 0.f;
    for (int64_t i = threadIdx.x; i < batch; i += kBlock) s += scratch[i * L.stride + L.ls];
    part[threadIdx.x] = s;
    __syncthreads();
    for (int w = kBlock / 2; w >= 1; w >>= 1) {
        if (threadIdx.x < w) part[threadIdx.x] += part[threadIdx.x + w];
        __syncthreads();
    }
    if (threadIdx.x == 0) loss[0] = count[0] > 0.f ? part[0] / (2.f * count[0]) : 0.f;
}

// Adam (Kingma and Ba, Algorithm 1) with bias-corrected moments.
__global__ void adam_kernel(float *__restrict__ w, const float *__restrict__ g, float *__restrict__ mom,
                            float *__restrict__ vel, int64_t count, float lr, float b1, float b2, float eps, float c1,
                            float c2) {
    const int64_t i = static_cast<int64_t>(blockIdx.x) * blockDim.x + threadIdx.x;
    if (i >= count) return;
    const float gi = g[i];
    const float mi = b1 * mom[i] + (1.f - b1) * gi;
    const float vi = b2 * vel[i] + (1.f - b2) * gi * gi;
    mom[i] = mi;
    vel[i] = vi;
    w[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

// ---------------------------------------------------------------- host side
size_t features_ws_bytes(int64_t m) {
    return align_up(sizeof(long long) * kNFeat) + align_up(sizeof(int32_t) * static_cast<size_t>((m + 3) / 4 + 1)) +
           align_up(sizeof(int32_t) * 4);
}

hipError_t features_launch(int64_t m, int64_t n, int64_t nnz, const int32_t *rp, const int32_t *ci, int64_t *f,
                           void *ws, hipStream_t s) {
    unsigned long long *uf = reinterpret_cast<unsigned long long *>(f);
    hipLaunchKernelGGL(features_init_kernel, dim3(1), dim3(64), 0, s, m, n, nnz, uf);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || m == 0) return e;
    // grid-stride launches of at most kFeatureBlocks workgroups
    constexpr int64_t kFeatureBlocks = 2048;
    const int64_t rows_wg = (m + (kBlock / kWave) - 1) / (kBlock / kWave);
    const unsigned nb = static_cast<unsigned>(rows_wg < kFeatureBlocks ? rows_wg : kFeatureBlocks);
    hipLaunchKernelGGL(features_rows_kernel, dim3(nb), dim3(kBlock), 0, s, m, rp, ci, uf);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    (void)ws;
    const int64_t bm_bytes = (n + 127) / 128 * 4;
    const int64_t nbr = (m + 3) / 4;
    if (bm_bytes <= kBitmapLds) {
        const unsigned nbb = static_cast<unsigned>(nbr < kFeatureBlocks ? nbr : kFeatureBlocks);
        hipLaunchKernelGGL(features_blocks_lds_kernel, dim3(nbb), dim3(kBlock), static_cast<size_t>(bm_bytes), s, m,
                           n, rp, ci, uf);
    } else {
        hipLaunchKernelGGL(features_blocks_kernel, dim3(nb), dim3(kBlock), 0, s, m, rp, ci, uf);
    }
    return hipGetLastError();
}

hipError_t inputs_launch(const int64_t *f, int64_t K, int32_t dtype, float *x, hipStream_t s) {
    hipLaunchKernelGGL(inputs_kernel, dim3(1), dim3(64), 0, s, reinterpret_cast<const long long *>(f), K, dtype, x);
    return hipGetLastError();
}

bool mlp_dims_ok(int64_t F, int64_t H, int64_t P) {
    return F >= 1 && F <= kMaxIn && H >= 1 && H <= kMaxHidden && P >= 1 && P <= kMaxOut;
}

hipError_t mlp_forward_launch(const float *params, int64_t F, int64_t H, int64_t P, const float *X, int64_t batch,
                              float *Y, hipStream_t s) {
    if (batch == 0) return hipSuccess;
    Dims d{static_cast<int>(F), static_cast<int>(H), static_cast<int>(P)};
    hipLaunchKernelGGL(mlp_forward_kernel, dim3(static_cast<unsigned>(batch)), dim3(kMaxHidden), 0, s, params, d, X,
                       batch, Y);
    return hipGetLastError();
}

size_t mlp_train_ws_bytes(int64_t F, int64_t H, int64_t P, int64_t batch) {
    Dims d{static_cast<int>(F), static_cast<int>(H), static_cast<int>(P)};
    return align_up(sizeof(float) * 4) + align_up(sizeof(float) * static_cast<size_t>(train_layout(d).stride * batch));
}

hipError_t mlp_loss_grad_launch(const float *params, int64_t F, int64_t H, int64_t P, const float *X, const float *T,
                                const float *mask, int64_t batch, float *grads, float *loss, void *ws, hipStream_t s) {
    Dims d{static_cast<int>(F), static_cast<int>(H), static_cast<int>(P)};
    float *count = static_cast<float *>(ws);
    float *scratch = reinterpret_cast<float *>(static_cast<char *>(ws) + align_up(sizeof(float) * 4));
    hipLaunchKernelGGL(mask_count_kernel, dim3(1), dim3(kBlock), 0, s, mask, batch * P, count);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    if (batch > 0) {
        hipLaunchKernelGGL(mlp_delta_kernel, dim3(static_cast<unsigned>(batch)), dim3(kMaxHidden), 0, s, params, d, X,
                           T, mask, count, scratch);
        if ((e = hipGetLastError()) != hipSuccess) return e;
    }
    const int64_t np = H * F + H + H * H + H + P * H + P;
    hipLaunchKernelGGL(mlp_grad_kernel, dim3(static_cast<unsigned>((np + kBlock - 1) / kBlock)), dim3(kBlock), 0, s, d,
                       X, batch, scratch, grads);
    if ((e = hipGetLastError()) != hipSuccess) return e;
    hipLaunchKernelGGL(mlp_loss_kernel, dim3(1), dim3(kBlock), 0, s, d, batch, scratch, count, loss);
    return hipGetLastError();
}

hipError_t adam_launch(float *w, const float *g, float *mom, float *vel, int64_t count, float lr, float b1, float b2,
                       float eps, int64_t step, hipStream_t s) {
    if (count == 0) return hipSuccess;
    const float c1 = 1.f - powf(b1, static_cast<float>(step));
    const float c2 = 1.f - powf(b2, static_cast<float>(step));
    hipLaunchKernelGGL(adam_kernel, dim3(static_cast<unsigned>((count + kBlock - 1) / kBlock)), dim3(kBlock), 0, s, w,
                       g, mom, vel, count, lr, b1, b2, eps, c1, c2);
    return hipGetLastError();
}

hipError_t selector_table_load(int32_t op, const float *host_table, int64_t F, int64_t H, int64_t P) {
    // mean[F] and scale[F] go to the two kMaxIn-sized slots, the parameters after them
    float staging[kTable];
    for (int i = 0; i < kTable; ++i) staging[i] = 0.f;
    for (int i = 0; i < kMaxIn; ++i) staging[kMaxIn + i] = 1.f;
    for (int64_t i = 0; i < F; ++i) {
        staging[i] = host_table[i];
        staging[kMaxIn + i] = host_table[F + i];
    }
    const int64_t np = H * F + H + H * H + H + P * H + P;
    for (int64_t i = 0; i < np; ++i) staging[2 * kMaxIn + i] = host_table[2 * F + i];
    return hipMemcpyToSymbol(HIP_SYMBOL(g_table), staging, sizeof(staging), sizeof(staging) * op, hipMemcpyHostToDevice);
}

hipError_t select_launch(int32_t op, const int64_t *f, int64_t K, int32_t dtype, int64_t F, int64_t H, int64_t P,
                         int32_t *out, hipStream_t s) {
    Dims d{static_cast<int>(F), static_cast<int>(H), static_cast<int>(P)};
    hipLaunchKernelGGL(select_kernel, dim3(1), dim3(kMaxHidden), 0, s, op, reinterpret_cast<const long long *>(f), K,
                       dtype, d, out);
    return hipGetLastError();
}

bool plan_valid_host(int32_t op, int idx, int64_t K, int32_t dtype) { return plan_valid(op, idx, K, dtype); }

}  // namespace spk
