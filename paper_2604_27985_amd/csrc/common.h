// common.h - device helpers shared by the library's HIP kernels (gfx950).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/spk.h"

namespace spk {

constexpr int kWave = 64;          // CDNA wavefront width
constexpr int kBlock = 256;        // threads per workgroup (4 waves)
constexpr int kXcds = 8;           // MI355X: 8 accelerator complex dies, own L2 each
constexpr int kDefaultChunk = 256; // merge-path / SDDMM items per group
constexpr size_t kTileLds = 65536; // LDS bytes of one staged slab (TILE variants)

// bfloat16 storage type: the upper half of a binary32 pattern.
struct bf16 {
    uint16_t bits;
};

// Accumulator type: binary64 operands accumulate in binary64, everything
// else in binary32.
template <typename T> struct acc_of { using type = float; };
template <> struct acc_of<double> { using type = double; };

// Exact widening of bf16 -> f32: shift the 16 stored bits into the top half.
__device__ __forceinline__ float bf16_lo(uint32_t w) { return __uint_as_float(w << 16); }
__device__ __forceinline__ float bf16_hi(uint32_t w) { return __uint_as_float(w & 0xFFFF0000u); }

// Load VW consecutive elements starting at p (p aligned to VW elements when
// VW > 1) and widen them to the accumulator type.
template <typename T, int VW> struct vec_load;

template <> struct vec_load<float, 1> {
    __device__ __forceinline__ static void run(const float *p, float *o) { o[0] = *p; }
};
template <> struct vec_load<float, 4> {
    __device__ __forceinline__ static void run(const float *p, float *o) {
        float4 v = *reinterpret_cast<const float4 *>(p);
        o[0] = v.x; o[1] = v.y; o[2] = v.z; o[3] = v.w;
    }
};
template <> struct vec_load<bf16, 1> {
    __device__ __forceinline__ static void run(const bf16 *p, float *o) {
        o[0] = __uint_as_float(static_cast<uint32_t>(p->bits) << 16);
    }
};
template <> struct vec_load<bf16, 4> {
    __device__ __forceinline__ static void run(const bf16 *p, float *o) {
        uint2 w = *reinterpret_cast<const uint2 *>(p);
        o[0] = bf16_lo(w.x); o[1] = bf16_hi(w.x); o[2] = bf16_lo(w.y); o[3] = bf16_hi(w.y);
    }
};
template <> struct vec_load<bf16, 8> {
    __device__ __forceinline__ static void run(const bf16 *p, float *o) {
        uint4 w = *reinterpret_cast<const uint4 *>(p);
        o[0] = bf16_lo(w.x); o[1] = bf16_hi(w.x); o[2] = bf16_lo(w.y); o[3] = bf16_hi(w.y);
        o[4] = bf16_lo(w.z); o[5] = bf16_hi(w.z); o[6] = bf16_lo(w.w); o[7] = bf16_hi(w.w);
    }
};
template <> struct vec_load<double, 1> {
    __device__ __forceinline__ static void run(const double *p, double *o) { o[0] = *p; }
};
template <> struct vec_load<double, 2> {
    __device__ __forceinline__ static void run(const double *p, double *o) {
        double2 v = *reinterpret_cast<const double2 *>(p);
        o[0] = v.x; o[1] = v.y;
    }
};

// Store VW accumulator values at p (aligned when VW > 1).
template <typename T, int VW> struct vec_store {
    __device__ __forceinline__ static void run(T *p, const T *v) {
#pragma unroll
        for (int i = 0; i < VW; ++i) p[i] = v[i];
    }
};
template <> struct vec_store<float, 4> {
    __device__ __forceinline__ static void run(float *p, const float *v) {
        *reinterpret_cast<float4 *>(p) = make_float4(v[0], v[1], v[2], v[3]);
    }
};
template <> struct vec_store<float, 8> {
    __device__ __forceinline__ static void run(float *p, const float *v) {
        reinterpret_cast<float4 *>(p)[0] = make_float4(v[0], v[1], v[2], v[3]);
        reinterpret_cast<float4 *>(p)[1] = make_float4(v[4], v[5], v[6], v[7]);
    }
};
template <> struct vec_store<double, 2> {
    __device__ __forceinline__ static void run(double *p, const double *v) {
        *reinterpret_cast<double2 *>(p) = make_double2(v[0], v[1]);
    }
};

// Read a 32-bit value from another lane of the wave (ds_bpermute: an LDS
// crossbar operation that touches no LDS memory).
__device__ __forceinline__ int lane_read(int v, int src_lane) {
    return __builtin_amdgcn_ds_bpermute(src_lane << 2, v);
}
__device__ __forceinline__ float lane_read(float v, int src_lane) {
    return __int_as_float(__builtin_amdgcn_ds_bpermute(src_lane << 2, __float_as_int(v)));
}
__device__ __forceinline__ double lane_read(double v, int src_lane) {
    int lo = __builtin_amdgcn_ds_bpermute(src_lane << 2, __double2loint(v));
    int hi = __builtin_amdgcn_ds_bpermute(src_lane << 2, __double2hiint(v));
    return __hiloint2double(hi, lo);
}

// Butterfly sum over aligned groups of G lanes (G a power of two <= 64);
// every lane of the group ends with the group total.
template <int G, typename T> __device__ __forceinline__ T group_sum(T v) {
    const int lane = threadIdx.x & (kWave - 1);
#pragma unroll
    for (int s = G / 2; s >= 1; s >>= 1) v += lane_read(v, lane ^ s);
    return v;
}

// A dispatch counts the work-items of each grid dimension (blocks times
// threads per block) in 32 bits.  Launchers check their block count with this
// and return kGridTooLarge, which the ABI reports as a size error, rather than
// hand the runtime a grid it refuses.
constexpr hipError_t kGridTooLarge = hipErrorInvalidConfiguration;
inline bool grid_fits(int64_t blocks, int threads) {
    return blocks >= 0 && blocks <= static_cast<int64_t>(0xFFFFFFFFu) / threads;
}

// Kernels that give one wave to each row stride over the rows past their
// grid: at most 2^16 workgroups (2^24 threads), which fill the chip many
// times over and stay far below that count for any row count.
inline unsigned wave_rows_grid(int64_t rows) {
    const int64_t nb = (rows + kBlock / kWave - 1) / (kBlock / kWave);
    return static_cast<unsigned>(nb < 65536 ? nb : 65536);
}

// Workgroups are dispatched to the 8 XCDs round-robin.  Renumber them so
// that each XCD works on one contiguous range of logical blocks: rows that
// are close together (and, for banded or clustered patterns, the dense rows
// they gather) then share that XCD's L2.
__device__ __forceinline__ int xcd_block(int bid, int nblocks) {
    const int q = nblocks / kXcds, r = nblocks % kXcds;
    const int x = bid % kXcds, k = bid / kXcds;
    return x * q + (x < r ? x : r) + k;
}

// Largest i in [lo, hi] with key(i) <= target for a nondecreasing key.
template <typename F> __device__ __forceinline__ int64_t last_at_most(int64_t lo, int64_t hi, int64_t target, F key) {
    while (lo < hi) {
        int64_t mid = (lo + hi + 1) >> 1;
        if (key(mid) <= target) lo = mid; else hi = mid - 1;
    }
    return lo;
}

}  // namespace spk
