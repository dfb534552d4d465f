// tile.h - pieces shared by the LDS-slab (TILE) kernels of SpMM and SDDMM:
// copies of a slab of a dense operand through registers into LDS, the
// chunked reading of a row's entries, and the DPP row broadcast.
#pragma once
#include "common.h"

namespace spk {

template <typename TB> constexpr int kTileSV = 16 / sizeof(TB);
constexpr int kTilePiece = kBlock * 16;  // bytes one copy round of a workgroup moves (4 KiB)
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

// Copy of a slab [c0, c0 + w) of B as [w][K] pieces of 16 bytes: thread t
// of a BS-thread workgroup moves pieces t + i * BS.  Indices past the slab are clamped to its last
// piece, so every thread always issues NPT loads; their copies land in the
// buffer's tail beyond the slab (a buffer holds NPT * 4 KiB).  The pieces'
// byte offsets from the slab's first row depend only on the slab width, so
// they are computed once per width; they fit 32 bits (the API admits TILE
// plans only when a slab spans less than 4 GiB of B), so every slab's loads
// are the uniform slab base plus a 32-bit offset, with no address arithmetic.
template <typename TB, int NPT, int BS = kBlock>
struct TileCopy {
    uint32_t off[NPT];

    __device__ __forceinline__ void layout(int w, int per_row, int64_t ldb) {
        const int items = w * per_row;
#pragma unroll
        for (int i = 0; i < NPT; ++i) {
            const int idx0 = static_cast<int>(threadIdx.x) + i * BS;
            const int idx = idx0 < items ? idx0 : items - 1;
            const int rr = idx / per_row;
            off[i] = static_cast<uint32_t>((rr * ldb + (idx - rr * per_row) * kTileSV<TB>) * sizeof(TB));
        }
    }

    __device__ __forceinline__ void load(const TB *__restrict__ B, int64_t ldb, int64_t c0,
                                         u32x4 (&stg)[NPT]) const {
        const unsigned char *base = reinterpret_cast<const unsigned char *>(B + c0 * ldb);
#pragma unroll
        for (int i = 0; i < NPT; ++i) stg[i] = *reinterpret_cast<const u32x4 *>(base + off[i]);
    }
};

template <typename TB, int NPT, int BS = kBlock>
__device__ __forceinline__ void tile_store(TB *dst, const u32x4 (&stg)[NPT]) {
#pragma unroll
    for (int i = 0; i < NPT; ++i)
        *reinterpret_cast<u32x4 *>(dst + (static_cast<int>(threadIdx.x) + i * BS) * kTileSV<TB>) = stg[i];
}

// Next chunk of one row: the lane reads entry p (its position in the chunk
// is fixed by the caller).  Positions are 32-bit (row_ptr is int32).  The
// index is clamped to the last entry of the matrix so both loads are always
// issued; whether the entry belongs to the row, and whether a value array
// exists (else vsrc aliases the column array and the weight is 1), is decided
// where the chunk is used.
template <typename TV>
__device__ __forceinline__ void tile_fetch(int32_t p, int32_t last, const int32_t *__restrict__ ci,
                                           const TV *__restrict__ vsrc, int &c, TV &v) {
    const uint32_t q = static_cast<uint32_t>(p < last ? p : last);
    c = ci[q];
    v = vsrc[q];
}

// A value held in a register from here on.  Used for a chunk entry's weight
// before the next chunk's fetch overwrites the entry: left to itself, the
// compiler may move the weight's use past the fetch, which then needs a
// second register and a copy back that waits for the load to arrive.
__device__ __forceinline__ float pin(float x) {
    asm volatile("" : "+v"(x));
    return x;
}

// row_newbcast:N (DPP control 0x150 + N): every lane of a 16-lane row reads
// lane N of the same row.  A VALU move; no LDS crossbar traffic.  Every lane
// has a valid source and all rows and banks are written, so the move needs no
// prior value (mov_dpp, unlike update_dpp with an old value, adds no
// zeroing move).
template <int N>
__device__ __forceinline__ int row_bcast(int v) {
    return __builtin_amdgcn_mov_dpp(v, 0x150 + N, 0xF, 0xF, false);
}
template <int N>
__device__ __forceinline__ float row_bcast(float v) {
    return __int_as_float(row_bcast<N>(__float_as_int(v)));
}

// Number of set lanes of a ballot among the 16 lanes starting at gbase (a
// multiple of 16): a 32-bit count on the ballot's half that holds them.
__device__ __forceinline__ int count16(uint64_t ballot, int gbase) {
    const uint32_t half = static_cast<uint32_t>(gbase < 32 ? ballot : ballot >> 32);
    return __popc(half & (0xFFFFu << (gbase & 31)));
}

// An LDS byte address: lane N's row offset (bytes) plus this lane's own base.
// Written as broadcast-then-add, the compiler folds the broadcast into the
// add (v_add_u32_dpp): one instruction per entry.  bound_ctrl (all sources
// are valid here anyway) lets the move go without a prior value.
template <int N>
__device__ __forceinline__ uint32_t row_bcast_add(int offb, uint32_t base) {
    return static_cast<uint32_t>(__builtin_amdgcn_update_dpp(0, offb, 0x150 + N, 0xF, 0xF, true)) + base;
}

// quad_perm [S,S,S,S] (DPP control 0x55 * S): every lane of a 4-lane quad
// reads lane S of the quad.  As with row_bcast_add, the broadcast of a row
// offset is folded into the add of this lane's own offset.
template <int S>
__device__ __forceinline__ uint32_t quad_bcast_add(int offb, uint32_t base) {
    return static_cast<uint32_t>(__builtin_amdgcn_update_dpp(0, offb, S * 0x55, 0xF, 0xF, true)) + base;
}
template <int S>
__device__ __forceinline__ float quad_bcast(float v) {
    return __int_as_float(__builtin_amdgcn_mov_dpp(__float_as_int(v), S * 0x55, 0xF, 0xF, false));
}

// The 64-byte group of a row that quad q reads in read i of a step, when a
// lane covers NP pieces of 16 bytes: (i + q) mod NP for NP <= 4; for NP = 8
// the rotation stays within each half of the row, (i + q) mod 4 + 4 (i / 4),
// so that the group a quad holds in register i depends on q only mod 4, the
// way the four quads of a 16-lane row are numbered.  In every read the four
// quads of a row take four different groups (different LDS banks).
template <int NP>
__device__ __forceinline__ int quad_group(int i, int q) {
    if constexpr (NP <= 4) return (i + q) % NP;
    else return (i + q) % 4 + 4 * (i / 4);
}

}  // namespace spk
