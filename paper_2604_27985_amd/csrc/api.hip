// api.hip - the library's C ABI: O(1) argument checks, plan defaults and
// dispatch to the HIP kernels.  Nothing here allocates device memory.
#include <stdint.h>

#include <mutex>

#include "common.h"
#include "internal.h"

using namespace spk;

namespace {

constexpr int64_t kMaxIndex = 0x7FFFFFFF;
constexpr int32_t kRankSlots = 32;  // plans a ranking can hold (the network's output limit)

bool valid_lanes(int32_t l) { return l == 4 || l == 8 || l == 16 || l == 32 || l == 64; }

int32_t check_csr(const spk_csr *A) {
    if (!A) return SPK_ERR_NULL;
    if (A->m < 0 || A->n < 0 || A->nnz < 0) return SPK_ERR_SIZE;
    if (A->m > kMaxIndex || A->n > kMaxIndex || A->nnz > kMaxIndex) return SPK_ERR_SIZE;
    if (A->m > 0 && !A->row_ptr) return SPK_ERR_NULL;
    if (A->nnz > 0 && !A->col_idx) return SPK_ERR_NULL;
    if (A->vals && A->vals_dtype != SPK_F32 && A->vals_dtype != SPK_F64) return SPK_ERR_DTYPE;
    return SPK_OK;
}

bool aligned(const void *p, size_t bytes) { return (reinterpret_cast<uintptr_t>(p) % bytes) == 0; }

size_t elem_size(int32_t dt) { return dt == SPK_F64 ? 8 : dt == SPK_BF16 ? 2 : 4; }

// Dense-operand dtype must match the values' dtype family: F64 with F64,
// F32 or BF16 operands with F32 (or absent) values.
int32_t check_dtypes(const spk_csr *A, int32_t dense) {
    if (dense != SPK_F32 && dense != SPK_BF16 && dense != SPK_F64) return SPK_ERR_DTYPE;
    if (A->vals) {
        if ((dense == SPK_F64) != (A->vals_dtype == SPK_F64)) return SPK_ERR_DTYPE;
    }
    return SPK_OK;
}

// Elements per lane of the vector path for a dense dtype.
int32_t native_vec(int32_t dt) { return dt == SPK_F64 ? 2 : 4; }

struct Resolved {
    int32_t variant, lanes, vec;
    int64_t chunk;
    int32_t rows_per_group = 4;
    int32_t quad_split = 0;
};

// LDS for the two slab buffers of a TILE plan: 64 KiB, or 128 KiB for the
// wide quad plans (flags bit 3), whose slabs above 32 KiB run in 1024-thread
// workgroups, one per CU.
int64_t tile_lds_budget(const Resolved &r, int64_t) {
    return r.quad_split && r.rows_per_group == 2 ? 2 * static_cast<int64_t>(kTileLds)
                                                 : static_cast<int64_t>(kTileLds);
}

int32_t default_spmm_lanes(int64_t K) {
    int32_t l = 4;
    while (l < 64 && l * 4 < K) l <<= 1;
    return l;
}

// Default slab width: the power of two (>= 256) whose slab of the dense
// operand takes at most 2 MiB, half of one XCD's L2.
int64_t default_slab_width(int64_t K, size_t es) {
    const int64_t row_bytes = (K > 0 ? K : 1) * static_cast<int64_t>(es);
    int64_t w = 256;
    while (w * 2 * row_bytes <= (int64_t(2) << 20)) w *= 2;
    return w;
}

// The TILE kernels read a row's entries in chunks at 32-bit positions (the
// row's current position plus up to 63 lanes), so they take nnz up to
// 2^31 - 65; the other variants hold positions in 64 bits.
constexpr int64_t kTileMaxNnz = kMaxIndex - 64;
int32_t tile_nnz_ok(const Resolved &r, int64_t nnz) {
    return r.variant == SPK_VAR_TILE && nnz > kTileMaxNnz ? SPK_ERR_SIZE : SPK_OK;
}

int32_t resolve_spmm(const spk_plan *plan, int64_t K, int32_t b_dtype, const void *B, int64_t ldb, const void *C,
                     int64_t ldc, Resolved &r) {
    r.variant = plan ? plan->variant : SPK_VAR_ROWS;
    r.lanes = plan ? plan->lanes : default_spmm_lanes(K);
    if (r.variant != SPK_VAR_ROWS && r.variant != SPK_VAR_MERGE && r.variant != SPK_VAR_SLAB &&
        r.variant != SPK_VAR_TILE)
        return SPK_ERR_PLAN;
    if (!valid_lanes(r.lanes)) return SPK_ERR_PLAN;
    if (r.variant == SPK_VAR_TILE) {
        // one K-tile of 16-byte (F32) or 8-byte (BF16) lanes; the slab fits kTileLds
        const size_t es = elem_size(b_dtype);
        const int64_t sv = 16 / static_cast<int64_t>(es);
        if (b_dtype == SPK_F64 || (plan && (plan->flags & ~14)) || (plan && plan->chunk < 0)) return SPK_ERR_PLAN;
        r.rows_per_group = plan && (plan->flags & 2) ? 8 : 4;
        const int64_t row_bytes = K * static_cast<int64_t>(es);
        // one entry per quad where a row of B is 128 or 256 bytes (16-lane
        // groups whatever the plan's lanes), else the plain split
        r.quad_split = plan && (plan->flags & 4) &&
                               (row_bytes == 128 || row_bytes == 256 || (row_bytes == 512 && es == 4))
                           ? 1
                           : 0;
        if (r.quad_split) r.lanes = 16;
        if (r.quad_split && (plan->flags & 8)) r.rows_per_group = 2;  // 512-thread workgroups
        if ((!r.quad_split && K > 4 * r.lanes) || K % sv != 0 || ldb % sv != 0 || !aligned(B, 16) || ldc % 4 != 0 ||
            !aligned(C, 16))
            return SPK_ERR_PLAN;
        const int64_t wmax = tile_lds_budget(r, row_bytes) / (2 * row_bytes);  // two buffers
        int64_t w = 16;  // default: the largest power of two whose slab fits 16 KiB
        while (w * 2 * row_bytes <= 16384) w *= 2;
        r.chunk = plan && plan->chunk > 0 ? plan->chunk : w;
        if (r.chunk < 1 || r.chunk > wmax) return SPK_ERR_PLAN;
        if (r.chunk * ldb * static_cast<int64_t>(es) >= (int64_t(1) << 32)) return SPK_ERR_PLAN;  // 32-bit slab offsets
        r.vec = 4;
        return SPK_OK;
    }
    if (plan && plan->chunk > 0) r.chunk = plan->chunk;
    else if (r.variant == SPK_VAR_SLAB) r.chunk = default_slab_width(K, elem_size(b_dtype));
    else r.chunk = 4 * K > kDefaultChunk ? 4 * K : kDefaultChunk;
    if (plan && (plan->flags & ~1)) return SPK_ERR_PLAN;
    if (plan && plan->chunk < 0) return SPK_ERR_PLAN;
    const bool force_scalar = plan && (plan->flags & 1);
    int32_t v = native_vec(b_dtype);
    if (b_dtype == SPK_BF16 && r.lanes * 8 <= K && K % 8 == 0 && ldb % 8 == 0 && aligned(B, 16)) v = 8;
    const size_t es = elem_size(b_dtype);
    const size_t cs = b_dtype == SPK_F64 ? 8 : 4;
    const bool ok = !force_scalar && K % v == 0 && ldb % v == 0 && ldc % (v > 4 ? 4 : v) == 0 &&
                    aligned(B, es * v) && aligned(C, cs * (v > 4 ? 4 : v));
    r.vec = ok ? v : 1;
    if ((K + r.lanes * r.vec - 1) / (r.lanes * r.vec) > 65535) return SPK_ERR_PLAN;
    return SPK_OK;
}

int32_t resolve_sddmm(const spk_plan *plan, int64_t K, int32_t dt, const void *U, int64_t ldu, const void *V,
                      int64_t ldv, Resolved &r) {
    const bool force_scalar = plan && (plan->flags & 1);
    int32_t v = native_vec(dt);
    const size_t es = elem_size(dt);
    const bool ok = !force_scalar && K % v == 0 && ldu % v == 0 && ldv % v == 0 && aligned(U, es * v) &&
                    aligned(V, es * v);
    r.vec = ok ? v : 1;
    r.variant = plan ? plan->variant : SPK_VAR_MERGE;
    if (r.variant == SPK_VAR_TILE) {
        // groups of 16, 32 or 64 lanes, one 4-wide slice of U and V per lane,
        // slabs of V rows in 16-byte pieces, two slab buffers in kTileLds
        const int64_t sv = 16 / static_cast<int64_t>(es);
        if (dt == SPK_F64 || (plan->flags & ~14) || plan->chunk < 0) return SPK_ERR_PLAN;
        r.lanes = plan->lanes;
        r.rows_per_group = (plan->flags & 2) ? 8 : 4;
        const int64_t row_bytes = K * static_cast<int64_t>(es);
        // one entry per quad where rows are 128 or 256 bytes and U is read in
        // 16-byte pieces (16-lane groups whatever the plan's lanes), else the
        // plain split
        r.quad_split = (plan->flags & 4) && (row_bytes == 128 || row_bytes == 256 || row_bytes == 512) &&
                               ldu % sv == 0 &&
                               aligned(U, 16) && K % sv == 0 && ldv % sv == 0 && aligned(V, 16)
                           ? 1
                           : 0;
        if (r.quad_split) r.lanes = 16;
        if (r.quad_split && (plan->flags & 8)) r.rows_per_group = 2;  // 512-thread workgroups
        if (r.lanes != 16 && r.lanes != 32 && r.lanes != 64) return SPK_ERR_PLAN;
        if ((!r.quad_split && K > 4 * r.lanes) || K % sv != 0 || ldv % sv != 0 || !aligned(V, 16) ||
            ldu % 4 != 0 || !aligned(U, 4 * es))
            return SPK_ERR_PLAN;
        const int64_t wmax = tile_lds_budget(r, row_bytes) / (2 * row_bytes);
        int64_t w = 16;  // default: the largest power of two whose slab fits 16 KiB
        while (w * 2 * row_bytes <= 16384) w *= 2;
        r.chunk = plan->chunk > 0 ? plan->chunk : w;
        if (r.chunk > wmax) return SPK_ERR_PLAN;
        if (r.chunk * ldv * static_cast<int64_t>(es) >= (int64_t(1) << 32)) return SPK_ERR_PLAN;  // 32-bit slab offsets
        r.vec = 4;
        return SPK_OK;
    }
    if (r.variant != SPK_VAR_ROWS && r.variant != SPK_VAR_MERGE && r.variant != SPK_VAR_SLAB) return SPK_ERR_PLAN;
    if (plan && plan->chunk > 0) r.chunk = plan->chunk;
    else if (r.variant == SPK_VAR_SLAB) r.chunk = default_slab_width(K, es);
    else r.chunk = kDefaultChunk;
    if (plan) {
        if (plan->flags & ~1) return SPK_ERR_PLAN;
        if (plan->chunk < 0) return SPK_ERR_PLAN;
        if (!valid_lanes(plan->lanes)) return SPK_ERR_PLAN;
        r.lanes = plan->lanes;
    } else {
        r.lanes = 8;
    }
    // At most 8 register slices of lanes*vec columns; widen the group if needed.
    if (!plan) {
        while (r.lanes < 64 && (K + r.lanes * r.vec - 1) / (r.lanes * r.vec) > 8) r.lanes <<= 1;
    }
    if ((K + r.lanes * r.vec - 1) / (r.lanes * r.vec) > 8) return SPK_ERR_PLAN;
    return SPK_OK;
}

int32_t check_ws(size_t need, const void *ws, size_t ws_bytes) {
    if (need == 0) return SPK_OK;
    if (!ws || ws_bytes < need) return SPK_ERR_WORKSPACE;
    return SPK_OK;
}

// kGridTooLarge marks a launch whose grid would pass the 32-bit work-item
// count of a dispatch: a shape beyond what the plan can cover.
int32_t hip_status(hipError_t e) {
    return e == hipSuccess ? SPK_OK : e == kGridTooLarge ? SPK_ERR_SIZE : SPK_ERR_HIP;
}

size_t spmm_ws(int64_t m, int64_t n, int64_t nnz, int64_t K, int32_t dt, const Resolved &r, bool permuted) {
    if (m == 0 || K == 0) return 0;
    if (r.variant == SPK_VAR_TILE) return permuted ? align_up(sizeof(float) * static_cast<size_t>(nnz)) : 0;
    if (r.variant == SPK_VAR_MERGE) return merge_layout(m, nnz, K, r.chunk, dt == SPK_F64 ? 8 : 4).total;
    if (r.variant == SPK_VAR_SLAB) return slab_layout(m, n, r.chunk).total;
    return 0;
}

size_t sddmm_ws(int64_t m, int64_t n, const Resolved &r) {
    return r.variant == SPK_VAR_SLAB ? slab_layout(m, n, r.chunk).total : 0;
}

}  // namespace

extern "C" {

const char *spk_strerror(int32_t status) {
    switch (status) {
    case SPK_OK: return "ok";
    case SPK_ERR_NULL: return "a required pointer is NULL";
    case SPK_ERR_SIZE: return "size out of range";
    case SPK_ERR_DTYPE: return "unsupported dtype combination";
    case SPK_ERR_LD: return "leading dimension smaller than K";
    case SPK_ERR_WORKSPACE: return "workspace missing or too small";
    case SPK_ERR_PLAN: return "plan invalid for this call";
    case SPK_ERR_HIP: return "HIP runtime error";
    case SPK_ERR_STRUCTURE: return "CSR is not canonical";
    case SPK_ERR_OP: return "unknown op";
    case SPK_ERR_NO_MODEL: return "no selector model loaded";
    default: return "unknown status";
    }
}

size_t spk_workspace_bytes(int32_t op, const spk_csr *A, int64_t K, const spk_plan *plan) {
    if (check_csr(A) != SPK_OK || K < 0) return 0;
    if (plan && (plan->chunk < 0 || plan->variant < SPK_VAR_ROWS || plan->variant > SPK_VAR_TILE)) return 0;
    // The size depends only on the variant, the chunk and the shapes.  Sizes
    // assume the widest element (8 bytes): the largest carry and, for the
    // default slab width, the most slabs, so any dtype's call fits.
    Resolved r;
    r.lanes = 4;
    r.vec = 1;
    const bool bwd = op == SPK_OP_BACKWARD;
    const int64_t m = bwd ? A->n : A->m, n = bwd ? A->m : A->n;
    switch (op) {
    case SPK_OP_SPMM:
    case SPK_OP_BACKWARD:
        r.variant = plan ? plan->variant : SPK_VAR_ROWS;
        if (plan && plan->chunk > 0) r.chunk = plan->chunk;
        else if (r.variant == SPK_VAR_SLAB) r.chunk = default_slab_width(K, 8);
        else r.chunk = 4 * K > kDefaultChunk ? 4 * K : kDefaultChunk;
        return spmm_ws(m, n, A->nnz, K, SPK_F64, r, bwd);
    case SPK_OP_SDDMM:
        r.variant = plan ? plan->variant : SPK_VAR_MERGE;
        r.chunk = plan && plan->chunk > 0 ? plan->chunk : default_slab_width(K, 8);
        return sddmm_ws(m, n, r);
    case SPK_OP_TRANSPOSE: return transpose_ws_bytes(A->m, A->n, A->nnz);
    case SPK_OP_BSR4: return scan_ws_bytes_i32((A->m + 3) / 4 + 1);
    case SPK_OP_SELECT:
        return align_up(sizeof(int64_t) * 28) + align_up(sizeof(int32_t) * kRankSlots) + features_ws_bytes(A->m);
    default: return 0;
    }
}

int32_t csr_to_bsr4_count(const spk_csr *A, int32_t *b_row_ptr, int64_t *nblocks, void *ws, size_t ws_bytes,
                          void *stream) {
    int32_t st = check_csr(A);
    if (st) return st;
    if (!b_row_ptr || !nblocks) return SPK_ERR_NULL;
    const int64_t mb = (A->m + 3) / 4;
    if ((st = check_ws(scan_ws_bytes_i32(mb + 1), ws, ws_bytes))) return st;
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (hipMemsetAsync(b_row_ptr, 0, sizeof(int32_t) * static_cast<size_t>(mb + 1), s) != hipSuccess) return SPK_ERR_HIP;
    if ((st = hip_status(bsr4_count_launch(A->m, A->row_ptr, A->col_idx, b_row_ptr, s)))) return st;
    if ((st = hip_status(exclusive_scan_i32(b_row_ptr, mb + 1, ws, s)))) return st;
    int32_t total = 0;
    if (hipMemcpyAsync(&total, b_row_ptr + mb, sizeof(int32_t), hipMemcpyDeviceToHost, s) != hipSuccess)
        return SPK_ERR_HIP;
    if (hipStreamSynchronize(s) != hipSuccess) return SPK_ERR_HIP;
    *nblocks = total;
    return SPK_OK;
}

int32_t csr_to_bsr4_fill(const spk_csr *A, const int32_t *b_row_ptr, int32_t *b_col, float *b_vals, void *stream) {
    int32_t st = check_csr(A);
    if (st) return st;
    if (A->vals && A->vals_dtype != SPK_F32) return SPK_ERR_DTYPE;
    if (!b_row_ptr || (A->nnz > 0 && (!b_col || !b_vals))) return SPK_ERR_NULL;
    if (A->nnz == 0) return SPK_OK;
    return hip_status(bsr4_fill_launch(A->m, A->row_ptr, A->col_idx, static_cast<const float *>(A->vals), b_row_ptr,
                                       b_col, b_vals, static_cast<hipStream_t>(stream)));
}

int32_t spmm_bsr4(const spk_bsr4 *A, const void *B, int64_t ldb, int32_t b_dtype, int64_t K, void *C, int64_t ldc,
                  void *stream) {
    if (!A) return SPK_ERR_NULL;
    if (A->m < 0 || A->n < 0 || A->nblocks < 0 || A->m > kMaxIndex || A->n > kMaxIndex) return SPK_ERR_SIZE;
    if (K < 0 || K > kMaxIndex) return SPK_ERR_SIZE;
    if (b_dtype != SPK_F32 && b_dtype != SPK_BF16) return SPK_ERR_DTYPE;
    if (A->m == 0 || K == 0) return SPK_OK;
    if (!C || !A->b_row_ptr) return SPK_ERR_NULL;
    if (ldc < K) return SPK_ERR_LD;
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (A->nblocks == 0 || A->n == 0) return hip_status(zero_fill(C, A->m, K, ldc, SPK_F32, s));
    if (!B || !A->b_col || !A->b_vals) return SPK_ERR_NULL;
    if (ldb < K) return SPK_ERR_LD;
    const size_t es = elem_size(b_dtype);
    const bool v4 = K >= 256 && K % 4 == 0 && ldb % 4 == 0 && ldc % 4 == 0 && aligned(B, es * 4) && aligned(C, 16);
    Bsr4Args a{A->m, A->n, K, A->b_row_ptr, A->b_col, A->b_vals, B, ldb, b_dtype, v4 ? 4 : 1,
               static_cast<float *>(C), ldc};
    return hip_status(bsr4_spmm_launch(a, s));
}

}  // extern "C"

namespace {

// Scratch of the allocation-free SpMM entry point: a file-scope device array,
// one copy per GPU, held until the process ends.  Host code never uses the
// array's name as an address: each device's address comes from
// hipGetSymbolAddress, once per device, with that device current.
constexpr size_t kNoAllocScratchBytes = size_t(64) << 20;
__device__ __align__(256) unsigned char scratch[kNoAllocScratchBytes];
constexpr int kScratchDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_ptr[kScratchDevices];

int32_t scratch_of_current_device(void **out) {
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kScratchDevices) return SPK_ERR_HIP;
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (!g_scratch_ptr[dev]) {
        void *ptr = nullptr;
        if (hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return SPK_ERR_HIP;
        g_scratch_ptr[dev] = ptr;
    }
    *out = g_scratch_ptr[dev];
    return SPK_OK;
}

// spmm_csr's body; with from_scratch the workspace is this device's scratch
// array (sizes beyond it are refused before anything is launched).
int32_t spmm_common(const spk_csr *A, const void *B, int64_t ldb, int32_t b_dtype, int64_t K, void *C, int64_t ldc,
                    const spk_plan *plan, void *ws, size_t ws_bytes, bool from_scratch, hipStream_t s) {
    int32_t st = check_csr(A);
    if (st) return st;
    if (K < 0 || K > kMaxIndex) return SPK_ERR_SIZE;
    if ((st = check_dtypes(A, b_dtype))) return st;
    if (A->m == 0 || K == 0) return SPK_OK;
    if (!C || (A->nnz > 0 && !B)) return SPK_ERR_NULL;
    if (ldc < K || (A->nnz > 0 && ldb < K)) return SPK_ERR_LD;
    const int32_t out_dt = b_dtype == SPK_F64 ? SPK_F64 : SPK_F32;
    if (A->nnz == 0) return hip_status(zero_fill(C, A->m, K, ldc, out_dt, s));
    Resolved r;
    if ((st = resolve_spmm(plan, K, b_dtype, B, ldb, C, ldc, r))) return st;
    if ((st = tile_nnz_ok(r, A->nnz))) return st;
    const size_t need = spmm_ws(A->m, A->n, A->nnz, K, b_dtype, r, false);
    if (from_scratch) {
        if (need > kNoAllocScratchBytes) return SPK_ERR_WORKSPACE;
        ws = nullptr;
        ws_bytes = 0;
        if (need > 0) {
            if ((st = scratch_of_current_device(&ws))) return st;
            ws_bytes = kNoAllocScratchBytes;
        }
    }
    if ((st = check_ws(need, ws, ws_bytes))) return st;
    SpmmArgs a{A->m, A->n, A->nnz, K, A->row_ptr, A->col_idx, A->vals, nullptr, B, ldb, b_dtype, C, ldc,
               r.variant, r.lanes, r.vec, r.chunk, ws, r.rows_per_group, r.quad_split};
    return hip_status(spmm_launch(a, s));
}

}  // namespace

extern "C" {

int32_t spmm_csr(const spk_csr *A, const void *B, int64_t ldb, int32_t b_dtype, int64_t K, void *C, int64_t ldc,
                 const spk_plan *plan, void *ws, size_t ws_bytes, void *stream) {
    return spmm_common(A, B, ldb, b_dtype, K, C, ldc, plan, ws, ws_bytes, false, static_cast<hipStream_t>(stream));
}

int32_t spmm_csr_noalloc(const spk_csr *A, const void *B, int64_t ldb, int32_t b_dtype, int64_t K, void *C,
                         int64_t ldc, const spk_plan *plan, void *stream) {
    return spmm_common(A, B, ldb, b_dtype, K, C, ldc, plan, nullptr, 0, true, static_cast<hipStream_t>(stream));
}

size_t spmm_csr_noalloc_max_bytes(void) { return kNoAllocScratchBytes; }

int32_t sddmm_csr(const spk_csr *A, const void *U, int64_t ldu, const void *V, int64_t ldv, int32_t uv_dtype,
                  int64_t K, void *S, const spk_plan *plan, void *ws, size_t ws_bytes, void *stream) {
    int32_t st = check_csr(A);
    if (st) return st;
    if (K < 0 || K > kMaxIndex) return SPK_ERR_SIZE;
    if ((st = check_dtypes(A, uv_dtype))) return st;
    if (A->nnz == 0) return SPK_OK;
    if (!S || !U || !V) return SPK_ERR_NULL;
    if (K > 0 && (ldu < K || ldv < K)) return SPK_ERR_LD;
    Resolved r;
    if ((st = resolve_sddmm(plan, K, uv_dtype, U, ldu, V, ldv, r))) return st;
    if ((st = tile_nnz_ok(r, A->nnz))) return st;
    if ((st = check_ws(sddmm_ws(A->m, A->n, r), ws, ws_bytes))) return st;
    SddmmArgs a{A->m, A->n, A->nnz, K, A->row_ptr, A->col_idx, A->vals, U, ldu, V, ldv, uv_dtype, S,
                r.variant, r.lanes, r.vec, r.chunk, ws, r.rows_per_group, r.quad_split};
    return hip_status(sddmm_launch(a, static_cast<hipStream_t>(stream)));
}

int32_t csr_transpose(const spk_csr *A, int32_t *at_row_ptr, int32_t *at_col_idx, int32_t *perm, void *ws,
                      size_t ws_bytes, void *stream) {
    int32_t st = check_csr(A);
    if (st) return st;
    if (!at_row_ptr || (A->nnz > 0 && (!at_col_idx || !perm))) return SPK_ERR_NULL;
    const size_t need = transpose_ws_bytes(A->m, A->n, A->nnz);
    if ((st = check_ws(need, ws, ws_bytes))) return st;
    return hip_status(transpose_launch(A->m, A->n, A->nnz, A->row_ptr, A->col_idx, at_row_ptr, at_col_idx, perm, ws,
                                       static_cast<hipStream_t>(stream)));
}

int32_t spmm_csr_backward(const spk_csr *A, const int32_t *at_row_ptr, const int32_t *at_col_idx, const int32_t *perm,
                          const void *B, int64_t ldb, const void *G, int64_t ldg, int32_t dtype, int64_t K, void *dB,
                          int64_t lddb, void *dvals, const spk_plan *plan, const spk_plan *dvals_plan, void *ws,
                          size_t ws_bytes, void *stream) {
    int32_t st = check_csr(A);
    if (st) return st;
    if (K < 0 || K > kMaxIndex) return SPK_ERR_SIZE;
    if (dtype != SPK_F32 && dtype != SPK_F64) return SPK_ERR_DTYPE;
    if ((st = check_dtypes(A, dtype))) return st;
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (dB && A->n > 0 && K > 0) {
        if (!G && A->nnz > 0) return SPK_ERR_NULL;
        if (!at_row_ptr || (A->nnz > 0 && (!at_col_idx || !perm))) return SPK_ERR_NULL;
        if (lddb < K || (A->nnz > 0 && ldg < K)) return SPK_ERR_LD;
        if (A->nnz == 0) {
            if ((st = hip_status(zero_fill(dB, A->n, K, lddb, dtype, s)))) return st;
        } else {
            Resolved r;
            if ((st = resolve_spmm(plan, K, dtype, G, ldg, dB, lddb, r))) return st;
            if ((st = tile_nnz_ok(r, A->nnz))) return st;
            const size_t need = spmm_ws(A->n, A->m, A->nnz, K, dtype, r, true);
            if ((st = check_ws(need, ws, ws_bytes))) return st;
            SpmmArgs a{A->n, A->m, A->nnz, K, at_row_ptr, at_col_idx, A->vals, perm, G, ldg, dtype, dB, lddb,
                       r.variant, r.lanes, r.vec, r.chunk, ws, r.rows_per_group, r.quad_split};
            if ((st = hip_status(spmm_launch(a, s)))) return st;
        }
    }
    if (dvals && A->nnz > 0) {
        if (!G || !B) return SPK_ERR_NULL;
        if (K > 0 && (ldg < K || ldb < K)) return SPK_ERR_LD;
        // the pattern SDDMM runs after A^T G on the same stream, so the two
        // share the workspace
        Resolved r;
        if ((st = resolve_sddmm(dvals_plan, K, dtype, G, ldg, B, ldb, r))) return st;
        if ((st = tile_nnz_ok(r, A->nnz))) return st;
        if ((st = check_ws(sddmm_ws(A->m, A->n, r), ws, ws_bytes))) return st;
        SddmmArgs a{A->m, A->n, A->nnz, K, A->row_ptr, A->col_idx, nullptr, G, ldg, B, ldb, dtype, dvals,
                    r.variant, r.lanes, r.vec, r.chunk, ws, r.rows_per_group, r.quad_split};
        if ((st = hip_status(sddmm_launch(a, s)))) return st;
    }
    return SPK_OK;
}

// ---------------------------------------------------------------- slab16
}  // extern "C"

namespace {

int64_t slab16_slabs(int64_t n, int64_t width) { return n > 0 ? (n + width - 1) / width : 1; }

int32_t check_slab16(const spk_slab16 *F) {
    if (!F) return SPK_ERR_NULL;
    if (F->m < 0 || F->n < 0 || F->nnz < 0 || F->m > kMaxIndex || F->n > kMaxIndex || F->nnz > kMaxIndex)
        return SPK_ERR_SIZE;
    if (F->width < 1 || F->width > 65536 || F->nslabs != slab16_slabs(F->n, F->width)) return SPK_ERR_SIZE;
    if (F->nslabs * F->m >= kMaxIndex) return SPK_ERR_SIZE;
    if (F->m > 0 && (!F->seg || !F->apos)) return SPK_ERR_NULL;
    if (F->nnz > 0 && !F->col16) return SPK_ERR_NULL;
    return SPK_OK;
}

// A plan for the row-split code path of the slab form (lanes and flags).
int32_t slab16_plan(const spk_plan *plan, spk_plan &out) {
    if (plan && plan->variant != SPK_VAR_SLAB16) return SPK_ERR_PLAN;
    out = plan ? spk_plan{SPK_VAR_ROWS, plan->lanes, 0, plan->flags} : spk_plan{SPK_VAR_ROWS, 0, 0, 0};
    return SPK_OK;
}

}  // namespace

extern "C" {

size_t slab16_workspace_bytes(const spk_csr *A, int64_t width) {
    if (check_csr(A) != SPK_OK || width < 1 || width > 65536) return 0;
    const int64_t S = slab16_slabs(A->n, width);
    if (S * A->m >= kMaxIndex) return 0;
    return slab16_ws_bytes(A->m, S);
}

int32_t csr_to_slab16(const spk_csr *A, int64_t width, int32_t *seg, int32_t *apos, uint16_t *col16, void *ws,
                      size_t ws_bytes, void *stream) {
    int32_t st = check_csr(A);
    if (st) return st;
    if (width < 1 || width > 65536) return SPK_ERR_SIZE;
    const int64_t S = slab16_slabs(A->n, width);
    if (S * A->m >= kMaxIndex) return SPK_ERR_SIZE;
    if (!seg || (A->m > 0 && !apos) || (A->nnz > 0 && !col16)) return SPK_ERR_NULL;
    if ((st = check_ws(slab16_ws_bytes(A->m, S), ws, ws_bytes))) return st;
    return hip_status(slab16_build_launch(A->m, A->nnz, A->row_ptr, A->col_idx, width, S, seg, apos, col16, ws,
                                          static_cast<hipStream_t>(stream)));
}

int32_t spmm_slab16(const spk_slab16 *F, const void *vals, const void *B, int64_t ldb, int32_t b_dtype, int64_t K,
                    void *C, int64_t ldc, const spk_plan *plan, void *stream) {
    int32_t st = check_slab16(F);
    if (st) return st;
    if (K < 0 || K > kMaxIndex) return SPK_ERR_SIZE;
    if (b_dtype != SPK_F32 && b_dtype != SPK_BF16) return SPK_ERR_DTYPE;
    if (F->m == 0 || K == 0) return SPK_OK;
    if (!C || (F->nnz > 0 && !B)) return SPK_ERR_NULL;
    if (ldc < K || (F->nnz > 0 && ldb < K)) return SPK_ERR_LD;
    spk_plan p;
    if ((st = slab16_plan(plan, p))) return st;
    if (!plan) p.lanes = default_spmm_lanes(K);
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (F->nnz == 0) return hip_status(zero_fill(C, F->m, K, ldc, SPK_F32, s));
    Resolved r;
    if ((st = resolve_spmm(&p, K, b_dtype, B, ldb, C, ldc, r))) return st;
    SpmmArgs a{F->m, F->n, F->nnz, K, nullptr, nullptr, vals, nullptr, B, ldb, b_dtype, C, ldc,
               SPK_VAR_SLAB16, r.lanes, r.vec, F->width, nullptr};
    a.s16 = Slab16View{F->seg, F->apos, F->col16, F->width, F->nslabs};
    return hip_status(spmm_launch(a, s));
}

int32_t sddmm_slab16(const spk_slab16 *F, const void *vals, const void *U, int64_t ldu, const void *V, int64_t ldv,
                     int32_t uv_dtype, int64_t K, void *S, const spk_plan *plan, void *stream) {
    int32_t st = check_slab16(F);
    if (st) return st;
    if (K < 0 || K > kMaxIndex) return SPK_ERR_SIZE;
    if (uv_dtype != SPK_F32 && uv_dtype != SPK_BF16) return SPK_ERR_DTYPE;
    if (F->nnz == 0) return SPK_OK;
    if (!S || !U || !V) return SPK_ERR_NULL;
    if (K > 0 && (ldu < K || ldv < K)) return SPK_ERR_LD;
    spk_plan p;
    if ((st = slab16_plan(plan, p))) return st;
    if (!plan) {  // the default SDDMM group: 8 lanes, widened until K fits 8 register slices of 4 columns
        p.lanes = 8;
        while (p.lanes < 64 && (K + p.lanes * 4 - 1) / (p.lanes * 4) > 8) p.lanes <<= 1;
    }
    Resolved r;
    if ((st = resolve_sddmm(&p, K, uv_dtype, U, ldu, V, ldv, r))) return st;
    SddmmArgs a{F->m, F->n, F->nnz, K, nullptr, nullptr, vals, U, ldu, V, ldv, uv_dtype, S,
                SPK_VAR_SLAB16, r.lanes, r.vec, F->width, nullptr};
    a.s16 = Slab16View{F->seg, F->apos, F->col16, F->width, F->nslabs};
    return hip_status(sddmm_launch(a, static_cast<hipStream_t>(stream)));
}

// ---------------------------------------------------------------- hyper-sparse
}  // extern "C"

namespace {

int32_t check_dcsr(const spk_dcsr *D) {
    if (!D) return SPK_ERR_NULL;
    if (D->m < 0 || D->n < 0 || D->nnz < 0 || D->m > kMaxIndex || D->n > kMaxIndex || D->nnz > kMaxIndex)
        return SPK_ERR_SIZE;
    if (D->nrows < 0 || D->nrows > D->m) return SPK_ERR_SIZE;
    if (D->m > 0 && (!D->row_ptr || !D->order)) return SPK_ERR_NULL;
    if (D->nnz > 0 && !D->col_idx) return SPK_ERR_NULL;
    return SPK_OK;
}

// Lanes and flags of a hyper-sparse plan (variant `want`), as a ROWS plan.
int32_t hyper_plan(const spk_plan *plan, int32_t want, spk_plan &out) {
    if (plan && plan->variant != want) return SPK_ERR_PLAN;
    out = plan ? spk_plan{SPK_VAR_ROWS, plan->lanes, 0, plan->flags} : spk_plan{SPK_VAR_ROWS, 0, 0, 0};
    return SPK_OK;
}

int32_t default_sddmm_lanes(int64_t K) {
    int32_t lanes = 8;
    while (lanes < 64 && (K + lanes * 4 - 1) / (lanes * 4) > 8) lanes <<= 1;
    return lanes;
}

}  // namespace

extern "C" {

size_t nonempty_order_workspace_bytes(const spk_csr *A) {
    if (check_csr(A) != SPK_OK) return 0;
    return align_up(sizeof(int32_t)) + nonempty_order_ws_bytes(A->m);
}

int32_t csr_nonempty_order(const spk_csr *A, int32_t *order, int64_t *nrows, void *ws, size_t ws_bytes,
                           void *stream) {
    int32_t st = check_csr(A);
    if (st) return st;
    if (!nrows || (A->m > 0 && !order)) return SPK_ERR_NULL;
    if (A->m == 0) {
        *nrows = 0;
        return SPK_OK;
    }
    if ((st = check_ws(align_up(sizeof(int32_t)) + nonempty_order_ws_bytes(A->m), ws, ws_bytes))) return st;
    hipStream_t s = static_cast<hipStream_t>(stream);
    int32_t *count = static_cast<int32_t *>(ws);
    if ((st = hip_status(nonempty_order_launch(A->m, A->row_ptr, order, count,
                                               static_cast<char *>(ws) + align_up(sizeof(int32_t)), s))))
        return st;
    int32_t host = 0;
    if (hipMemcpyAsync(&host, count, sizeof(int32_t), hipMemcpyDeviceToHost, s) != hipSuccess) return SPK_ERR_HIP;
    if (hipStreamSynchronize(s) != hipSuccess) return SPK_ERR_HIP;
    *nrows = host;
    return SPK_OK;
}

int32_t spmm_dcsr(const spk_dcsr *D, const void *B, int64_t ldb, int32_t b_dtype, int64_t K, void *C, int64_t ldc,
                  const spk_plan *plan, void *stream) {
    int32_t st = check_dcsr(D);
    if (st) return st;
    if (K < 0 || K > kMaxIndex) return SPK_ERR_SIZE;
    if (b_dtype != SPK_F32 && b_dtype != SPK_BF16) return SPK_ERR_DTYPE;
    if (D->m == 0 || K == 0) return SPK_OK;
    if (!C || (D->nnz > 0 && !B)) return SPK_ERR_NULL;
    if (ldc < K || (D->nnz > 0 && ldb < K)) return SPK_ERR_LD;
    spk_plan p;
    if ((st = hyper_plan(plan, SPK_VAR_DCSR, p))) return st;
    if (!plan) p.lanes = default_spmm_lanes(K);
    hipStream_t s = static_cast<hipStream_t>(stream);
    if (D->nnz == 0) return hip_status(zero_fill(C, D->m, K, ldc, SPK_F32, s));
    Resolved r;
    if ((st = resolve_spmm(&p, K, b_dtype, B, ldb, C, ldc, r))) return st;
    SpmmArgs a{D->m, D->n, D->nnz, K, D->row_ptr, D->col_idx, D->vals, nullptr, B, ldb, b_dtype, C, ldc,
               SPK_VAR_DCSR, r.lanes, r.vec, 0, nullptr};
    a.hv.order = D->order;
    a.hv.nrows = D->nrows;
    return hip_status(spmm_launch(a, s));
}

int32_t sddmm_dcsr(const spk_dcsr *D, const void *U, int64_t ldu, const void *V, int64_t ldv, int32_t uv_dtype,
                   int64_t K, void *S, const spk_plan *plan, void *stream) {
    int32_t st = check_dcsr(D);
    if (st) return st;
    if (K < 0 || K > kMaxIndex) return SPK_ERR_SIZE;
    if (uv_dtype != SPK_F32 && uv_dtype != SPK_BF16) return SPK_ERR_DTYPE;
    if (D->nnz == 0) return SPK_OK;
    if (!S || !U || !V) return SPK_ERR_NULL;
    if (K > 0 && (ldu < K || ldv < K)) return SPK_ERR_LD;
    spk_plan p;
    if ((st = hyper_plan(plan, SPK_VAR_DCSR, p))) return st;
    if (!plan) p.lanes = default_sddmm_lanes(K);
    Resolved r;
    if ((st = resolve_sddmm(&p, K, uv_dtype, U, ldu, V, ldv, r))) return st;
    SddmmArgs a{D->m, D->n, D->nnz, K, D->row_ptr, D->col_idx, D->vals, U, ldu, V, ldv, uv_dtype, S,
                SPK_VAR_DCSR, r.lanes, r.vec, 0, nullptr};
    a.hv.order = D->order;
    a.hv.nrows = D->nrows;
    return hip_status(sddmm_launch(a, static_cast<hipStream_t>(stream)));
}

int32_t csr_row_index(const spk_csr *A, int32_t *rowidx, void *stream) {
    int32_t st = check_csr(A);
    if (st) return st;
    if (A->nnz > 0 && !rowidx) return SPK_ERR_NULL;
    if (A->nnz == 0) return SPK_OK;
    return hip_status(row_index_launch(A->m, A->row_ptr, rowidx, static_cast<hipStream_t>(stream)));
}

int32_t sddmm_coo(const spk_csr *A, const int32_t *rowidx, const void *U, int64_t ldu, const void *V, int64_t ldv,
                  int32_t uv_dtype, int64_t K, void *S, const spk_plan *plan, void *stream) {
    int32_t st = check_csr(A);
    if (st) return st;
    if (K < 0 || K > kMaxIndex) return SPK_ERR_SIZE;
    if (uv_dtype != SPK_F32 && uv_dtype != SPK_BF16) return SPK_ERR_DTYPE;
    if (A->vals && A->vals_dtype != SPK_F32) return SPK_ERR_DTYPE;
    if (A->nnz == 0) return SPK_OK;
    if (!S || !U || !V || !rowidx) return SPK_ERR_NULL;
    if (K > 0 && (ldu < K || ldv < K)) return SPK_ERR_LD;
    if (plan && plan->chunk < 0) return SPK_ERR_PLAN;
    spk_plan p;
    if ((st = hyper_plan(plan, SPK_VAR_COO, p))) return st;
    if (!plan) p.lanes = default_sddmm_lanes(K);
    Resolved r;
    if ((st = resolve_sddmm(&p, K, uv_dtype, U, ldu, V, ldv, r))) return st;
    const int64_t chunk = plan && plan->chunk > 0 ? plan->chunk : 64;
    SddmmArgs a{A->m, A->n, A->nnz, K, A->row_ptr, A->col_idx, A->vals, U, ldu, V, ldv, uv_dtype, S,
                SPK_VAR_COO, r.lanes, r.vec, chunk, nullptr};
    a.hv.rowidx = rowidx;
    return hip_status(sddmm_launch(a, static_cast<hipStream_t>(stream)));
}

// ---------------------------------------------------------------- attention chain
}  // extern "C"

namespace {

constexpr int64_t kAttnItems = 512;  // entries per run of the entry-split attention

int32_t resolve_attn(const spk_plan *plan, int32_t &variant, int64_t &items) {
    variant = plan ? plan->variant : SPK_VAR_MERGE;
    if (variant != SPK_VAR_ROWS && variant != SPK_VAR_MERGE) return SPK_ERR_PLAN;
    if (plan && (!valid_lanes(plan->lanes) || (plan->flags & ~1) || plan->chunk < 0)) return SPK_ERR_PLAN;
    items = plan && plan->chunk > 0 ? plan->chunk : kAttnItems;
    return SPK_OK;
}

}  // namespace

extern "C" {

size_t attention_workspace_bytes(const spk_csr *A, int64_t K2, const spk_plan *plan) {
    int32_t variant;
    int64_t items;
    if (check_csr(A) != SPK_OK || K2 < 0 || resolve_attn(plan, variant, items) != SPK_OK) return 0;
    return variant == SPK_VAR_MERGE ? attn_layout(A->nnz, K2, items, true).total : 0;
}

int32_t sddmm_softmax_spmm(const spk_csr *A, const void *U, int64_t ldu, const void *V, int64_t ldv, int64_t K1,
                           const void *B, int64_t ldb, int64_t K2, int32_t dtype, float *O, int64_t ldo, float *lse,
                           const spk_plan *plan, void *ws, size_t ws_bytes, void *stream) {
    int32_t st = check_csr(A);
    if (st) return st;
    if (K1 < 0 || K2 < 0 || K1 > kMaxIndex || K2 > kMaxIndex) return SPK_ERR_SIZE;
    if (dtype != SPK_F32 && dtype != SPK_BF16) return SPK_ERR_DTYPE;
    if (A->vals && A->vals_dtype != SPK_F32) return SPK_ERR_DTYPE;
    int32_t variant;
    int64_t items;
    if ((st = resolve_attn(plan, variant, items))) return st;
    if (A->m == 0 || (K2 == 0 && !lse)) return SPK_OK;
    if ((K2 > 0 && (!O || !B)) || (K1 > 0 && (!U || !V))) return SPK_ERR_NULL;
    if ((K2 > 0 && (ldo < K2 || ldb < K2)) || (K1 > 0 && (ldu < K1 || ldv < K1))) return SPK_ERR_LD;
    const int64_t kmax = K1 > K2 ? K1 : K2;
    int32_t lanes = 8;
    if (plan) lanes = plan->lanes;
    else
        while (lanes < 64 && (kmax + lanes * 4 - 1) / (lanes * 4) > 8) lanes <<= 1;
    const size_t es = elem_size(dtype);
    const bool v4 = !(plan && (plan->flags & 1)) && K1 % 4 == 0 && K2 % 4 == 0 && ldu % 4 == 0 && ldv % 4 == 0 &&
                    ldb % 4 == 0 && ldo % 4 == 0 && aligned(U, es * 4) && aligned(V, es * 4) && aligned(B, es * 4) &&
                    aligned(O, 16);
    const int32_t vec = v4 ? 4 : 1;
    if ((kmax + lanes * vec - 1) / (lanes * vec) > 8) return SPK_ERR_PLAN;
    if (variant == SPK_VAR_MERGE && (st = check_ws(attn_layout(A->nnz, K2, items, true).total, ws, ws_bytes))) return st;
    AttnArgs a{A->m, A->n, A->nnz, K1, K2, A->row_ptr, A->col_idx, static_cast<const float *>(A->vals), U, ldu, V, ldv,
               B, ldb, dtype, O, ldo, lse, lanes, vec, variant, items, ws};
    return hip_status(attn_launch(a, static_cast<hipStream_t>(stream)));
}

size_t row_softmax_workspace_bytes(const spk_csr *A) {
    if (check_csr(A) != SPK_OK) return 0;
    return row_softmax_ws_bytes(A->m, A->nnz);
}

int32_t csr_row_softmax(const spk_csr *A, float *S, float *lse, void *ws, size_t ws_bytes, void *stream) {
    int32_t st = check_csr(A);
    if (st) return st;
    if (A->nnz > 0 && !S) return SPK_ERR_NULL;
    if (A->m == 0) return SPK_OK;
    if ((st = check_ws(row_softmax_ws_bytes(A->m, A->nnz), ws, ws_bytes))) return st;
    return hip_status(row_softmax_launch(A->m, A->nnz, A->row_ptr, S, lse, ws, static_cast<hipStream_t>(stream)));
}

// ---------------------------------------------------------------- selector
static constexpr int kMaxDevices = 64;
static int32_t g_loaded[kMaxDevices][2];
static int64_t g_dims[kMaxDevices][2][3];

static int current_device() {
    int d = 0;
    if (hipGetDevice(&d) != hipSuccess || d < 0 || d >= kMaxDevices) return -1;
    return d;
}

int32_t plan_count(int32_t op) { return op == SPK_OP_SPMM ? 30 : op == SPK_OP_SDDMM ? 29 : 0; }

int32_t plan_of_index(int32_t op, int32_t index, int64_t K, int32_t dtype, spk_plan *out, int32_t *valid) {
    if (!out) return SPK_ERR_NULL;
    if (op != SPK_OP_SPMM && op != SPK_OP_SDDMM) return SPK_ERR_OP;
    if (dtype != SPK_F32 && dtype != SPK_BF16 && dtype != SPK_F64) return SPK_ERR_DTYPE;
    if (index < 0 || index >= plan_count(op)) return SPK_ERR_PLAN;
    const int64_t k = K > 0 ? K : 1;
    // widths below are in F32 rows (BF16 slabs take half the bytes)
    const int32_t tile_first = op == SPK_OP_SPMM ? 16 : 15;
    const int32_t wide_first = op == SPK_OP_SPMM ? 24 : 23;
    int32_t sddmm_lanes = 8;  // the default SDDMM group, widened until K fits 8 register slices
    while (sddmm_lanes < 64 && (k + sddmm_lanes * 4 - 1) / (sddmm_lanes * 4) > 8) sddmm_lanes <<= 1;
    const int32_t tile_lanes =
        op == SPK_OP_SDDMM && default_spmm_lanes(K) < 16 ? 16 : default_spmm_lanes(K);  // SDDMM TILE: 16-lane rows
    const int32_t row_lanes = op == SPK_OP_SPMM ? default_spmm_lanes(K) : sddmm_lanes;
    auto slab16_width = [&](int64_t bytes) {
        int64_t w = bytes / (4 * k);
        return static_cast<int32_t>(w < 256 ? 256 : w > 65536 ? 65536 : w);
    };
    if (op == SPK_OP_SPMM && index == 15) {
        *out = spk_plan{SPK_VAR_BSR4, 64, 0, 0};
    } else if (index >= tile_first && index < wide_first) {
        // LDS slabs of 16 or 32 KiB, 4 or 8 rows per lane group; the last
        // four split the work one entry per quad (16 KiB slabs, then 32 KiB)
        const int t = index - tile_first;
        const int64_t bytes = (t < 4 ? t % 2 == 1 : t >= 6) ? 32768 : 16384;
        const int64_t w = bytes / (4 * k);
        const int32_t flags = t < 4 ? (t >= 2 ? 2 : 0) : 4 | (t % 2 == 1 ? 2 : 0);
        *out = spk_plan{SPK_VAR_TILE, tile_lanes, static_cast<int32_t>(w > 0 ? w : 1), flags};
    } else if (index == wide_first || index == wide_first + 1) {
        // one entry per quad in wide workgroups, slabs of 32 or 64 KiB
        const int64_t w = (index == wide_first ? 32768 : 65536) / (4 * k);
        *out = spk_plan{SPK_VAR_TILE, tile_lanes, static_cast<int32_t>(w > 0 ? w : 1), 12};
    } else if (index == wide_first + 2 || index == wide_first + 3) {
        // column-slab form: 4 (SpMM; SDDMM 2) or 8 MiB of the dense operand
        // per slab; SDDMM groups of 8 lanes widened until a lane holds at
        // most 8 columns; the 8 MiB SpMM plan likewise, with at least 16
        // lanes and no more than the plain ones
        int32_t s16_lanes = 8;
        while (s16_lanes < 64 && s16_lanes * 8 < k) s16_lanes <<= 1;
        const int64_t small = op == SPK_OP_SPMM ? 4 << 20 : 2 << 20;
        int32_t lanes = s16_lanes;
        if (op == SPK_OP_SPMM) {
            const int32_t wide_lanes = s16_lanes < 16 ? 16 : s16_lanes;
            lanes = index == wide_first + 2 || wide_lanes > row_lanes ? row_lanes : wide_lanes;
        }
        *out = spk_plan{SPK_VAR_SLAB16, lanes, slab16_width(index == wide_first + 2 ? small : 8 << 20), 0};
    } else if (index == wide_first + 4) {
        *out = spk_plan{SPK_VAR_DCSR, row_lanes, 0, 0};
    } else if (index == wide_first + 5) {
        *out = op == SPK_OP_SPMM ? spk_plan{SPK_VAR_DCSR, 4, 0, 0} : spk_plan{SPK_VAR_COO, 16, 16, 0};
    } else {
        static const int32_t variants[3] = {SPK_VAR_ROWS, SPK_VAR_MERGE, SPK_VAR_SLAB};
        const int32_t v = variants[index / 5];
        const int32_t chunk = (op == SPK_OP_SDDMM && v == SPK_VAR_MERGE) ? 256 : 0;
        *out = spk_plan{v, 4 << (index % 5), chunk, 0};
    }
    if (valid) *valid = plan_valid_host(op, index, K, dtype) ? 1 : 0;
    return SPK_OK;
}

int32_t csr_features(const spk_csr *A, int64_t *features, void *ws, size_t ws_bytes, void *stream) {
    int32_t st = check_csr(A);
    if (st) return st;
    if (!features) return SPK_ERR_NULL;
    if ((st = check_ws(features_ws_bytes(A->m), ws, ws_bytes))) return st;
    return hip_status(features_launch(A->m, A->n, A->nnz, A->row_ptr, A->col_idx, features, ws,
                                      static_cast<hipStream_t>(stream)));
}

int32_t selector_inputs(const int64_t *features, int64_t K, int32_t dtype, float *x, void *stream) {
    if (!features || !x) return SPK_ERR_NULL;
    if (K < 0) return SPK_ERR_SIZE;
    if (dtype != SPK_F32 && dtype != SPK_BF16 && dtype != SPK_F64) return SPK_ERR_DTYPE;
    return hip_status(inputs_launch(features, K, dtype, x, static_cast<hipStream_t>(stream)));
}

int32_t mlp_forward(const float *params, int64_t F, int64_t H, int64_t P, const float *X, int64_t batch, float *Y,
                    void *stream) {
    if (!mlp_dims_ok(F, H, P) || batch < 0 || batch > kMaxIndex) return SPK_ERR_SIZE;
    if (batch > 0 && (!params || !X || !Y)) return SPK_ERR_NULL;
    return hip_status(mlp_forward_launch(params, F, H, P, X, batch, Y, static_cast<hipStream_t>(stream)));
}

size_t mlp_workspace_bytes(int64_t F, int64_t H, int64_t P, int64_t batch) {
    if (!mlp_dims_ok(F, H, P) || batch < 0) return 0;
    return mlp_train_ws_bytes(F, H, P, batch);
}

int32_t mlp_loss_grad(const float *params, int64_t F, int64_t H, int64_t P, const float *X, const float *T,
                      const float *mask, int64_t batch, float *grads, float *loss, void *ws, size_t ws_bytes,
                      void *stream) {
    if (!mlp_dims_ok(F, H, P) || batch < 0 || batch > kMaxIndex) return SPK_ERR_SIZE;
    if (!params || !grads || !loss || (batch > 0 && (!X || !T || !mask))) return SPK_ERR_NULL;
    int32_t st = check_ws(mlp_train_ws_bytes(F, H, P, batch), ws, ws_bytes);
    if (st) return st;
    return hip_status(
        mlp_loss_grad_launch(params, F, H, P, X, T, mask, batch, grads, loss, ws, static_cast<hipStream_t>(stream)));
}

int32_t adam_update(float *params, const float *grads, float *mom, float *vel, int64_t count, float lr, float beta1,
                    float beta2, float eps, int64_t step, void *stream) {
    if (count < 0 || step < 1) return SPK_ERR_SIZE;
    if (count > 0 && (!params || !grads || !mom || !vel)) return SPK_ERR_NULL;
    return hip_status(adam_launch(params, grads, mom, vel, count, lr, beta1, beta2, eps, step,
                                  static_cast<hipStream_t>(stream)));
}

int32_t selector_load(int32_t op, const float *table, int64_t F, int64_t H, int64_t P) {
    if (op != SPK_OP_SPMM && op != SPK_OP_SDDMM) return SPK_ERR_OP;
    if (!table) return SPK_ERR_NULL;
    if (F != 33 || !mlp_dims_ok(F, H, P) || P != plan_count(op)) return SPK_ERR_SIZE;
    const int dev = current_device();
    if (dev < 0) return SPK_ERR_HIP;
    int32_t st = hip_status(selector_table_load(op, table, F, H, P));
    if (st) return st;
    g_loaded[dev][op] = 1;
    g_dims[dev][op][0] = F;
    g_dims[dev][op][1] = H;
    g_dims[dev][op][2] = P;
    return SPK_OK;
}

int32_t plan_rank(const spk_csr *A, int64_t K, int32_t op, int32_t dtype, int32_t k, spk_plan *out, int32_t *count,
                  void *ws, size_t ws_bytes, void *stream) {
    int32_t st = check_csr(A);
    if (st) return st;
    if (dtype != SPK_F32 && dtype != SPK_BF16 && dtype != SPK_F64) return SPK_ERR_DTYPE;
    if (!out || !count) return SPK_ERR_NULL;
    if (k < 1 || k > kRankSlots) return SPK_ERR_SIZE;
    if (K < 0 || K > kMaxIndex) return SPK_ERR_SIZE;
    if (op != SPK_OP_SPMM && op != SPK_OP_SDDMM) return SPK_ERR_OP;
    const int dev = current_device();
    if (dev < 0) return SPK_ERR_HIP;
    if (!g_loaded[dev][op]) return SPK_ERR_NO_MODEL;
    const size_t f_bytes = align_up(sizeof(int64_t) * 28), o_bytes = align_up(sizeof(int32_t) * kRankSlots);
    if ((st = check_ws(f_bytes + o_bytes + features_ws_bytes(A->m), ws, ws_bytes))) return st;
    hipStream_t s = static_cast<hipStream_t>(stream);
    char *w = static_cast<char *>(ws);
    int64_t *f = reinterpret_cast<int64_t *>(w);
    int32_t *idx = reinterpret_cast<int32_t *>(w + f_bytes);
    if ((st = hip_status(features_launch(A->m, A->n, A->nnz, A->row_ptr, A->col_idx, f, w + f_bytes + o_bytes, s))))
        return st;
    const int64_t *d = g_dims[dev][op];
    if ((st = hip_status(select_launch(op, f, K, dtype, d[0], d[1], d[2], idx, s)))) return st;
    int32_t host[kRankSlots];
    if (hipMemcpyAsync(host, idx, sizeof(host), hipMemcpyDeviceToHost, s) != hipSuccess) return SPK_ERR_HIP;
    if (hipStreamSynchronize(s) != hipSuccess) return SPK_ERR_HIP;
    int32_t c = 0;
    for (; c < k && host[c] >= 0; ++c)
        if ((st = plan_of_index(op, host[c], K, dtype, &out[c], nullptr))) return st;
    *count = c;
    return c > 0 ? SPK_OK : SPK_ERR_PLAN;
}

int32_t plan_select(const spk_csr *A, int64_t K, int32_t op, int32_t dtype, spk_plan *out, void *ws, size_t ws_bytes,
                    void *stream) {
    if (!out) return SPK_ERR_NULL;
    int32_t count = 0;
    return plan_rank(A, K, op, dtype, 1, out, &count, ws, ws_bytes, stream);
}

int32_t spk_csr_validate(const spk_csr *A, int32_t *rules, void *ws, size_t ws_bytes, void *stream) {
    int32_t st = check_csr(A);
    if (st) return st;
    if (!ws || ws_bytes < 16) return SPK_ERR_WORKSPACE;
    hipStream_t s = static_cast<hipStream_t>(stream);
    int32_t *flag = static_cast<int32_t *>(ws);
    if ((st = hip_status(validate_launch(A->m, A->n, A->nnz, A->row_ptr, A->col_idx, flag, s)))) return st;
    int32_t host = 0;
    if (hipMemcpyAsync(&host, flag, sizeof(int32_t), hipMemcpyDeviceToHost, s) != hipSuccess) return SPK_ERR_HIP;
    if (hipStreamSynchronize(s) != hipSuccess) return SPK_ERR_HIP;
    if (A->m == 0 && A->nnz != 0) host |= SPK_CSR_BAD_END;  // no rows, yet stored entries
    if (rules) *rules = host;
    return host == 0 ? SPK_OK : SPK_ERR_STRUCTURE;
}

}  // extern "C"
