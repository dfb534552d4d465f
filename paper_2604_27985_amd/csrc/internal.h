// internal.h - host-side launch descriptors shared by the library's sources.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "../../include/spk.h"

namespace spk {

constexpr size_t kAlign = 256;
inline size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

// The column-slab form with 16-bit slab-relative columns (slab16.hip).
struct Slab16View {
    const int32_t *seg = nullptr, *apos = nullptr;
    const uint16_t *col16 = nullptr;
    int64_t width = 0, nslabs = 0;
};

// Hyper-sparse forms (hyper.hip): the row order of the doubly compressed
// form (non-empty rows first) and the COO row index of every entry.
struct HyperView {
    const int32_t *order = nullptr;   // DCSR: m rows, the first nrows non-empty
    int64_t nrows = 0;
    const int32_t *rowidx = nullptr;  // COO: row of every entry
};

struct SpmmArgs {
    int64_t m, n, nnz, K;
    const int32_t *rp, *ci;
    const void *vals;      // F32 or F64 (nullable: all ones)
    const int32_t *vperm;  // nullable: value of entry q is vals[vperm[q]]
    const void *B;
    int64_t ldb;
    int32_t b_dtype;
    void *C;
    int64_t ldc;
    int32_t variant, lanes, vec;
    int64_t chunk;
    void *ws;
    int32_t rows_per_group = 4;  // TILE: rows each lane group owns (4 or 8)
    int32_t quad_split = 0;      // TILE: one entry per 4-lane quad, 16-lane groups
    Slab16View s16{};            // SLAB16: the column-slab form (ci unused)
    HyperView hv{};              // DCSR
};

struct SddmmArgs {
    int64_t m, n, nnz, K;
    const int32_t *rp, *ci;
    const void *vals;  // nullable
    const void *U;
    int64_t ldu;
    const void *V;
    int64_t ldv;
    int32_t uv_dtype;
    void *S;
    int32_t variant, lanes, vec;
    int64_t chunk;
    void *ws;
    int32_t rows_per_group = 4;  // TILE: rows each lane group owns (4 or 8)
    int32_t quad_split = 0;      // TILE: one entry per 4-lane quad, 16-lane groups
    Slab16View s16{};            // SLAB16: the column-slab form (ci unused)
    HyperView hv{};              // DCSR, COO
};

// Column slabs of the SLAB variants: nslabs slabs of `width` columns; the
// workspace holds the (nslabs - 1) interior boundaries of every row.
struct SlabLayout {
    int64_t width, nslabs;
    size_t total;
};

inline SlabLayout slab_layout(int64_t m, int64_t n, int64_t width) {
    SlabLayout L;
    L.width = width > 0 ? width : 1;
    L.nslabs = n > 0 ? (n + L.width - 1) / L.width : 1;
    L.total = L.nslabs > 1 ? align_up(sizeof(int32_t) * static_cast<size_t>(m) * static_cast<size_t>(L.nslabs - 1)) : 0;
    return L;
}

// Workspace of the merge-path SpMM: share start rows, carry rows, carry sums.
struct MergeLayout {
    int64_t items, ngroups;
    size_t part_off, row_off, val_off, total;
};

inline MergeLayout merge_layout(int64_t m, int64_t nnz, int64_t K, int64_t chunk, size_t acc_size) {
    MergeLayout L;
    L.items = chunk;
    const int64_t total = m + nnz;
    L.ngroups = total > 0 ? (total + chunk - 1) / chunk : 0;
    L.part_off = 0;
    L.row_off = align_up(sizeof(int32_t) * static_cast<size_t>(L.ngroups + 1));
    L.val_off = L.row_off + align_up(sizeof(int32_t) * static_cast<size_t>(L.ngroups));
    L.total = L.val_off + align_up(acc_size * static_cast<size_t>(L.ngroups) * static_cast<size_t>(K));
    return L;
}

hipError_t spmm_launch(const SpmmArgs &a, hipStream_t s);
// Interior column-slab boundaries of every row into bnd[(nslabs-1) * m].
hipError_t slab_bounds_launch(int64_t m, const int32_t *rp, const int32_t *ci, int64_t width, int64_t nslabs,
                              int32_t *bnd, hipStream_t s);
hipError_t sddmm_launch(const SddmmArgs &a, hipStream_t s);
hipError_t zero_fill(void *C, int64_t m, int64_t K, int64_t ld, int32_t dtype, hipStream_t s);

// 4x4 block-sparse SpMM on matrix cores (bsr.hip).
struct Bsr4Args {
    int64_t m, n, K;
    const int32_t *b_rp, *b_col;
    const float *b_vals;
    const void *B;
    int64_t ldb;
    int32_t b_dtype, vec;
    float *C;
    int64_t ldc;
};
hipError_t bsr4_count_launch(int64_t m, const int32_t *rp, const int32_t *ci, int32_t *counts, hipStream_t s);
hipError_t bsr4_fill_launch(int64_t m, const int32_t *rp, const int32_t *ci, const float *vals, const int32_t *b_rp,
                            int32_t *b_col, float *b_vals, hipStream_t s);
hipError_t bsr4_spmm_launch(const Bsr4Args &a, hipStream_t s);

// Learned plan selection (selector.hip).
size_t features_ws_bytes(int64_t m);
hipError_t features_launch(int64_t m, int64_t n, int64_t nnz, const int32_t *rp, const int32_t *ci, int64_t *f,
                           void *ws, hipStream_t s);
hipError_t inputs_launch(const int64_t *f, int64_t K, int32_t dtype, float *x, hipStream_t s);
bool mlp_dims_ok(int64_t F, int64_t H, int64_t P);
hipError_t mlp_forward_launch(const float *params, int64_t F, int64_t H, int64_t P, const float *X, int64_t batch,
                              float *Y, hipStream_t s);
size_t mlp_train_ws_bytes(int64_t F, int64_t H, int64_t P, int64_t batch);
hipError_t mlp_loss_grad_launch(const float *params, int64_t F, int64_t H, int64_t P, const float *X, const float *T,
                                const float *mask, int64_t batch, float *grads, float *loss, void *ws, hipStream_t s);
hipError_t adam_launch(float *w, const float *g, float *mom, float *vel, int64_t count, float lr, float b1, float b2,
                       float eps, int64_t step, hipStream_t s);
hipError_t selector_table_load(int32_t op, const float *host_table, int64_t F, int64_t H, int64_t P);
hipError_t select_launch(int32_t op, const int64_t *f, int64_t K, int32_t dtype, int64_t F, int64_t H, int64_t P,
                         int32_t *out, hipStream_t s);
bool plan_valid_host(int32_t op, int idx, int64_t K, int32_t dtype);

// In-place exclusive scan of int32 values (transpose.hip).
size_t scan_ws_bytes_i32(int64_t count);
hipError_t exclusive_scan_i32(int32_t *data, int64_t count, void *ws, hipStream_t s);

// CSR transpose (transpose.hip).
size_t transpose_ws_bytes(int64_t m, int64_t n, int64_t nnz);
hipError_t transpose_launch(int64_t m, int64_t n, int64_t nnz, const int32_t *rp, const int32_t *ci,
                            int32_t *trp, int32_t *tci, int32_t *perm, void *ws, hipStream_t s);

// Column-slab form with 16-bit columns (slab16.hip): runs of S slabs of W
// columns over m rows; the workspace serves the scan of S m + 1 run starts.
size_t slab16_ws_bytes(int64_t m, int64_t S);
hipError_t slab16_build_launch(int64_t m, int64_t nnz, const int32_t *rp, const int32_t *ci, int64_t W, int64_t S,
                               int32_t *seg, int32_t *apos, uint16_t *col16, void *ws, hipStream_t s);

// Attention on A's pattern in one pass (attn.hip): O = softmax_rows(A (.) U V^T) B.
struct AttnArgs {
    int64_t m, n, nnz, K1, K2;
    const int32_t *rp, *ci;
    const float *vals;  // nullable: every entry 1
    const void *U;
    int64_t ldu;
    const void *V;
    int64_t ldv;
    const void *B;
    int64_t ldb;
    int32_t dtype;  // of U, V and B: SPK_F32 or SPK_BF16
    float *O;
    int64_t ldo;
    float *lse;  // nullable
    int32_t lanes, vec;
    int32_t variant = SPK_VAR_ROWS;  // ROWS: a group per row; MERGE: equal runs of entries
    int64_t items = 0;               // MERGE: entries per run
    void *ws = nullptr;              // MERGE: the runs' partial states
};

// Workspace of the entry-split attention: per run two slots (a row id, the
// running maximum and normaliser, K2 accumulated values), and with `fold`
// two more slots of (maximum, normaliser, K2 values) per run for the partial
// states of long rows folded 64 pieces at a time.
struct AttnLayout {
    int64_t items, ngroups;
    size_t row_off, ml_off, acc_off, fold_ml_off, fold_acc_off, total;
};

inline AttnLayout attn_layout(int64_t nnz, int64_t K2, int64_t items, bool fold = false) {
    AttnLayout L;
    L.items = items > 0 ? items : 1;
    L.ngroups = nnz > 0 ? (nnz + L.items - 1) / L.items : 0;
    const size_t ml_bytes = align_up(sizeof(float) * 4 * static_cast<size_t>(L.ngroups));
    const size_t acc_bytes = align_up(sizeof(float) * 2 * static_cast<size_t>(L.ngroups) * static_cast<size_t>(K2));
    L.row_off = 0;
    L.ml_off = align_up(sizeof(int32_t) * 2 * static_cast<size_t>(L.ngroups));
    L.acc_off = L.ml_off + ml_bytes;
    L.fold_ml_off = L.acc_off + acc_bytes;
    L.fold_acc_off = L.fold_ml_off + (fold ? ml_bytes : 0);
    L.total = L.fold_acc_off + (fold ? acc_bytes : 0);
    return L;
}
hipError_t attn_launch(const AttnArgs &a, hipStream_t s);
// Row softmax of stored scores in place (the unfused middle step), balanced
// over runs of kSoftmaxItems entries; the workspace holds each row's maximum
// and normaliser and the runs' partial states.
constexpr int64_t kSoftmaxItems = 256;
size_t row_softmax_ws_bytes(int64_t m, int64_t nnz);
hipError_t row_softmax_launch(int64_t m, int64_t nnz, const int32_t *rp, float *S, float *lse, void *ws, hipStream_t s);

// Hyper-sparse preprocessing (hyper.hip).
size_t nonempty_order_ws_bytes(int64_t m);
hipError_t nonempty_order_launch(int64_t m, const int32_t *rp, int32_t *order, int32_t *count_dev, void *ws,
                                 hipStream_t s);
hipError_t row_index_launch(int64_t m, const int32_t *rp, int32_t *rowidx, hipStream_t s);

// Structural validation (transpose.hip): writes 0 to *flag_dev when A is
// canonical, a positive code otherwise.
hipError_t validate_launch(int64_t m, int64_t n, int64_t nnz, const int32_t *rp, const int32_t *ci,
                           int32_t *flag_dev, hipStream_t s);

}  // namespace spk
