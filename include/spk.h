/*
 * spk.h - C ABI of the MI355X (gfx950) sparse-product library.
 *
 * Two kernels from "Exploring Sparse Matrix Multiplication Kernels on the
 * Cerebras CS-3" (Shah, Di, Becchi), re-designed for one MI355X:
 *
 *   SpMM   C = A B            Section II-A, Eq. (1) (the paper writes Y = A X)
 *   SDDMM  S = A (.) (U V^T)  Section II-A, Eq. (2) (the paper writes
 *                             Y = A (.) (B C); here U = B and V = C^T), one
 *                             output per stored entry of A, never forming U V^T.
 *
 * plus the backward of SpMM (dB = A^T G, dvals = SDDMM(pattern, G, B)), the
 * CSR transpose it needs, and a learned plan selector.
 *
 * Conventions shared by every call
 * --------------------------------
 * - A is CSR (Section III-A: 32-bit column indices, 32-bit float values):
 *   row_ptr[m+1] and col_idx[nnz] int32, canonical (row_ptr[0] = 0, monotone,
 *   row_ptr[m] = nnz, columns strictly increasing within a row), nnz < 2^31.
 *   Empty rows are allowed and give zero rows of C.  Non-square A is allowed.
 * - Every pointer named "device" is device memory of the current HIP device;
 *   every dense matrix is row-major with the stated leading dimension (in
 *   elements).  The caller owns every buffer; the library never allocates
 *   device memory.  Scratch memory comes from the caller as a workspace whose
 *   size spk_workspace_bytes() reports (it may be NULL when that size is 0).
 * - Outputs must not alias inputs.  Inputs are never written.
 * - `stream` is a hipStream_t (NULL = the null stream).  All calls are
 *   asynchronous on it except plan_select, which synchronises the stream to
 *   return its choice on the host.
 * - Calls return SPK_OK (0) or a negative status; nothing is thrown across the
 *   ABI.  O(1) argument checks always run before any launch.  Faults inside
 *   a kernel surface at the caller's next synchronisation.
 * - K = 0 or m = 0 is a no-op.  nnz = 0 writes zeros to C.
 */
#ifndef SPK_H
#define SPK_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* Element types. */
enum spk_dtype {
    SPK_F32 = 0,  /* IEEE binary32 */
    SPK_BF16 = 1, /* bfloat16 dense operands (B, U, V); values and outputs stay F32 */
    SPK_F64 = 2   /* binary64 throughout: used for finite-difference checks only */
};

/* Status codes. */
enum spk_status {
    SPK_OK = 0,
    SPK_ERR_NULL = -1,        /* a required pointer is NULL */
    SPK_ERR_SIZE = -2,        /* negative size, nnz >= 2^31, or n > 2^31-1 */
    SPK_ERR_DTYPE = -3,       /* unsupported dtype combination */
    SPK_ERR_LD = -4,          /* leading dimension smaller than K */
    SPK_ERR_WORKSPACE = -5,   /* workspace NULL or smaller than required */
    SPK_ERR_PLAN = -6,        /* plan fields out of range for this call */
    SPK_ERR_HIP = -7,         /* the HIP runtime rejected a launch */
    SPK_ERR_STRUCTURE = -8,   /* spk_csr_validate found a non-canonical CSR */
    SPK_ERR_OP = -9,          /* unknown op code */
    SPK_ERR_NO_MODEL = -10    /* plan_select called before selector_load */
};

/* Operation codes (workspace queries and plan selection). */
enum spk_op {
    SPK_OP_SPMM = 0,      /* spmm_csr */
    SPK_OP_SDDMM = 1,     /* sddmm_csr */
    SPK_OP_BACKWARD = 2,  /* spmm_csr_backward (the plan applies to A^T G) */
    SPK_OP_TRANSPOSE = 3, /* csr_transpose (plan ignored) */
    SPK_OP_BSR4 = 4       /* csr_to_bsr4_count (plan and K ignored) */
};

/* A sparse matrix in CSR form. */
typedef struct spk_csr {
    int64_t m, n, nnz;      /* rows, columns, stored entries */
    const int32_t *row_ptr; /* device, m+1 */
    const int32_t *col_idx; /* device, nnz */
    const void *vals;       /* device, nnz of vals_dtype; NULL = every entry is 1 */
    int32_t vals_dtype;     /* SPK_F32, or SPK_F64 with F64 dense operands */
} spk_csr;

/* Kernel variants. */
enum spk_variant {
    SPK_VAR_ROWS = 0,  /* row-split: a group of `lanes` lanes owns one row */
    SPK_VAR_MERGE = 1, /* merge-path: each group owns an equal share of
                          rows + entries; split rows are fixed up in order */
    SPK_VAR_BSR4 = 2,  /* 4x4 block-sparse with matrix cores (SpMM only;
                          needs the block form from csr_to_bsr4) */
    SPK_VAR_SLAB = 3   /* row-split over column slabs: one launch per slab
                          of `chunk` columns, so the slab of the dense operand
                          being gathered stays in L2 */
};

/* An execution plan: plain data, owned by the caller.
 * variant  one of spk_variant.  SpMM: ROWS, MERGE, SLAB.  SDDMM: ROWS (a
 *          group per row), MERGE (equal runs of entries per group), SLAB.
 * lanes    lanes cooperating on one row: 4, 8, 16, 32 or 64.  Each lane
 *          covers `vec` consecutive columns of the dense operand (4 for F32
 *          and BF16, 8 for BF16 SpMM when K allows, 2 for F64), so one pass
 *          covers lanes * vec columns.
 * chunk    SpMM MERGE: rows + entries per group (0: max(256, 4K)).
 *          SDDMM MERGE: entries per group (0: 256).
 *          SLAB: slab width in columns (0: the width whose slab of the dense
 *          operand takes 2 MiB, at least 256).
 * flags    bit 0: use scalar (one element per lane) loads even when the
 *          operands allow 8/16-byte vector loads; other bits must be 0.
 * Vector loads are used when K and the leading dimensions are multiples of
 * the vector width and the base pointers are aligned to it; otherwise the
 * call falls back to scalar loads by itself.
 * A NULL plan means the plain method: row-split SpMM with the smallest
 * power-of-two `lanes` >= K/4 (at most 64), and entry-split (MERGE) SDDMM
 * with lanes = 8 (widened until K fits in 8 register slices). */
typedef struct spk_plan {
    int32_t variant;
    int32_t lanes;
    int32_t chunk;
    int32_t flags;
} spk_plan;

/* Size in bytes of the workspace that `op` needs for this matrix, K and plan
 * (0 when none).  Returns 0 for invalid arguments as well. */
size_t spk_workspace_bytes(int32_t op, const spk_csr *A, int64_t K, const spk_plan *plan);

/* Text of a status code (static storage). */
const char *spk_strerror(int32_t status);

/* SpMM, Eq. (1):  C[i, :] = sum over stored (i, j) of a_ij * B[j, :].
 * B     device [n x K] of b_dtype (SPK_F32, SPK_BF16, or SPK_F64 when
 *       A->vals_dtype is SPK_F64), leading dimension ldb >= K.
 * C     device [m x K], F32 (F64 in F64 mode), leading dimension ldc >= K;
 *       fully overwritten.
 * plan  NULL or a plan (variants ROWS, MERGE, SLAB; BSR4 goes through spmm_bsr4).
 * ws    workspace of spk_workspace_bytes(SPK_OP_SPMM, ...) bytes. */
int32_t spmm_csr(const spk_csr *A, const void *B, int64_t ldb, int32_t b_dtype, int64_t K,
                 void *C, int64_t ldc, const spk_plan *plan, void *ws, size_t ws_bytes,
                 void *stream);

/* SDDMM, Eq. (2):  S[p] = a_p * <U[row(p), :], V[col(p), :]> for every stored
 * entry p (a_p = 1 when A->vals is NULL: the pattern-only form used by the
 * backward).
 * U     device [m x K], V device [n x K], both of uv_dtype (F32 or BF16; F64
 *       in F64 mode), leading dimensions ldu, ldv >= K.
 * S     device [nnz], F32 (F64 in F64 mode), in A's storage order. */
int32_t sddmm_csr(const spk_csr *A, const void *U, int64_t ldu, const void *V, int64_t ldv,
                  int32_t uv_dtype, int64_t K, void *S, const spk_plan *plan, void *ws,
                  size_t ws_bytes, void *stream);

/* Stable transpose of A's pattern (needed for dB = A^T G).
 * at_row_ptr device [n+1], at_col_idx device [nnz], perm device [nnz]:
 * row j of A^T lists the rows i holding column j in increasing order, and
 * perm[q] is the position in A of entry q of A^T.  The result is unique.
 * ws    spk_workspace_bytes(SPK_OP_TRANSPOSE, ...) bytes. */
int32_t csr_transpose(const spk_csr *A, int32_t *at_row_ptr, int32_t *at_col_idx,
                      int32_t *perm, void *ws, size_t ws_bytes, void *stream);

/* Backward of C = A B for a loss with dL/dC = G (device [m x K]):
 *   dB    = A^T G                    device [n x K], nullable (skipped)
 *   dvals = SDDMM(pattern of A, G, B) device [nnz],  nullable (skipped)
 * The transpose (at_row_ptr, at_col_idx, perm) comes from csr_transpose; the
 * values of A^T are gathered through perm.  dtype is F32 (B and G F32, or
 * BF16 operands with F32 outputs) or F64 (everything F64).
 * plan  applies to the A^T SpMM (NULL = plain); the SDDMM uses its default.
 * ws    spk_workspace_bytes(SPK_OP_BACKWARD, ...) bytes. */
int32_t spmm_csr_backward(const spk_csr *A, const int32_t *at_row_ptr, const int32_t *at_col_idx,
                          const int32_t *perm, const void *B, int64_t ldb, const void *G,
                          int64_t ldg, int32_t dtype, int64_t K, void *dB, int64_t lddb,
                          void *dvals, const spk_plan *plan, void *ws, size_t ws_bytes,
                          void *stream);

/* A 4x4 block-sparse matrix (block CSR): block row I holds rows 4I..4I+3 of
 * A, block column J columns 4J..4J+3; edge blocks are padded with zeros. */
typedef struct spk_bsr4 {
    int64_t m, n;             /* rows and columns of A */
    int64_t nblocks;          /* stored 4x4 tiles */
    const int32_t *b_row_ptr; /* device, ceil(m/4)+1 */
    const int32_t *b_col;     /* device, nblocks, ascending within a block row */
    const float *b_vals;      /* device, nblocks * 16, row-major 4x4 tiles */
} spk_bsr4;

/* CSR -> 4x4 block form, first half: b_row_ptr (device, ceil(m/4)+1) of the
 * blocks holding at least one stored entry, and their number in *nblocks
 * (host).  ws: spk_workspace_bytes(SPK_OP_BSR4, ...) bytes.  Synchronises
 * `stream` (the caller allocates the block arrays from *nblocks). */
int32_t csr_to_bsr4_count(const spk_csr *A, int32_t *b_row_ptr, int64_t *nblocks, void *ws,
                          size_t ws_bytes, void *stream);

/* Second half: block columns b_col (device, nblocks) and tiles b_vals (device,
 * nblocks * 16 floats; zeros where A stores nothing, ones in pattern mode).
 * A->vals must be F32 or NULL. */
int32_t csr_to_bsr4_fill(const spk_csr *A, const int32_t *b_row_ptr, int32_t *b_col, float *b_vals,
                         void *stream);

/* SpMM on the block form with matrix cores: C = A B as in spmm_csr (C F32,
 * B F32 or BF16).  The block form computes exactly the CSR product: padded
 * zeros add nothing. */
int32_t spmm_bsr4(const spk_bsr4 *A, const void *B, int64_t ldb, int32_t b_dtype, int64_t K, void *C,
                  int64_t ldc, void *stream);

/* Opt-in O(nnz) structural check of A (canonical CSR as described above).
 * ws    at least 16 bytes.  Synchronises `stream`.  Returns SPK_OK or
 *       SPK_ERR_STRUCTURE. */
int32_t spk_csr_validate(const spk_csr *A, void *ws, size_t ws_bytes, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* SPK_H */
