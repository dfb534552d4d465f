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
    SPK_ERR_SIZE = -2,        /* negative size, nnz >= 2^31, n > 2^31-1, or a
                                 shape whose launch under the plan would need a
                                 grid of 2^32 or more threads (one-dimensional
                                 grids count work-items in 32 bits) */
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
    SPK_OP_BSR4 = 4,      /* csr_to_bsr4_count (plan and K ignored) */
    SPK_OP_SELECT = 5     /* plan_select and csr_features (plan and K ignored) */
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
    SPK_VAR_SLAB = 3,  /* row-split over column slabs: one launch per slab
                          of `chunk` columns, so the slab of the dense operand
                          being gathered stays in L2 */
    SPK_VAR_TILE = 4,  /* SpMM: a workgroup owns (256 / lanes) x 4 (or 8)
                          rows and stages each slab of `chunk` rows of B in
                          LDS once, so every staged row serves all of the
                          workgroup's entries in it.  F32 or BF16 operands
                          with K <= 4 * lanes, K and ldb multiples of 16
                          bytes, B and C 16-byte aligned, a slab of at most
                          32 KiB (two are double-buffered in LDS) spanning
                          less than 4 GiB of B (chunk * ldb * element size).
                          SDDMM: the same scheme with slabs of V and each
                          group's rows of U in registers; lanes 16, 32 or 64,
                          K <= 4 * lanes, K and ldv multiples of 16 bytes, V
                          16-byte aligned, ldu a multiple of 4, chunk * ldv *
                          element size below 4 GiB.
                          With flags bit 2, where a row of the dense operand
                          is 128 or 256 bytes, or 512 bytes with F32 rows or
                          (SDDMM) either type (SDDMM: ldu a multiple of 16
                          bytes and U 16-byte aligned too), the work inside a
                          16-lane group is split one entry per 4-lane quad
                          (the lanes field is then not used; rows of 512
                          bytes keep 4 rows per group); other shapes run the
                          split above.  TILE reads entries at 32-bit
                          positions plus up to 63 lanes: nnz above 2^31 - 65
                          gives SPK_ERR_SIZE. */
    SPK_VAR_SLAB16 = 5, /* the column-slab form with 16-bit columns
                           (spmm_slab16 / sddmm_slab16 only): row-split over
                           the slabs of the form, one launch per slab */
    SPK_VAR_DCSR = 6,   /* doubly compressed rows (spmm_dcsr / sddmm_dcsr
                           only): row-split over the non-empty rows */
    SPK_VAR_COO = 7     /* COO entries (sddmm_coo only): flat runs of
                           `chunk` entries whatever their rows */
};

/* An execution plan: plain data, owned by the caller.
 * variant  one of spk_variant.  SpMM: ROWS, MERGE, SLAB, TILE.  SDDMM: ROWS (a
 *          group per row), MERGE (equal runs of entries per group), SLAB,
 *          TILE.
 * lanes    lanes cooperating on one row: 4, 8, 16, 32 or 64.  Each lane
 *          covers `vec` consecutive columns of the dense operand (4 for F32
 *          and BF16, 8 for BF16 SpMM when K allows, 2 for F64), so one pass
 *          covers lanes * vec columns.
 * chunk    SpMM MERGE: rows + entries per group (0: max(256, 4K)).
 *          SDDMM MERGE: entries per group (0: 256).
 *          SLAB: slab width in columns (0: the width whose slab of the dense
 *          operand takes 2 MiB, at least 256).
 *          TILE: slab width in rows of B (SDDMM: of V; 0: the largest power
 *          of two >= 16 whose slab fits 16 KiB).
 * flags    bit 0: use scalar (one element per lane) loads even when the
 *          operands allow 8/16-byte vector loads (not TILE).  bit 1 (TILE
 *          only): 8 rows per lane group instead of 4 (quad splits of 512-byte
 *          rows and SpMM quad splits of BF16 rows of 128 elements keep 4).
 *          bit 2 (TILE only): one entry per 4-lane quad where the rows fit
 *          (see SPK_VAR_TILE).  bit 3 (TILE with bit 2, where the quad
 *          split applies): wide workgroups - slabs up to 32 KiB run in
 *          512-thread workgroups with 2 rows per group, larger slabs (up to
 *          64 KiB, two buffers in 128 KiB of LDS) and all 512-byte rows in
 *          1024-thread workgroups with 1 row per group; more waves per SIMD
 *          than the 256-thread form.  Other bits must be 0.
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

/* SpMM as spmm_csr, for callers that cannot allocate (code under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation): no
 * workspace argument, and nothing is allocated by the call.  Plans that need
 * scratch (MERGE, SLAB) use the library's own device array of
 * spmm_csr_noalloc_max_bytes() bytes (64 MiB), one per GPU, kept until the
 * process ends.  A call whose plan needs more than that returns
 * SPK_ERR_WORKSPACE before launching anything.  Every call on one GPU shares
 * that GPU's array, so calls that overlap on one GPU (other streams, other
 * threads) race: serialise them.  Results are those of spmm_csr on the same
 * arguments (the same kernels). */
int32_t spmm_csr_noalloc(const spk_csr *A, const void *B, int64_t ldb, int32_t b_dtype, int64_t K,
                         void *C, int64_t ldc, const spk_plan *plan, void *stream);

/* Size in bytes of spmm_csr_noalloc's per-GPU scratch array. */
size_t spmm_csr_noalloc_max_bytes(void);

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
 * (chain rule on Eq. (1): dC/dB[j,:] collects the entries of column j, and
 * dC[i,:]/da_p = B[col(p), :], sampled on A's pattern as in Eq. (2)).
 * The transpose (at_row_ptr, at_col_idx, perm) comes from csr_transpose; the
 * values of A^T are gathered through perm.  dtype is F32 (B and G F32) or
 * F64 (everything F64).
 * plan        applies to the A^T SpMM (NULL = plain row-split), as a plan of
 *             spmm_csr would on the matrix A^T (BSR4 is not accepted).
 * dvals_plan  applies to the pattern SDDMM, as a plan of sddmm_csr would on A
 *             (NULL = the default entry-split plan).
 * ws    the two products run one after the other on `stream` and share it:
 *       max(spk_workspace_bytes(SPK_OP_BACKWARD, A, K, plan),
 *           spk_workspace_bytes(SPK_OP_SDDMM, A, K, dvals_plan)) bytes. */
int32_t spmm_csr_backward(const spk_csr *A, const int32_t *at_row_ptr, const int32_t *at_col_idx,
                          const int32_t *perm, const void *B, int64_t ldb, const void *G,
                          int64_t ldg, int32_t dtype, int64_t K, void *dB, int64_t lddb,
                          void *dvals, const spk_plan *plan, const spk_plan *dvals_plan, void *ws,
                          size_t ws_bytes, void *stream);

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

/* ------------------------------------------------------------------------
 * Column-slab form with 16-bit slab-relative column indices.  The paper's
 * host sends a nonzero's column as a 16-bit offset inside the column range of
 * the worker row that owns it, and packs nonzeros by owner (Section III-A,
 * Optimization 1; footprint in Section IV-B).  Here the owners are slabs of
 * `width` columns: a product runs one launch per slab (as SPK_VAR_SLAB), reads
 * 2 bytes of column per entry instead of 4, and needs no per-call search
 * for the slab boundaries.  Built once per pattern on the GPU; values stay in
 * A's own array (the form stores where each run starts in it), so new values
 * need no rebuild.
 * ------------------------------------------------------------------------ */
typedef struct spk_slab16 {
    int64_t m, n, nnz;      /* A's shape and entry count */
    int64_t width;          /* W: columns per slab, 1..65536 */
    int64_t nslabs;         /* S = ceil(n / W), at least 1; S * m < 2^31 - 1 */
    const int32_t *seg;     /* device, S*m + 1: slab-major start of run (s, i)
                               (row i's entries with columns in [sW, (s+1)W));
                               seg[S*m] = nnz */
    const int32_t *apos;    /* device, S*m: position in A of run (s, i)'s first
                               entry (where it would start when empty) */
    const uint16_t *col16;  /* device, nnz: column - s W, slab-major */
} spk_slab16;

/* Scratch bytes of csr_to_slab16 for A and this width (0 for bad arguments). */
size_t slab16_workspace_bytes(const spk_csr *A, int64_t width);

/* Build the form of A's pattern (A canonical): seg (device, S*m + 1), apos
 * (device, S*m) and col16 (device, nnz), caller-allocated.  The result is
 * unique.  ws: slab16_workspace_bytes(A, width) bytes.  SPK_ERR_SIZE when
 * width is outside 1..65536 or S*m >= 2^31 - 1. */
int32_t csr_to_slab16(const spk_csr *A, int64_t width, int32_t *seg, int32_t *apos, uint16_t *col16, void *ws,
                      size_t ws_bytes, void *stream);

/* SpMM (Eq. 1) on the form: C = A B with A's values vals (device, nnz F32 in
 * A's storage order; NULL = pattern, every entry 1).  B F32 or BF16 [n x K],
 * C F32 [m x K], as in spmm_csr.  plan NULL or SPK_VAR_SLAB16 with lanes 4..64
 * and flags bit 0 (scalar loads).  Slab 0 writes C, later slabs add their
 * runs (a row's partial sums are added in slab order: deterministic). */
int32_t spmm_slab16(const spk_slab16 *F, const void *vals, const void *B, int64_t ldb, int32_t b_dtype,
                    int64_t K, void *C, int64_t ldc, const spk_plan *plan, void *stream);

/* SDDMM (Eq. 2) on the form: S[p] = a_p <U[row(p)], V[col(p)]> for every
 * stored entry p, written at p's position in A (S device, nnz F32).  U, V F32
 * or BF16 as in sddmm_csr; plan as for spmm_slab16 (at most 8 register
 * slices of lanes * 4 columns). */
int32_t sddmm_slab16(const spk_slab16 *F, const void *vals, const void *U, int64_t ldu, const void *V,
                     int64_t ldv, int32_t uv_dtype, int64_t K, void *S, const spk_plan *plan, void *stream);

/* ------------------------------------------------------------------------
 * Hyper-sparse forms, for the region above 99% sparsity where the paper's
 * design falls back towards the CPU (Sections I and IV-C; first future-work
 * item, Section V).  Both are per-pattern preprocessing built on the GPU.
 * ------------------------------------------------------------------------ */

/* Doubly compressed rows: A's CSR arrays plus a row order whose first nrows
 * entries are the rows holding an entry (ascending) and the rest the empty
 * rows (ascending).  Products launch groups for the non-empty rows only and
 * write the empty rows' zeros with plain stores. */
typedef struct spk_dcsr {
    int64_t m, n, nnz;
    int64_t nrows;           /* rows holding an entry */
    const int32_t *row_ptr;  /* device, m+1 (A's) */
    const int32_t *col_idx;  /* device, nnz (A's) */
    const void *vals;        /* device, nnz F32 (A's); NULL = pattern */
    const int32_t *order;    /* device, m (from csr_nonempty_order) */
} spk_dcsr;

/* Scratch bytes of csr_nonempty_order for A (0 for bad arguments). */
size_t nonempty_order_workspace_bytes(const spk_csr *A);

/* The row order (device, m) and the number of non-empty rows (*nrows, host).
 * The result is unique.  Synchronises `stream` to return the count. */
int32_t csr_nonempty_order(const spk_csr *A, int32_t *order, int64_t *nrows, void *ws, size_t ws_bytes,
                           void *stream);

/* SpMM (Eq. 1) on the doubly compressed form: C = A B, C fully written (F32),
 * B F32 or BF16 as in spmm_csr.  plan NULL or SPK_VAR_DCSR with lanes 4..64
 * and flags bit 0 (scalar loads). */
int32_t spmm_dcsr(const spk_dcsr *D, const void *B, int64_t ldb, int32_t b_dtype, int64_t K, void *C,
                  int64_t ldc, const spk_plan *plan, void *stream);

/* SDDMM (Eq. 2) on the doubly compressed form (S device [nnz] F32, A's
 * order); plan as for spmm_dcsr, at most 8 register slices of lanes * 4
 * columns. */
int32_t sddmm_dcsr(const spk_dcsr *D, const void *U, int64_t ldu, const void *V, int64_t ldv, int32_t uv_dtype,
                   int64_t K, void *S, const spk_plan *plan, void *stream);

/* COO row index of A's entries: rowidx device [nnz], rowidx[p] = the row
 * holding entry p. */
int32_t csr_row_index(const spk_csr *A, int32_t *rowidx, void *stream);

/* SDDMM (Eq. 2) over COO entries: flat runs of `chunk` entries (0: 64)
 * whatever their rows, each entry's row of U gathered like its row of V, so
 * the work splits evenly however the entries fall into rows.  A's col_idx
 * and vals (F32 or NULL), rowidx from csr_row_index.  plan NULL or
 * SPK_VAR_COO with lanes 4..64 (NULL: 8, widened until K fits 8 register
 * slices) and flags bit 0. */
int32_t sddmm_coo(const spk_csr *A, const int32_t *rowidx, const void *U, int64_t ldu, const void *V,
                  int64_t ldv, int32_t uv_dtype, int64_t K, void *S, const spk_plan *plan, void *stream);

/* ------------------------------------------------------------------------
 * Back-to-back products with the intermediate kept on chip (the paper's
 * future work on consecutive operations whose result stays resident,
 * Section V): attention on A's pattern,
 *   S = A (.) (U V^T)      scores on A's stored entries (Eq. 2)
 *   P = softmax of each row's stored scores
 *   O = P B                (Eq. 1 with the probabilities as values)
 * ------------------------------------------------------------------------ */

/* The whole chain in one pass: P is never written.  A's values scale the
 * scores (NULL: pattern, every a_p = 1; F32 only).  U [m x K1], V [n x K1]
 * and B [n x K2] device, all of dtype (SPK_F32 or SPK_BF16), row-major with
 * leading dimensions ldu, ldv >= K1 and ldb >= K2 (required whenever K1 or K2
 * is positive, even when nnz = 0).  O device [m x K2] F32, ldo >= K2, fully
 * written; a row without stored entries gets zeros.  lse device [m] F32,
 * nullable: log of each row's normaliser, max + log(sum exp(S - max))
 * (-inf for an empty row).
 * plan  NULL or a plan with flags bit 0 (scalar loads) and lanes 4..64 per
 *       group (at most 8 register slices of lanes * 4 columns of
 *       max(K1, K2); NULL: 8 lanes, widened as needed):
 *       SPK_VAR_MERGE (the NULL plan's) - each group takes a run of `chunk`
 *         entries (0: 512) whatever the rows, so rows of very different
 *         lengths cost no imbalance; a row cut by a run's ends leaves a
 *         partial state (maximum, normaliser, K2 sums) that a fix-up
 *         combines in run order (for a row cut into more than 64 pieces,
 *         64 pieces at a time first, then those folds in order);
 *       SPK_VAR_ROWS - one group per row (no workspace).
 *       Each row's entries are taken in storage order with an online
 *       (rescaled) softmax and fixed reductions: deterministic.
 * ws    attention_workspace_bytes(A, K2, plan) bytes (MERGE: per run two
 *       partial states and two folds). */
int32_t sddmm_softmax_spmm(const spk_csr *A, const void *U, int64_t ldu, const void *V, int64_t ldv,
                           int64_t K1, const void *B, int64_t ldb, int64_t K2, int32_t dtype, float *O,
                           int64_t ldo, float *lse, const spk_plan *plan, void *ws, size_t ws_bytes,
                           void *stream);

/* Workspace bytes of sddmm_softmax_spmm for A, K2 and plan (0 for ROWS plans
 * and for bad arguments). */
size_t attention_workspace_bytes(const spk_csr *A, int64_t K2, const spk_plan *plan);

/* The middle step alone, for the unfused chain (sddmm_csr, this, spmm_csr
 * with S as values): S (device [nnz] F32, A's storage order) holds scores on
 * entry and each row's softmax probabilities on return; lse as above
 * (nullable).  Balanced over runs of entries like the MERGE attention, so a
 * row of any length costs no imbalance.
 * ws    row_softmax_workspace_bytes(A) bytes (each row's maximum and
 *       normaliser, the runs' partial states). */
int32_t csr_row_softmax(const spk_csr *A, float *S, float *lse, void *ws, size_t ws_bytes, void *stream);

/* Workspace bytes of csr_row_softmax for A (0 for bad arguments). */
size_t row_softmax_workspace_bytes(const spk_csr *A);

/* ------------------------------------------------------------------------
 * Learned plan selection.  Not in the paper: the paper's kernels expose
 * compile-time tile parameters (rows buffered per chunk, columns per worker
 * row, Section III-A and IV-C) chosen by sweeping; here a small network maps
 * sparsity features to the fastest plan and an exhaustive timed search is
 * the fallback and the yardstick of its regret.
 * ------------------------------------------------------------------------ */

/* Number of plans in an op's plan list (SPK_OP_SPMM: 30, SPK_OP_SDDMM: 29),
 * or 0 for other ops. */
int32_t plan_count(int32_t op);

/* Plan `index` of an op's plan list:
 *   0..14   variant v = index / 5 (ROWS, MERGE, SLAB) with lanes 4 << (index % 5)
 *           (SDDMM MERGE plans use 256 entries per group);
 *   SpMM 15 SPK_VAR_BSR4 (lanes 64);
 *   TILE    SpMM 16..23, SDDMM 15..22: the plain lanes for K (SDDMM at least
 *           16), slabs of 16 KiB (SpMM 16, 18, 20, 21) or 32 KiB (17, 19, 22,
 *           23) of F32 rows, 8 rows per group for the odd indices, one entry
 *           per quad (flags bit 2) for the last four;
 *   wide    SpMM 24, 25 / SDDMM 23, 24: one entry per quad in wide
 *           workgroups (flags 12), slabs of 32 and 64 KiB of F32 rows;
 *   SLAB16  SpMM 26, 27 / SDDMM 25, 26: the column-slab form with 4 (SpMM;
 *           SDDMM 2) or 8 MiB of F32 rows per slab (between 256 and 65536
 *           columns); SpMM 26 the plain lanes, SDDMM and SpMM 27 8 lanes
 *           widened until a lane holds at most 8 columns (SpMM 27: at least
 *           16, at most the plain lanes);
 *   DCSR    SpMM 28 (plain lanes), 29 (4 lanes) / SDDMM 27;
 *   COO     SDDMM 28: 16 lanes, runs of 16 entries.
 * Slab widths count F32 rows; BF16 slabs of the same width take half the
 * bytes.  *valid is 1 when the plan suits dense width K and the dense dtype
 * (SPK_F32, SPK_BF16 or SPK_F64: rows lanes not wider than twice K rounded up
 * to a power of two, at least 16; SDDMM: at most 8 register slices; TILE:
 * K a multiple of 8 in [8, 256]; wide 64 KiB: rows the quad split takes;
 * F64 only plans 0..14).  Host only. */
int32_t plan_of_index(int32_t op, int32_t index, int64_t K, int32_t dtype, spk_plan *out, int32_t *valid);

/* Integer structural features of A into features (device, 28 int64):
 *   0 m, 1 n, 2 nnz, 3..22 row-length histogram (bin 0 empty rows, bin b in
 *   1..18 lengths in [2^(b-1), 2^b), bin 19 lengths >= 2^18), 23 max row
 *   length, 24 sum of squared row lengths, 25 max |i - j| over entries,
 *   26 sum of |i - j|, 27 number of aligned 4x4 blocks holding an entry.
 * ws    spk_workspace_bytes(SPK_OP_SELECT, ...) bytes. */
int32_t csr_features(const spk_csr *A, int64_t *features, void *ws, size_t ws_bytes, void *stream);

/* The 33 network inputs from features (device, 28), K and the dense
 * operands' dtype, into x (device, 33):
 *   x0 log2(1+m)/20, x1 log2(1+n)/20, x2 log2(1+nnz)/30, x3..x22 fraction of
 *   rows per length bin, x23 log2(1+max len)/20, x24 log2(1+mean len)/20,
 *   x25 log2(1+cv)/4 (cv: std / mean of row lengths), x26 log2(1+max|i-j|)/20,
 *   x27 mean |i-j| / n, x28 nnz / (16 blocks), x29 log2(K)/8,
 *   x30 1 + log10(density)/5, x31 1, x32 1 for SPK_BF16 and 0 otherwise.
 *   Binary32 arithmetic. */
int32_t selector_inputs(const int64_t *features, int64_t K, int32_t dtype, float *x, void *stream);

/* Network y = W3 relu(W2 relu(W1 x + b1) + b2) + b3 for `batch` rows of X
 * (device [batch x F]) into Y (device [batch x P]).  params (device) holds
 * W1[H][F], b1[H], W2[H][H], b2[H], W3[P][H], b3[P] contiguously.
 * F <= 64, H <= 192, P <= 32. */
int32_t mlp_forward(const float *params, int64_t F, int64_t H, int64_t P, const float *X, int64_t batch,
                    float *Y, void *stream);

/* Scratch bytes of mlp_loss_grad for these sizes. */
size_t mlp_workspace_bytes(int64_t F, int64_t H, int64_t P, int64_t batch);

/* Masked mean squared error L = sum mask (y - T)^2 / (2 count) (count = number
 * of nonzero mask entries; mask values other than 0/1 weigh the terms) and
 * its gradient with respect to params (same
 * layout) for a batch: X [batch x F], T and mask [batch x P], all device.
 * loss: device, 1 float.  Gradients are summed over samples in order (the
 * result does not vary between runs). */
int32_t mlp_loss_grad(const float *params, int64_t F, int64_t H, int64_t P, const float *X, const float *T,
                      const float *mask, int64_t batch, float *grads, float *loss, void *ws,
                      size_t ws_bytes, void *stream);

/* One Adam step (Kingma and Ba, Algorithm 1) on `count` parameters (device):
 * mom = b1 mom + (1-b1) g, vel = b2 vel + (1-b2) g^2,
 * params -= lr (mom / (1-b1^step)) / (sqrt(vel / (1-b2^step)) + eps). */
int32_t adam_update(float *params, const float *grads, float *mom, float *vel, int64_t count, float lr,
                    float beta1, float beta2, float eps, int64_t step, void *stream);

/* Load a trained selector for op (SPK_OP_SPMM or SPK_OP_SDDMM) on the current
 * device from host memory: mean[F], scale[F] (inputs are standardised as
 * (x - mean) / scale), then the F x H x P parameters as for mlp_forward.
 * F must be 33 and P the op's plan count.  Synchronous; copies into a static
 * table of the library (no allocation). */
int32_t selector_load(int32_t op, const float *table, int64_t F, int64_t H, int64_t P);

/* Learned plan for op on A with dense width K and dense dtype: features,
 * inputs, network and the argmin of its outputs over the plans valid for K
 * and dtype, all on the device.  Synchronises `stream` to return the plan in
 * *out.  SPK_ERR_NO_MODEL when no selector is loaded for op on this device
 * (callers then fall back to a timed search).
 * ws: spk_workspace_bytes(SPK_OP_SELECT, ...) bytes. */
int32_t plan_select(const spk_csr *A, int64_t K, int32_t op, int32_t dtype, spk_plan *out, void *ws,
                    size_t ws_bytes, void *stream);

/* The network's k best plans (1 <= k <= 32) for op on A with dense width K
 * and dtype, in ascending predicted time, into out[0 .. *count) (host;
 * *count <= k, the number of plans valid for K and dtype).  Same features,
 * network and workspace as plan_select (whose plan is out[0]); a caller may
 * time these few candidates and keep the fastest, which guards against a
 * mispredicted first choice at the cost of a short timed search.
 * Synchronises `stream`. */
int32_t plan_rank(const spk_csr *A, int64_t K, int32_t op, int32_t dtype, int32_t k, spk_plan *out,
                  int32_t *count, void *ws, size_t ws_bytes, void *stream);

/* Rules of canonical CSR, as bits of spk_csr_validate's *rules.  The paper
 * sends CSR with 32-bit column indices (Section III-A) and leaves order and
 * duplicates open; the library reads it as the canonical form. */
enum spk_csr_rule {
    SPK_CSR_BAD_START = 1,  /* m > 0 and row_ptr[0] != 0 */
    SPK_CSR_BAD_END = 2,    /* row_ptr[m] != nnz (m = 0: nnz != 0) */
    SPK_CSR_BAD_ORDER = 4,  /* a row with row_ptr[i+1] < row_ptr[i], row_ptr[i] < 0
                               or row_ptr[i+1] > nnz */
    SPK_CSR_BAD_COL = 8,    /* a column outside [0, n) (rows passing rule 4) */
    SPK_CSR_BAD_SORT = 16,  /* neighbours in decreasing column order (same rows) */
    SPK_CSR_BAD_DUP = 32    /* neighbours with equal columns (same rows) */
};

/* Opt-in O(nnz) structural check of A against canonical CSR (above).  Only
 * rows whose range lies inside [0, nnz] are read, so any int32 contents of
 * row_ptr are safe to check.
 * rules  host, nullable: receives the OR of the spk_csr_rule bits A breaks
 *        (0 when it is canonical).
 * ws     device, at least 16 bytes.  Synchronises `stream`.  Returns SPK_OK,
 *        SPK_ERR_STRUCTURE, or an argument error. */
int32_t spk_csr_validate(const spk_csr *A, int32_t *rules, void *ws, size_t ws_bytes, void *stream);

#ifdef __cplusplus
}
#endif

#endif /* SPK_H */
