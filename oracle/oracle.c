/*
 * oracle.c - plain, slow, FP64 CPU reference for the sparse products.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the library links, loads or calls this
 * file; only the tests, the smoke check and the CPU-baseline leg of the
 * benchmark do.  It shares no code, header or helper with the GPU library.
 *
 * Every routine is the plain definition written out as loops, in double
 * precision, with no blocking, fusion or reordering beyond the definition.
 * Where a routine is parallel (OpenMP over output rows), each output element is
 * still produced by one thread in the definition's order, so results do not
 * depend on the thread count.
 *
 * Sources:
 *   - SpMM, Section II-A, Eq. (1): Y = A X with A sparse, X dense.
 *   - SDDMM, Section II-A, Eq. (2): Y = A (.) (B C), evaluated only where A has a
 *     stored entry (Section II-A and Section III-B: workers hold row index,
 *     column index and value of each nonzero and produce one output per
 *     nonzero).  The paper's B, C are this library's U and V^T.
 *   - CSR input with 32-bit column indices and 32-bit float values,
 *     Section III-A.
 *   - Backward of SpMM: for L(C) with C = A B, dL/dB = A^T G and
 *     dL/dvals[p] = <G[row(p),:], B[col(p),:]> (chain rule on Eq. (1)).
 *   - bfloat16 rounding: IEEE-754 binary32 -> 8-bit-significand rounding to
 *     nearest, ties to even, by integer manipulation of the bit pattern.
 *   - MLP: three affine layers with ReLU between them, masked mean-squared
 *     error, hand-derived gradients, and the Adam update (Kingma and Ba, ICLR
 *     2015, Algorithm 1).
 *
 * All row_ptr arrays may start at any offset: entries of row i are the
 * positions row_ptr[i] .. row_ptr[i+1]-1 of col_idx / vals, so a caller can
 * pass a slice of rows together with the full index arrays.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ---------------------------------------------------------------------- */
/* SpMM, Eq. (1):  C[i,k] = sum_{p in row i} v_p * B[col_p, k].            */
/* vals == NULL means every stored entry is 1 (the pattern alone).         */
/* bound (optional) receives sum |v_p| * |B[col_p, k]|, the scale of the    */
/* error allowed for a floating-point evaluation of C[i,k].                */
/* ---------------------------------------------------------------------- */
void oracle_spmm(int64_t m, int64_t K, const int32_t *row_ptr, const int32_t *col_idx,
                 const double *vals, const double *B, int64_t ldb, double *C, int64_t ldc,
                 double *bound) {
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t i = 0; i < m; ++i) {
        for (int64_t k = 0; k < K; ++k) {
            double acc = 0.0, mag = 0.0;
            for (int64_t p = row_ptr[i]; p < row_ptr[i + 1]; ++p) {
                double v = vals ? vals[p] : 1.0;
                double b = B[(int64_t)col_idx[p] * ldb + k];
                acc += v * b;
                mag += fabs(v) * fabs(b);
            }
            C[i * ldc + k] = acc;
            if (bound) bound[i * ldc + k] = mag;
        }
    }
}

/* ---------------------------------------------------------------------- */
/* SDDMM, Eq. (2):  S[p] = v_p * sum_k U[row_p, k] * V[col_p, k]           */
/* for every stored entry p; (U V^T) is never formed densely.              */
/* ---------------------------------------------------------------------- */
void oracle_sddmm(int64_t m, int64_t K, const int32_t *row_ptr, const int32_t *col_idx,
                  const double *vals, const double *U, int64_t ldu, const double *V,
                  int64_t ldv, double *S, double *bound) {
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t i = 0; i < m; ++i) {
        for (int64_t p = row_ptr[i]; p < row_ptr[i + 1]; ++p) {
            int64_t j = col_idx[p];
            double dot = 0.0, mag = 0.0;
            for (int64_t k = 0; k < K; ++k) {
                dot += U[i * ldu + k] * V[j * ldv + k];
                mag += fabs(U[i * ldu + k]) * fabs(V[j * ldv + k]);
            }
            double v = vals ? vals[p] : 1.0;
            S[p] = v * dot;
            if (bound) bound[p] = fabs(v) * mag;
        }
    }
}

/* ---------------------------------------------------------------------- */
/* Transpose of a CSR pattern, by a stable counting sort on the column.    */
/* Entries of A are visited in storage order (row-major); entry p with     */
/* column j becomes the next entry of row j of A^T, so rows of A^T list    */
/* their columns (rows of A) in increasing order and perm[q] = p records   */
/* where entry q of A^T came from.  row_ptr of A must start at 0 here.      */
/* ---------------------------------------------------------------------- */
void oracle_csr_transpose(int64_t m, int64_t n, const int32_t *row_ptr,
                          const int32_t *col_idx, int32_t *t_row_ptr, int32_t *t_col_idx,
                          int32_t *perm) {
    int64_t nnz = row_ptr[m];
    int64_t *next = (int64_t *)calloc((size_t)n + 1, sizeof(int64_t));
    for (int64_t p = 0; p < nnz; ++p) next[col_idx[p] + 1] += 1;
    for (int64_t j = 0; j < n; ++j) next[j + 1] += next[j];
    for (int64_t j = 0; j <= n; ++j) t_row_ptr[j] = (int32_t)next[j];
    for (int64_t i = 0; i < m; ++i) {
        for (int64_t p = row_ptr[i]; p < row_ptr[i + 1]; ++p) {
            int64_t q = next[col_idx[p]]++;
            t_col_idx[q] = (int32_t)i;
            perm[q] = (int32_t)p;
        }
    }
    free(next);
}

/* ---------------------------------------------------------------------- */
/* A^T G by its definition: (A^T G)[j,k] = sum over entries p of A with     */
/* column j of v_p * G[row_p, k].  Evaluated as a scatter over A's entries */
/* in storage order (so it does not use the transpose routine above).      */
/* ---------------------------------------------------------------------- */
void oracle_spmm_t(int64_t m, int64_t n, int64_t K, const int32_t *row_ptr,
                   const int32_t *col_idx, const double *vals, const double *G, int64_t ldg,
                   double *D, int64_t ldd, double *bound) {
    for (int64_t j = 0; j < n; ++j)
        for (int64_t k = 0; k < K; ++k) {
            D[j * ldd + k] = 0.0;
            if (bound) bound[j * ldd + k] = 0.0;
        }
#pragma omp parallel for schedule(static)
    for (int64_t k = 0; k < K; ++k) {
        for (int64_t i = 0; i < m; ++i) {
            for (int64_t p = row_ptr[i]; p < row_ptr[i + 1]; ++p) {
                double v = vals ? vals[p] : 1.0;
                double g = G[i * ldg + k];
                D[(int64_t)col_idx[p] * ldd + k] += v * g;
                if (bound) bound[(int64_t)col_idx[p] * ldd + k] += fabs(v) * fabs(g);
            }
        }
    }
}

/* ---------------------------------------------------------------------- */
/* Column-slab form with 16-bit slab-relative column indices (the paper    */
/* sends a column as a 16-bit offset inside the range a worker row holds,  */
/* Section III-A, and groups nonzeros by the worker that owns their column */
/* range in its SELLPACK-like format, Optimization 1).  Columns are cut    */
/* into S = max(1, ceil(n / W)) slabs of W <= 65536 columns.  The entries  */
/* of slab s are stored together (slab-major), row by row; row i's entries */
/* in slab s are the run of A's row whose columns lie in [s W, (s+1) W),   */
/* a contiguous run of A's storage since rows are sorted.                  */
/*   seg[s m + i]   position (slab-major) of the run of (slab s, row i);   */
/*                  seg[S m] = nnz, so the run ends at seg[s m + i + 1]     */
/*   apos[s m + i]  position in A of the run's first entry (where it would  */
/*                  start when empty)                                       */
/*   col16[q]       column minus s W of the run's entries, in order         */
/* Values stay in A's array: entry k of run (s, i) has value               */
/* vals[apos[s m + i] + k].  row_ptr must start at 0 and be canonical.      */
/* Returns S; pass NULL outputs to ask for S alone.                        */
/* ---------------------------------------------------------------------- */
int64_t oracle_csr_to_slab16(int64_t m, int64_t n, int64_t W, const int32_t *row_ptr,
                             const int32_t *col_idx, int32_t *seg, int32_t *apos,
                             uint16_t *col16) {
    int64_t S = n > 0 ? (n + W - 1) / W : 1;
    if (!seg) return S;
    int64_t q = 0;
    for (int64_t s = 0; s < S; ++s) {
        for (int64_t i = 0; i < m; ++i) {
            /* first entry of row i with column >= s W, by a scan of the row */
            int64_t p = row_ptr[i];
            while (p < row_ptr[i + 1] && col_idx[p] < s * W) ++p;
            seg[s * m + i] = (int32_t)q;
            apos[s * m + i] = (int32_t)p;
            while (p < row_ptr[i + 1] && col_idx[p] < (s + 1) * W) {
                col16[q] = (uint16_t)(col_idx[p] - s * W);
                ++q;
                ++p;
            }
        }
    }
    seg[S * m] = (int32_t)q;
    return S;
}

/* ---------------------------------------------------------------------- */
/* Back-to-back products with the intermediate kept (the paper's future     */
/* work on consecutive operations whose result stays resident, Section V):  */
/* attention on A's pattern, written as its three steps.                    */
/*   1. S = A (.) (U V^T) on A's pattern (Eq. 2):                           */
/*        S_p = a_p <U[i,:], V[c_p,:]>         (a_p = 1 when vals == NULL)  */
/*   2. P = softmax of each row's stored scores:                            */
/*        P_p = exp(S_p - mx_i) / sum_q exp(S_q - mx_i), mx_i = max of row i */
/*   3. O = P B (Eq. 1 with P as the values):                               */
/*        O[i,k] = sum_p P_p B[c_p, k]                                      */
/* A row with no stored entry has O[i,:] = 0 and lse_i = -inf.              */
/* Optional outputs:                                                        */
/*   bound[i,k] = sum_p P_p |B[c_p,k]|          (the scale of O's error)     */
/*   escale[i]  = max_p |a_p| sum_k |U[i,k]| |V[c_p,k]|  (the scores' scale) */
/*   lse[i]     = mx_i + log sum_q exp(S_q - mx_i)  (log of the normaliser)  */
/* ---------------------------------------------------------------------- */
void oracle_sddmm_softmax_spmm(int64_t m, int64_t K1, int64_t K2, const int32_t *row_ptr,
                               const int32_t *col_idx, const double *vals, const double *U,
                               int64_t ldu, const double *V, int64_t ldv, const double *B,
                               int64_t ldb, double *O, int64_t ldo, double *bound, double *escale,
                               double *lse) {
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t i = 0; i < m; ++i) {
        int64_t a = row_ptr[i], b = row_ptr[i + 1];
        double *S = (double *)malloc(sizeof(double) * (size_t)(b > a ? b - a : 1));
        double mx = -INFINITY, emax = 0.0;
        for (int64_t p = a; p < b; ++p) { /* step 1 */
            int64_t j = col_idx[p];
            double dot = 0.0, mag = 0.0;
            for (int64_t k = 0; k < K1; ++k) {
                dot += U[i * ldu + k] * V[j * ldv + k];
                mag += fabs(U[i * ldu + k]) * fabs(V[j * ldv + k]);
            }
            double v = vals ? vals[p] : 1.0;
            S[p - a] = v * dot;
            if (fabs(v) * mag > emax) emax = fabs(v) * mag;
            if (S[p - a] > mx) mx = S[p - a];
        }
        double sum = 0.0; /* step 2 */
        for (int64_t p = a; p < b; ++p) sum += exp(S[p - a] - mx);
        for (int64_t p = a; p < b; ++p) S[p - a] = exp(S[p - a] - mx) / sum;
        for (int64_t k = 0; k < K2; ++k) { /* step 3 */
            double acc = 0.0, mag = 0.0;
            for (int64_t p = a; p < b; ++p) {
                double bb = B[(int64_t)col_idx[p] * ldb + k];
                acc += S[p - a] * bb;
                mag += S[p - a] * fabs(bb);
            }
            O[i * ldo + k] = acc;
            if (bound) bound[i * ldo + k] = mag;
        }
        if (escale) escale[i] = emax;
        if (lse) lse[i] = b > a ? mx + log(sum) : -INFINITY;
        free(S);
    }
}

/* ---------------------------------------------------------------------- */
/* Hyper-sparse forms (the paper's weak region above 99% sparsity,         */
/* Sections I and IV-C, and its first future-work item, Section V).        */
/* Row order of the doubly compressed form: the rows holding an entry in   */
/* increasing order, then the empty rows in increasing order; returns the  */
/* number of non-empty rows.  A product then visits only order[0 .. nr).   */
/* ---------------------------------------------------------------------- */
int64_t oracle_nonempty_order(int64_t m, const int32_t *row_ptr, int32_t *order) {
    int64_t nr = 0;
    for (int64_t i = 0; i < m; ++i)
        if (row_ptr[i + 1] > row_ptr[i]) order[nr++] = (int32_t)i;
    int64_t k = nr;
    for (int64_t i = 0; i < m; ++i)
        if (row_ptr[i + 1] == row_ptr[i]) order[k++] = (int32_t)i;
    return nr;
}

/* Coordinate (COO) row index of every stored entry: rowidx[p] = the row    */
/* whose range holds p (the paper's workers keep row, column and value of   */
/* each nonzero, Section III-B).                                            */
void oracle_row_index(int64_t m, const int32_t *row_ptr, int32_t *rowidx) {
    for (int64_t i = 0; i < m; ++i)
        for (int64_t p = row_ptr[i]; p < row_ptr[i + 1]; ++p) rowidx[p] = (int32_t)i;
}

/* ---------------------------------------------------------------------- */
/* Canonical CSR, the input form every product assumes (the paper sends    */
/* CSR with 32-bit column indices, Section III-A, and is silent on order   */
/* and duplicates; the reading taken here is the usual canonical form).    */
/* Returns the OR of the rules A breaks, 0 when it is canonical:           */
/*   1  row_ptr[0] != 0                       (m > 0)                      */
/*   2  row_ptr[m] != nnz                     (for m = 0: nnz != 0)        */
/*   4  some row has row_ptr[i+1] < row_ptr[i], row_ptr[i] < 0 or           */
/*      row_ptr[i+1] > nnz                                                  */
/*   8  a column outside [0, n) in a row that passed rule 4                 */
/*  16  two neighbours of such a row in decreasing column order             */
/*  32  two neighbours of such a row with the same column (a duplicate)     */
/* Rules 8..32 look only at rows whose range lies inside [0, nnz], so no   */
/* rule reads outside the arrays.  row_ptr may be NULL when m = 0.          */
/* ---------------------------------------------------------------------- */
int32_t oracle_csr_canonical(int64_t m, int64_t n, int64_t nnz, const int32_t *row_ptr,
                             const int32_t *col_idx) {
    int32_t bad = 0;
    if (m == 0) return nnz != 0 ? 2 : 0;
    if (row_ptr[0] != 0) bad |= 1;
    if ((int64_t)row_ptr[m] != nnz) bad |= 2;
    for (int64_t i = 0; i < m; ++i) {
        int64_t a = row_ptr[i], b = row_ptr[i + 1];
        if (b < a || a < 0 || b > nnz) {
            bad |= 4;
            continue;
        }
        for (int64_t p = a; p < b; ++p) {
            if (col_idx[p] < 0 || (int64_t)col_idx[p] >= n) bad |= 8;
            if (p + 1 < b) {
                if (col_idx[p + 1] < col_idx[p]) bad |= 16;
                if (col_idx[p + 1] == col_idx[p]) bad |= 32;
            }
        }
    }
    return bad;
}

/* ---------------------------------------------------------------------- */
/* bfloat16 rounding of binary32 values, round to nearest, ties to even.   */
/* The result is returned as a binary32 value whose low 16 bits are zero.  */
/* NaN inputs stay NaN (quiet bit forced); infinities are kept.            */
/* ---------------------------------------------------------------------- */
void oracle_round_bf16(const float *in, float *out, int64_t count) {
    for (int64_t i = 0; i < count; ++i) {
        uint32_t u;
        memcpy(&u, &in[i], 4);
        uint32_t r;
        if ((u & 0x7F800000u) == 0x7F800000u && (u & 0x007FFFFFu) != 0) {
            r = (u | 0x00400000u) & 0xFFFF0000u;
        } else {
            uint32_t lower = u & 0xFFFFu;
            uint32_t upper = u & 0xFFFF0000u;
            uint32_t half = 0x8000u;
            int round_up = lower > half || (lower == half && (upper & 0x10000u));
            r = upper + (round_up ? 0x10000u : 0u);
        }
        memcpy(&out[i], &r, 4);
    }
}

/* ---------------------------------------------------------------------- */
/* Structural features of a CSR pattern (all integer counts):               */
/*   f[0] m, f[1] n, f[2] nnz,                                              */
/*   f[3..22] row-length histogram: bin 0 = empty rows, bin b in 1..18 =    */
/*            lengths in [2^(b-1), 2^b), bin 19 = lengths >= 2^18,          */
/*   f[23] max row length, f[24] sum of squared row lengths,                 */
/*   f[25] max |i - j| over entries, f[26] sum of |i - j| over entries,      */
/*   f[27] number of 4x4 blocks (aligned at multiples of 4) holding at      */
/*         least one entry.                                                  */
/* ---------------------------------------------------------------------- */
#define ORACLE_NFEAT 28
int oracle_feature_count(void) { return ORACLE_NFEAT; }

void oracle_features(int64_t m, int64_t n, const int32_t *row_ptr, const int32_t *col_idx,
                     int64_t *f) {
    for (int i = 0; i < ORACLE_NFEAT; ++i) f[i] = 0;
    f[0] = m;
    f[1] = n;
    f[2] = (int64_t)row_ptr[m] - row_ptr[0];
    for (int64_t i = 0; i < m; ++i) {
        int64_t L = (int64_t)row_ptr[i + 1] - row_ptr[i];
        int bin;
        if (L == 0) {
            bin = 0;
        } else {
            bin = 1;
            while (bin < 19 && L >= ((int64_t)1 << bin)) ++bin;
        }
        f[3 + bin] += 1;
        if (L > f[23]) f[23] = L;
        f[24] += L * L;
        for (int64_t p = row_ptr[i]; p < row_ptr[i + 1]; ++p) {
            int64_t d = i - (int64_t)col_idx[p];
            if (d < 0) d = -d;
            if (d > f[25]) f[25] = d;
            f[26] += d;
        }
    }
    /* Count distinct (i/4, j/4) pairs: mark block columns per block row. */
    int64_t nbc = (n + 3) / 4;
    unsigned char *seen = (unsigned char *)calloc((size_t)(nbc > 0 ? nbc : 1), 1);
    for (int64_t I = 0; I * 4 < m; ++I) {
        int64_t r1 = (I * 4 + 4 < m) ? I * 4 + 4 : m;
        for (int64_t i = I * 4; i < r1; ++i)
            for (int64_t p = row_ptr[i]; p < row_ptr[i + 1]; ++p) {
                int64_t J = col_idx[p] / 4;
                if (!seen[J]) { seen[J] = 1; f[27] += 1; }
            }
        for (int64_t i = I * 4; i < r1; ++i)
            for (int64_t p = row_ptr[i]; p < row_ptr[i + 1]; ++p) seen[col_idx[p] / 4] = 0;
    }
    free(seen);
}

/* ---------------------------------------------------------------------- */
/* Selector inputs: 33 numbers derived from the integer features f, the   */
/* dense width K and the dense dtype, each scaled to roughly [0, 1]:      */
/*   x0 log2(1+m)/20, x1 log2(1+n)/20, x2 log2(1+nnz)/30,                  */
/*   x3..x22 fraction of rows in each row-length bin,                      */
/*   x23 log2(1+max len)/20, x24 log2(1+mean len)/20 (mean = nnz/m),       */
/*   x25 log2(1+cv)/4, cv = sqrt(max(0, E[L^2] - mean^2)) / mean,          */
/*   x26 log2(1+max |i-j|)/20, x27 mean |i-j| / n,                         */
/*   x28 block fill nnz / (16 * blocks), x29 log2(K)/8,                    */
/*   x30 1 + log10(nnz / (m n)) / 5, x31 = 1, x32 = 1 for bfloat16 dense   */
/*   operands and 0 for binary32.                                          */
/* Empty denominators count as 1.                                          */
/* ---------------------------------------------------------------------- */
#define ORACLE_NIN 33
int oracle_input_count(void) { return ORACLE_NIN; }

/* dtype: the dense operands' element type, 0 binary32, 1 bfloat16 (x32). */
void oracle_selector_inputs(const int64_t *f, int64_t K, int32_t dtype, double *x) {
    double m = (double)f[0], n = (double)f[1], nnz = (double)f[2];
    double md = m > 0 ? m : 1.0, nd = n > 0 ? n : 1.0, zd = nnz > 0 ? nnz : 1.0;
    x[0] = log2(1.0 + m) / 20.0;
    x[1] = log2(1.0 + n) / 20.0;
    x[2] = log2(1.0 + nnz) / 30.0;
    for (int b = 0; b < 20; ++b) x[3 + b] = (double)f[3 + b] / md;
    double mean = nnz / md;
    x[23] = log2(1.0 + (double)f[23]) / 20.0;
    x[24] = log2(1.0 + mean) / 20.0;
    double var = (double)f[24] / md - mean * mean;
    double cv = mean > 0 ? sqrt(var > 0 ? var : 0.0) / mean : 0.0;
    x[25] = log2(1.0 + cv) / 4.0;
    x[26] = log2(1.0 + (double)f[25]) / 20.0;
    x[27] = ((double)f[26] / zd) / nd;
    x[28] = nnz / (16.0 * (f[27] > 0 ? (double)f[27] : 1.0));
    x[29] = log2((double)(K > 0 ? K : 1)) / 8.0;
    double dens = nnz / (md * nd);
    x[30] = 1.0 + log10(dens > 1e-12 ? dens : 1e-12) / 5.0;
    x[31] = 1.0;
    x[32] = dtype == 1 ? 1.0 : 0.0;
}

/* ---------------------------------------------------------------------- */
/* CSR -> 4x4 block CSR.  Block (I, J) exists when any entry (i, j) has     */
/* i/4 == I and j/4 == J.  Block values are dense row-major 4x4 tiles with   */
/* zeros where A has no entry; block columns ascend within a block row.     */
/* Count pass: b_col == NULL, returns the number of blocks and fills        */
/* b_row_ptr.  Fill pass: writes b_col and b_vals (16 per block).            */
/* ---------------------------------------------------------------------- */
int64_t oracle_csr_to_bsr4(int64_t m, int64_t n, const int32_t *row_ptr,
                           const int32_t *col_idx, const double *vals, int32_t *b_row_ptr,
                           int32_t *b_col, double *b_vals) {
    int64_t mb = (m + 3) / 4, nbc = (n + 3) / 4;
    int64_t *slot = (int64_t *)malloc(sizeof(int64_t) * (size_t)(nbc > 0 ? nbc : 1));
    for (int64_t J = 0; J < nbc; ++J) slot[J] = -1;
    int64_t total = 0;
    for (int64_t I = 0; I < mb; ++I) {
        int64_t r1 = (I * 4 + 4 < m) ? I * 4 + 4 : m;
        int64_t start = total;
        /* ascending block columns: sweep J over the sorted union */
        int64_t cnt = 0;
        for (int64_t i = I * 4; i < r1; ++i)
            for (int64_t p = row_ptr[i]; p < row_ptr[i + 1]; ++p) {
                int64_t J = col_idx[p] / 4;
                if (slot[J] < 0) { slot[J] = 0; ++cnt; }
            }
        if (b_col) {
            int64_t k = start;
            for (int64_t J = 0; J < nbc; ++J)
                if (slot[J] >= 0) { slot[J] = k; b_col[k] = (int32_t)J; ++k; }
            for (int64_t q = start * 16; q < (start + cnt) * 16; ++q) b_vals[q] = 0.0;
            for (int64_t i = I * 4; i < r1; ++i)
                for (int64_t p = row_ptr[i]; p < row_ptr[i + 1]; ++p) {
                    int64_t J = col_idx[p] / 4;
                    b_vals[slot[J] * 16 + (i - I * 4) * 4 + (col_idx[p] - J * 4)] +=
                        vals ? vals[p] : 1.0;
                }
        } else {
            b_row_ptr[I] = (int32_t)start;
        }
        for (int64_t i = I * 4; i < r1; ++i)
            for (int64_t p = row_ptr[i]; p < row_ptr[i + 1]; ++p) slot[col_idx[p] / 4] = -1;
        total += cnt;
    }
    if (!b_col) b_row_ptr[mb] = (int32_t)total;
    free(slot);
    return total;
}

/* ---------------------------------------------------------------------- */
/* Three-layer perceptron  y = W3 relu(W2 relu(W1 x + b1) + b2) + b3.       */
/* Weights are row-major [out][in].  X is [batch][F], Y is [batch][P].      */
/* ---------------------------------------------------------------------- */
typedef struct {
    int64_t F, H, P;
    const double *W1, *b1, *W2, *b2, *W3, *b3;
} oracle_mlp;

static void affine(int64_t nout, int64_t nin, const double *W, const double *b,
                   const double *x, double *y) {
    for (int64_t o = 0; o < nout; ++o) {
        double acc = b[o];
        for (int64_t i = 0; i < nin; ++i) acc += W[o * nin + i] * x[i];
        y[o] = acc;
    }
}

void oracle_mlp_forward(int64_t F, int64_t H, int64_t P, const double *W1, const double *b1,
                        const double *W2, const double *b2, const double *W3,
                        const double *b3, int64_t batch, const double *X, double *Y) {
    double *h1 = (double *)malloc(sizeof(double) * (size_t)H);
    double *h2 = (double *)malloc(sizeof(double) * (size_t)H);
    for (int64_t s = 0; s < batch; ++s) {
        affine(H, F, W1, b1, X + s * F, h1);
        for (int64_t o = 0; o < H; ++o) h1[o] = h1[o] > 0.0 ? h1[o] : 0.0;
        affine(H, H, W2, b2, h1, h2);
        for (int64_t o = 0; o < H; ++o) h2[o] = h2[o] > 0.0 ? h2[o] : 0.0;
        affine(P, H, W3, b3, h2, Y + s * P);
    }
    free(h1);
    free(h2);
}

/* Masked mean-squared error  L = (1 / (2 * count)) * sum mask * (y - t)^2, */
/* count = number of nonzero mask entries, and its gradient with respect    */
/* to every weight and bias (accumulated over the batch).  Returns L.       */
/* The mask's values weigh the terms (0 drops a term; a 0/1 mask is the     */
/* plain masked mean).                                                      */
double oracle_mlp_loss_grad(int64_t F, int64_t H, int64_t P, const double *W1,
                            const double *b1, const double *W2, const double *b2,
                            const double *W3, const double *b3, int64_t batch,
                            const double *X, const double *T, const double *mask,
                            double *gW1, double *gb1, double *gW2, double *gb2,
                            double *gW3, double *gb3) {
    memset(gW1, 0, sizeof(double) * (size_t)(H * F));
    memset(gb1, 0, sizeof(double) * (size_t)H);
    memset(gW2, 0, sizeof(double) * (size_t)(H * H));
    memset(gb2, 0, sizeof(double) * (size_t)H);
    memset(gW3, 0, sizeof(double) * (size_t)(P * H));
    memset(gb3, 0, sizeof(double) * (size_t)P);
    double count = 0.0;
    for (int64_t q = 0; q < batch * P; ++q) count += mask[q] != 0.0 ? 1.0 : 0.0;
    if (count == 0.0) return 0.0;
    double *z1 = (double *)malloc(sizeof(double) * (size_t)H);
    double *a1 = (double *)malloc(sizeof(double) * (size_t)H);
    double *z2 = (double *)malloc(sizeof(double) * (size_t)H);
    double *a2 = (double *)malloc(sizeof(double) * (size_t)H);
    double *y = (double *)malloc(sizeof(double) * (size_t)P);
    double *dy = (double *)malloc(sizeof(double) * (size_t)P);
    double *d2 = (double *)malloc(sizeof(double) * (size_t)H);
    double *d1 = (double *)malloc(sizeof(double) * (size_t)H);
    double loss = 0.0;
    for (int64_t s = 0; s < batch; ++s) {
        const double *x = X + s * F;
        affine(H, F, W1, b1, x, z1);
        for (int64_t o = 0; o < H; ++o) a1[o] = z1[o] > 0.0 ? z1[o] : 0.0;
        affine(H, H, W2, b2, a1, z2);
        for (int64_t o = 0; o < H; ++o) a2[o] = z2[o] > 0.0 ? z2[o] : 0.0;
        affine(P, H, W3, b3, a2, y);
        for (int64_t o = 0; o < P; ++o) {
            double w = mask[s * P + o];
            double e = y[o] - T[s * P + o];
            loss += w * e * e;
            dy[o] = w * e / count; /* dL/dy */
        }
        /* layer 3 */
        for (int64_t o = 0; o < P; ++o) {
            gb3[o] += dy[o];
            for (int64_t i = 0; i < H; ++i) gW3[o * H + i] += dy[o] * a2[i];
        }
        for (int64_t i = 0; i < H; ++i) {
            double acc = 0.0;
            for (int64_t o = 0; o < P; ++o) acc += W3[o * H + i] * dy[o];
            d2[i] = z2[i] > 0.0 ? acc : 0.0;
        }
        /* layer 2 */
        for (int64_t o = 0; o < H; ++o) {
            gb2[o] += d2[o];
            for (int64_t i = 0; i < H; ++i) gW2[o * H + i] += d2[o] * a1[i];
        }
        for (int64_t i = 0; i < H; ++i) {
            double acc = 0.0;
            for (int64_t o = 0; o < H; ++o) acc += W2[o * H + i] * d2[o];
            d1[i] = z1[i] > 0.0 ? acc : 0.0;
        }
        /* layer 1 */
        for (int64_t o = 0; o < H; ++o) {
            gb1[o] += d1[o];
            for (int64_t i = 0; i < F; ++i) gW1[o * F + i] += d1[o] * x[i];
        }
    }
    free(z1); free(a1); free(z2); free(a2); free(y); free(dy); free(d2); free(d1);
    return loss / (2.0 * count);
}

/* Adam (Kingma and Ba, Algorithm 1), step number t >= 1, in place. */
void oracle_adam(int64_t count, double *w, const double *g, double *mom, double *vel,
                 double lr, double beta1, double beta2, double eps, int64_t t) {
    double c1 = 1.0 - pow(beta1, (double)t);
    double c2 = 1.0 - pow(beta2, (double)t);
    for (int64_t i = 0; i < count; ++i) {
        mom[i] = beta1 * mom[i] + (1.0 - beta1) * g[i];
        vel[i] = beta2 * vel[i] + (1.0 - beta2) * g[i] * g[i];
        double mh = mom[i] / c1;
        double vh = vel[i] / c2;
        w[i] -= lr * mh / (sqrt(vh) + eps);
    }
}
