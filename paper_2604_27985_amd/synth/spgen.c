/*
 * spgen.c - seeded synthetic inputs for the SpMM / SDDMM library.
 *
 * This module only draws random numbers and lays them out as CSR patterns and
 * dense arrays.  It holds none of the arithmetic of the sparse products: both
 * the GPU library and the CPU oracle consume the arrays it writes, so neither
 * depends on the other.
 *
 * Random numbers come from a counter-based generator: the SplitMix64 output
 * function (Steele, Lea and Flood, "Fast splittable pseudorandom number
 * generators", OOPSLA 2014) applied to a key built from (seed, stream, item)
 * plus a per-item counter.  Every row or element owns its own counter space,
 * so results do not depend on the OpenMP thread count.
 *
 * Pattern families (all canonical CSR: columns strictly increasing per row):
 *   - Bernoulli: each (i, j) present independently with probability p; rows
 *     are drawn by geometric skipping (gap = floor(log(u) / log(1 - p))), which
 *     samples the same distribution in O(nnz).  An optional band |i - j| <= bw
 *     restricts the candidate columns.
 *   - Fixed degree: row i gets exactly deg[i] distinct columns drawn uniformly
 *     (Floyd's sampling algorithm, CACM 30(9), 1987), used for power-law rows.
 *   - 4x4 blocks: a Bernoulli draw over the grid of 4x4 blocks; a chosen block
 *     is fully dense (ragged at the right and bottom edges).
 *
 * Build: gcc -O2 -fopenmp -shared -fPIC spgen.c -o libspgen.so -lm
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define SPGEN_GOLDEN 0x9E3779B97F4A7C15ULL

static inline uint64_t mix64(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

/* Key of one item (a row, a block row or a dense element pair). */
static inline uint64_t item_key(uint64_t seed, uint64_t stream, uint64_t item) {
    uint64_t k = mix64(seed + SPGEN_GOLDEN);
    k = mix64(k ^ (stream * 0xD1B54A32D192ED03ULL + SPGEN_GOLDEN));
    return mix64(k ^ (item + 1) * SPGEN_GOLDEN);
}

/* The ctr-th 64-bit draw of an item. */
static inline uint64_t draw(uint64_t key, uint64_t ctr) {
    return mix64(key + (ctr + 1) * SPGEN_GOLDEN);
}

/* Uniform double in (0, 1): 53 random bits, offset by half a step. */
static inline double unit_open(uint64_t x) {
    return ((double)(x >> 11) + 0.5) * (1.0 / 9007199254740992.0);
}

uint64_t spgen_u64(uint64_t seed, uint64_t stream, uint64_t item, uint64_t ctr) {
    return draw(item_key(seed, stream, item), ctr);
}

/* ------------------------------------------------------------------------ */
/* Bernoulli rows: one geometric-skip walk per row over [lo, hi].            */
/* Count pass (row_ptr == NULL): writes row_len[i].                          */
/* Fill pass: writes col_idx[row_ptr[i] ...].                                */
/* ------------------------------------------------------------------------ */
static inline int64_t walk_row(uint64_t key, int64_t lo, int64_t hi, double p,
                               double inv_log_q, int32_t *out) {
    int64_t cnt = 0;
    if (hi < lo || p <= 0.0) return 0;
    if (p >= 1.0) {
        for (int64_t j = lo; j <= hi; ++j) {
            if (out) out[cnt] = (int32_t)j;
            ++cnt;
        }
        return cnt;
    }
    int64_t pos = lo - 1;
    for (uint64_t ctr = 0;; ++ctr) {
        double u = unit_open(draw(key, ctr));
        double g = floor(log(u) * inv_log_q);
        if (g > (double)(hi - pos)) break;
        pos += (int64_t)g + 1;
        if (pos > hi) break;
        if (out) out[cnt] = (int32_t)pos;
        ++cnt;
    }
    return cnt;
}

int spgen_bernoulli(int64_t m, int64_t n, double p, int64_t band, uint64_t seed,
                    uint64_t stream, int64_t *row_len, const int64_t *row_ptr,
                    int32_t *col_idx) {
    if (m < 0 || n < 0 || n > 2147483647LL) return -1;
    double inv_log_q = (p > 0.0 && p < 1.0) ? 1.0 / log1p(-p) : 0.0;
#pragma omp parallel for schedule(dynamic, 256)
    for (int64_t i = 0; i < m; ++i) {
        int64_t lo = 0, hi = n - 1;
        if (band >= 0) {
            lo = i - band < 0 ? 0 : i - band;
            hi = i + band > n - 1 ? n - 1 : i + band;
        }
        uint64_t key = item_key(seed, stream, (uint64_t)i);
        if (row_ptr == NULL)
            row_len[i] = walk_row(key, lo, hi, p, inv_log_q, NULL);
        else
            walk_row(key, lo, hi, p, inv_log_q, col_idx + row_ptr[i]);
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* 4x4 block rows: block row I = i / 4 draws its block columns once; all     */
/* rows of the block row expand the same blocks to 4 columns each.           */
/* ------------------------------------------------------------------------ */
int spgen_block4(int64_t m, int64_t n, double p, uint64_t seed, uint64_t stream,
                 int64_t *row_len, const int64_t *row_ptr, int32_t *col_idx) {
    if (m < 0 || n < 0 || n > 2147483647LL) return -1;
    int64_t nb = (n + 3) / 4;
    double inv_log_q = (p > 0.0 && p < 1.0) ? 1.0 / log1p(-p) : 0.0;
#pragma omp parallel
    {
        int32_t *blk = (int32_t *)malloc(sizeof(int32_t) * (size_t)(nb > 0 ? nb : 1));
#pragma omp for schedule(dynamic, 64)
        for (int64_t i = 0; i < m; ++i) {
            uint64_t key = item_key(seed, stream, (uint64_t)(i / 4));
            int64_t nblk = walk_row(key, 0, nb - 1, p, inv_log_q, blk);
            int64_t cnt = 0;
            for (int64_t b = 0; b < nblk; ++b) {
                int64_t c0 = (int64_t)blk[b] * 4;
                for (int64_t c = c0; c < c0 + 4 && c < n; ++c) {
                    if (row_ptr) col_idx[row_ptr[i] + cnt] = (int32_t)c;
                    ++cnt;
                }
            }
            if (!row_ptr) row_len[i] = cnt;
        }
        free(blk);
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Power-law degrees: d_i = min(n, max(1, floor(x_min * (1-u_i)^(-1/(a-1))))) */
/* with x_min bisected so that the realised mean degree is within `tol`      */
/* (relative) of `mean`.  Writes deg[m]; returns the x_min used via *xmin.   */
/* ------------------------------------------------------------------------ */
static int64_t degree_of(double xmin, double e, double tail, int64_t n) {
    double d = floor(xmin * tail);
    (void)e;
    if (!(d >= 1.0)) return 1;
    if (d >= (double)n) return n;
    return (int64_t)d;
}

int spgen_powerlaw_degrees(int64_t m, int64_t n, double alpha, double mean,
                           double tol, uint64_t seed, uint64_t stream,
                           int32_t *deg, double *xmin_out) {
    if (m <= 0 || n <= 0 || alpha <= 1.0 || mean <= 0.0) return -1;
    double e = -1.0 / (alpha - 1.0);
    double *tail = (double *)malloc(sizeof(double) * (size_t)m);
    if (!tail) return -2;
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < m; ++i) {
        double u = unit_open(draw(item_key(seed, stream, (uint64_t)i), 0));
        tail[i] = pow(u, e); /* 1-u has the same law as u */
    }
    double lo = 1e-3, hi = (double)n;
    double xmin = 1.0;
    for (int it = 0; it < 200; ++it) {
        xmin = 0.5 * (lo + hi);
        int64_t total = 0;
#pragma omp parallel for reduction(+ : total) schedule(static)
        for (int64_t i = 0; i < m; ++i) total += degree_of(xmin, e, tail[i], n);
        double got = (double)total / (double)m;
        if (fabs(got - mean) <= tol * mean) break;
        if (got < mean) lo = xmin; else hi = xmin;
    }
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < m; ++i) deg[i] = (int32_t)degree_of(xmin, e, tail[i], n);
    free(tail);
    if (xmin_out) *xmin_out = xmin;
    return 0;
}

/* ------------------------------------------------------------------------ */
/* Fixed-degree rows: row i receives row_ptr[i+1]-row_ptr[i] distinct       */
/* columns drawn uniformly from [0, n), written sorted.                      */
/* ------------------------------------------------------------------------ */
static int cmp_i32(const void *a, const void *b) {
    int32_t x = *(const int32_t *)a, y = *(const int32_t *)b;
    return (x > y) - (x < y);
}

/* Floyd: for j = n-L .. n-1, draw t in [0, j]; take t unless already taken,
 * then take j.  Membership through an open-addressing hash set. */
static void floyd(uint64_t key, int64_t n, int64_t L, int32_t *out, int32_t *set,
                  int64_t cap) {
    for (int64_t s = 0; s < cap; ++s) set[s] = -1;
    int64_t mask = cap - 1, cnt = 0;
    uint64_t ctr = 0;
    for (int64_t j = n - L; j < n; ++j) {
        uint64_t r = draw(key, ctr++);
        int64_t t = (int64_t)(r % (uint64_t)(j + 1));
        int64_t pick = t;
        for (int pass = 0; pass < 2; ++pass) {
            int64_t h = (int64_t)(mix64((uint64_t)pick) & (uint64_t)mask);
            int found = 0;
            while (set[h] >= 0) {
                if (set[h] == pick) { found = 1; break; }
                h = (h + 1) & mask;
            }
            if (!found) {
                set[h] = (int32_t)pick;
                out[cnt++] = (int32_t)pick;
                break;
            }
            pick = j; /* t was taken: j cannot be, by construction */
        }
    }
    qsort(out, (size_t)cnt, sizeof(int32_t), cmp_i32);
}

int spgen_distinct_cols(int64_t m, int64_t n, const int64_t *row_ptr, uint64_t seed,
                        uint64_t stream, int32_t *col_idx) {
    if (m < 0 || n < 0 || n > 2147483647LL) return -1;
    int bad = 0;
#pragma omp parallel for schedule(dynamic, 16) reduction(| : bad)
    for (int64_t i = 0; i < m; ++i) {
        int64_t L = row_ptr[i + 1] - row_ptr[i];
        int32_t *out = col_idx + row_ptr[i];
        uint64_t key = item_key(seed, stream, (uint64_t)i);
        if (L <= 0) continue;
        if (L > n) { bad = 1; continue; }
        if (L == n) {
            for (int64_t j = 0; j < n; ++j) out[j] = (int32_t)j;
            continue;
        }
        int complement = L > n / 2;
        int64_t draw_n = complement ? n - L : L;
        int64_t cap = 16;
        while (cap < 2 * draw_n) cap <<= 1;
        int32_t *set = (int32_t *)malloc(sizeof(int32_t) * (size_t)cap);
        int32_t *tmp = complement ? (int32_t *)malloc(sizeof(int32_t) * (size_t)(draw_n + 1)) : out;
        floyd(key, n, draw_n, tmp, set, cap);
        if (complement) {
            int64_t k = 0, c = 0;
            for (int64_t j = 0; j < n; ++j) {
                if (k < draw_n && tmp[k] == j) { ++k; continue; }
                out[c++] = (int32_t)j;
            }
            free(tmp);
        }
        free(set);
    }
    return bad ? -1 : 0;
}

/* ------------------------------------------------------------------------ */
/* Dense values.                                                             */
/* ------------------------------------------------------------------------ */
/* Standard normal by the Box-Muller transform on pairs of draws. */
int spgen_normal_f32(uint64_t seed, uint64_t stream, int64_t count, float *out) {
    const double two_pi = 6.283185307179586476925286766559;
#pragma omp parallel for schedule(static)
    for (int64_t pair = 0; pair < (count + 1) / 2; ++pair) {
        uint64_t key = item_key(seed, stream, (uint64_t)pair);
        double u1 = unit_open(draw(key, 0));
        double u2 = unit_open(draw(key, 1));
        double r = sqrt(-2.0 * log(u1));
        int64_t i = 2 * pair;
        out[i] = (float)(r * cos(two_pi * u2));
        if (i + 1 < count) out[i + 1] = (float)(r * sin(two_pi * u2));
    }
    return 0;
}

/* Uniform on [lo, hi). */
int spgen_uniform_f32(uint64_t seed, uint64_t stream, int64_t count, double lo,
                      double hi, float *out) {
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < count; ++i) {
        uint64_t key = item_key(seed, stream, (uint64_t)i);
        double u = (double)(draw(key, 0) >> 11) * (1.0 / 9007199254740992.0);
        float v = (float)(lo + (hi - lo) * u);
        if (v >= (float)hi) v = nextafterf((float)hi, (float)lo);
        out[i] = v;
    }
    return 0;
}

/* Uniform integers in [0, n): used to pick sample rows and coordinates. */
int spgen_randint(uint64_t seed, uint64_t stream, int64_t count, int64_t n, int64_t *out) {
    if (n <= 0) return -1;
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < count; ++i)
        out[i] = (int64_t)(draw(item_key(seed, stream, (uint64_t)i), 0) % (uint64_t)n);
    return 0;
}
