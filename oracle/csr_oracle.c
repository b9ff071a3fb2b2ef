/*
 * csr_oracle.c - plain, slow, obviously correct CSR kernels for the CPU
 * oracle.  TEST INFRASTRUCTURE ONLY: the GPU library never links or calls
 * this file; only the tests, the smoke check and the CPU baseline leg of
 * the benchmark do.  Everything is fp64 and follows the definitions below
 * with no blocking, fusion or reordering.
 *
 * The symmetric matrix H is given by its stored upper triangle U_s (diagonal
 * included), the storage of one triangle described in Section 4.1 of the
 * paper (the paper stores the lower one; the transpose is the same data).
 * H_ij = H_ji = U_s(min(i,j), max(i,j)).
 */
#include <stdint.h>
#include <stdlib.h>
#include <math.h>

/*
 * Y = H X with H held as one stored triangle: for every stored (i, j, a),
 * Y_i += a X_j and, when i != j, Y_j += a X_i.  Sequential, in storage
 * order.  X, Y are n x m row-major.
 */
void oracle_spmm_half(int64_t n, const int64_t *rowptr, const int32_t *colind,
                      const double *vals, int64_t m, const double *X, double *Y) {
    for (int64_t t = 0; t < n * m; t++) Y[t] = 0.0;
    for (int64_t i = 0; i < n; i++) {
        for (int64_t p = rowptr[i]; p < rowptr[i + 1]; p++) {
            int64_t j = colind[p];
            double a = vals[p];
            for (int64_t k = 0; k < m; k++) Y[i * m + k] += a * X[j * m + k];
            if (j != i)
                for (int64_t k = 0; k < m; k++) Y[j * m + k] += a * X[i * m + k];
        }
    }
}

/* number of entries of the full (mirrored) matrix, per row */
void oracle_full_counts(int64_t n, const int64_t *rowptr, const int32_t *colind,
                        int64_t *counts) {
    for (int64_t i = 0; i < n; i++) counts[i] = 0;
    for (int64_t i = 0; i < n; i++)
        for (int64_t p = rowptr[i]; p < rowptr[i + 1]; p++) {
            counts[i]++;
            if (colind[p] != i) counts[colind[p]]++;
        }
}

/*
 * Mirror the stored triangle into full CSR.  frowptr must be the prefix sum
 * of oracle_full_counts.  Rows come out column-sorted because row i first
 * receives the mirrored entries of rows r < i (in increasing r) and then its
 * own stored entries (columns >= i, increasing).
 */
void oracle_full_fill(int64_t n, const int64_t *rowptr, const int32_t *colind,
                      const double *vals, const int64_t *frowptr, int32_t *fcol,
                      double *fval) {
    int64_t *cur = (int64_t *)malloc(sizeof(int64_t) * (n > 0 ? n : 1));
    for (int64_t i = 0; i < n; i++) cur[i] = frowptr[i];
    for (int64_t i = 0; i < n; i++) {
        for (int64_t p = rowptr[i]; p < rowptr[i + 1]; p++) {
            int64_t j = colind[p];
            int64_t q = cur[i]++;
            fcol[q] = (int32_t)j; fval[q] = vals[p];
            if (j != i) {
                int64_t q2 = cur[j]++;
                fcol[q2] = (int32_t)i; fval[q2] = vals[p];
            }
        }
    }
    free(cur);
}

/* Y = A X for a full CSR matrix A; rows are independent (OpenMP over rows). */
void oracle_spmm_full(int64_t n, const int64_t *frowptr, const int32_t *fcol,
                      const double *fval, int64_t m, const double *X, double *Y) {
    #pragma omp parallel for schedule(dynamic, 1024)
    for (int64_t i = 0; i < n; i++) {
        for (int64_t k = 0; k < m; k++) {
            double s = 0.0;
            for (int64_t p = frowptr[i]; p < frowptr[i + 1]; p++)
                s += fval[p] * X[(int64_t)fcol[p] * m + k];
            Y[i * m + k] = s;
        }
    }
}

/* ||H||_1 = max over rows of the absolute row sum of the full matrix */
double oracle_norm1(int64_t n, const int64_t *rowptr, const int32_t *colind,
                    const double *vals) {
    double *s = (double *)calloc((size_t)(n > 0 ? n : 1), sizeof(double));
    for (int64_t i = 0; i < n; i++)
        for (int64_t p = rowptr[i]; p < rowptr[i + 1]; p++) {
            s[i] += fabs(vals[p]);
            if (colind[p] != i) s[colind[p]] += fabs(vals[p]);
        }
    double mx = 0.0;
    for (int64_t i = 0; i < n; i++) if (s[i] > mx) mx = s[i];
    free(s);
    return mx;
}

/* diagonal of H (0 where no diagonal entry is stored) */
void oracle_diagonal(int64_t n, const int64_t *rowptr, const int32_t *colind,
                     const double *vals, double *d) {
    for (int64_t i = 0; i < n; i++) {
        d[i] = 0.0;
        for (int64_t p = rowptr[i]; p < rowptr[i + 1]; p++)
            if (colind[p] == i) d[i] += vals[p];
    }
}

/*
 * Dense diagonal blocks of H over consecutive chunks of bs rows (the last
 * chunk may be shorter): out[b] is a bs x bs row-major block, zero padded.
 */
void oracle_diag_blocks(int64_t n, const int64_t *rowptr, const int32_t *colind,
                        const double *vals, int64_t bs, double *out) {
    int64_t nb = (n + bs - 1) / bs;
    for (int64_t t = 0; t < nb * bs * bs; t++) out[t] = 0.0;
    for (int64_t i = 0; i < n; i++) {
        int64_t b = i / bs;
        for (int64_t p = rowptr[i]; p < rowptr[i + 1]; p++) {
            int64_t j = colind[p];
            if (j / bs != b) continue;
            int64_t li = i - b * bs, lj = j - b * bs;
            out[b * bs * bs + li * bs + lj] = vals[p];
            out[b * bs * bs + lj * bs + li] = vals[p];
        }
    }
}
