/*
 * hsymgen.c - seeded synthetic generator of sparse symmetric matrices shaped
 * like configuration-interaction Hamiltonians, emitted as upper-triangle CSR.
 *
 * This module holds no arithmetic of the eigensolver.  It only draws inputs:
 * the matrix H (diagonal plus strictly-upper entries), Gaussian start blocks
 * and start vectors.  Both the CPU oracle and the GPU library consume the
 * arrays it writes.
 *
 * Structure (after the tile picture of Section 2.2, Fig. 2 of the paper:
 * states are grouped, nonzero matrix elements only appear in tiles between
 * groups whose labels are close, and the diagonal tiles are the densest):
 *   - blocks ("groups") of size s ~ U{16..64} are drawn until n is covered;
 *     the last block is truncated.  Each block gets a level label q ~ U{0..4}.
 *   - H_ii = 10*q(i) + U(0,1).
 *   - inside a diagonal tile every strictly-upper position is present with
 *     probability 1/2; values N(0, 0.3^2).
 *   - an off-diagonal tile (I,J), I<J<=I+Wb, |q_I-q_J|<=2, is present with
 *     probability p_t; each of its positions with probability rho; values
 *     N(0, 0.3^2).  p_t is solved so that the expected number of nonzeros in
 *     a full row (diagonal included) equals N on the realised blocks.
 *
 * Random numbers: every draw is a pure function of (seed, purpose, a, b).
 * The mixing function is the SplitMix64 output function applied to a Weyl
 * sequence (Steele, Lea and Flood, "Fast splittable pseudorandom number
 * generators", OOPSLA 2014).  Draws never depend on thread count or on the
 * slab of rows that is generated, so any row range can be produced alone.
 * Uniforms use the top 53 bits; normals use the Box-Muller cosine branch.
 */
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <math.h>

#define GAMMA 0x9E3779B97F4A7C15ULL

enum {
    P_SIZE = 1, P_LABEL = 2, P_DIAGV = 3, P_DTILE = 4, P_TILE = 5,
    P_ENTRY = 6, P_VAL = 7, P_X0 = 8, P_V0 = 9
};

static inline uint64_t mix64(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

static inline uint64_t stream_key(uint64_t seed, uint64_t purpose) {
    return mix64(mix64(seed + GAMMA) ^ (purpose * GAMMA));
}

/* SplitMix64 output for counter (a,b) of the stream with key k */
static inline uint64_t draw(uint64_t k, uint64_t a, uint64_t b) {
    uint64_t ctr = (a << 32) | (b & 0xffffffffULL);
    return mix64(k + (ctr + 1ULL) * GAMMA);
}

static inline double uniform01(uint64_t k, uint64_t a, uint64_t b) {
    return (double)(draw(k, a, b) >> 11) * (1.0 / 9007199254740992.0);
}

static inline double normal01(uint64_t k, uint64_t a, uint64_t b) {
    double u1 = uniform01(k, a, 2 * b);
    double u2 = uniform01(k, a, 2 * b + 1);
    return sqrt(-2.0 * log(1.0 - u1)) * cos(6.283185307179586476925286766559 * u2);
}

/* ---------------------------------------------------------------------- */
/* block structure                                                          */
/* ---------------------------------------------------------------------- */

typedef struct {
    int64_t n;
    uint64_t seed;
    int64_t nblocks;
    int64_t *start;      /* nblocks+1 */
    int32_t *label;      /* nblocks */
    int64_t window;      /* Wb in blocks; <=0 means unlimited */
    double p_tile;       /* realised tile probability */
    double rho;          /* entry probability in an off-diagonal tile */
    double rho_diag;     /* entry probability in a diagonal tile */
    double sigma;        /* std dev of off-diagonal values */
    int variant;         /* 0 banded, 1 uniform window, 2 block-diagonal only */
    /* present off-diagonal tiles per block row, CSR over blocks */
    int64_t *tptr;       /* nblocks+1 */
    int32_t *tcol;       /* present J for each I, ascending */
} hsg_struct;

static int allowed(const hsg_struct *s, int64_t I, int64_t J) {
    if (J <= I) return 0;
    if (s->window > 0 && J > I + s->window) return 0;
    int d = s->label[I] - s->label[J];
    return (d >= -2 && d <= 2);
}

/*
 * Build the block structure.  target_nnz_row is the expected full-row count
 * including the diagonal.  Returns NULL on allocation failure.
 */
void *hsg_create(int64_t n, double target_nnz_row, uint64_t seed, int64_t window,
                 double rho, double rho_diag, double sigma, int variant) {
    if (n <= 0) return NULL;
    hsg_struct *s = (hsg_struct *)calloc(1, sizeof(hsg_struct));
    if (!s) return NULL;
    s->n = n; s->seed = seed; s->window = (variant == 1) ? 0 : window;
    s->rho = rho; s->rho_diag = rho_diag; s->sigma = sigma; s->variant = variant;
    uint64_t ksz = stream_key(seed, P_SIZE), klb = stream_key(seed, P_LABEL);
    int64_t cap = n / 16 + 2;
    s->start = (int64_t *)malloc(sizeof(int64_t) * (cap + 1));
    s->label = (int32_t *)malloc(sizeof(int32_t) * cap);
    if (!s->start || !s->label) { free(s->start); free(s->label); free(s); return NULL; }
    int64_t pos = 0, nb = 0;
    while (pos < n) {
        int64_t sz = 16 + (int64_t)(uniform01(ksz, 0, (uint64_t)nb) * 49.0);
        if (sz > 64) sz = 64;
        s->start[nb] = pos;
        s->label[nb] = (int32_t)(uniform01(klb, 0, (uint64_t)nb) * 5.0);
        if (s->label[nb] > 4) s->label[nb] = 4;
        pos += sz; if (pos > n) pos = n;
        nb++;
    }
    s->start[nb] = n;
    s->nblocks = nb;

    /* calibrate p_t so that the expected full nnz equals n*N */
    double diag_part = 0.0, off_area = 0.0;
    for (int64_t I = 0; I < nb; I++) {
        double sI = (double)(s->start[I + 1] - s->start[I]);
        diag_part += sI + rho_diag * sI * (sI - 1.0);   /* both halves of the tile */
    }
    if (variant != 2) {
        for (int64_t I = 0; I < nb; I++) {
            double sI = (double)(s->start[I + 1] - s->start[I]);
            int64_t Jmax = (s->window > 0) ? I + s->window : nb - 1;
            if (Jmax > nb - 1) Jmax = nb - 1;
            for (int64_t J = I + 1; J <= Jmax; J++)
                if (allowed(s, I, J))
                    off_area += sI * (double)(s->start[J + 1] - s->start[J]);
        }
    }
    double need = (double)n * target_nnz_row - diag_part;
    double pt = 0.0;
    if (variant != 2 && off_area > 0.0 && need > 0.0) pt = need / (2.0 * rho * off_area);
    if (pt > 1.0) { s->rho = rho * pt; if (s->rho > 1.0) s->rho = 1.0; pt = 1.0; }
    s->p_tile = pt;

    /* present tiles */
    uint64_t kt = stream_key(seed, P_TILE);
    s->tptr = (int64_t *)malloc(sizeof(int64_t) * (nb + 1));
    int64_t cnt = 0;
    for (int pass = 0; pass < 2; pass++) {
        cnt = 0;
        for (int64_t I = 0; I < nb; I++) {
            if (pass == 0) s->tptr[I] = cnt;
            if (variant == 2 || pt <= 0.0) continue;
            int64_t Jmax = (s->window > 0) ? I + s->window : nb - 1;
            if (Jmax > nb - 1) Jmax = nb - 1;
            for (int64_t J = I + 1; J <= Jmax; J++) {
                if (!allowed(s, I, J)) continue;
                if (uniform01(kt, (uint64_t)I, (uint64_t)J) < pt) {
                    if (pass == 1) s->tcol[cnt] = (int32_t)J;
                    cnt++;
                }
            }
        }
        if (pass == 0) {
            s->tptr[nb] = cnt;
            s->tcol = (int32_t *)malloc(sizeof(int32_t) * (cnt > 0 ? cnt : 1));
        }
    }
    return s;
}

void hsg_destroy(void *h) {
    hsg_struct *s = (hsg_struct *)h;
    if (!s) return;
    free(s->start); free(s->label); free(s->tptr); free(s->tcol); free(s);
}

int64_t hsg_nblocks(void *h) { return ((hsg_struct *)h)->nblocks; }
double hsg_ptile(void *h) { return ((hsg_struct *)h)->p_tile; }
double hsg_rho(void *h) { return ((hsg_struct *)h)->rho; }
int64_t hsg_ntiles(void *h) { hsg_struct *s = (hsg_struct *)h; return s->tptr[s->nblocks]; }

/* copy out block starts (nblocks+1) and labels (nblocks) */
void hsg_blocks(void *h, int64_t *start, int32_t *label) {
    hsg_struct *s = (hsg_struct *)h;
    memcpy(start, s->start, sizeof(int64_t) * (s->nblocks + 1));
    memcpy(label, s->label, sizeof(int32_t) * s->nblocks);
}

static int64_t block_of(const hsg_struct *s, int64_t i) {
    int64_t lo = 0, hi = s->nblocks - 1;
    while (lo < hi) {
        int64_t mid = (lo + hi + 1) / 2;
        if (s->start[mid] <= i) lo = mid; else hi = mid - 1;
    }
    return lo;
}

/*
 * Row i of the stored upper triangle: diagonal, diagonal-tile entries, then
 * present off-diagonal tiles in ascending J.  When cols != NULL the entries
 * are written; the count is returned either way.
 */
static int64_t gen_row(const hsg_struct *s, int64_t i, int64_t I, uint64_t kdv, uint64_t kdt,
                       uint64_t ken, uint64_t kval, int32_t *cols, double *vd, float *vf) {
    int64_t c = 0;
    if (cols) {
        double d = 10.0 * (double)s->label[I] + uniform01(kdv, 0, (uint64_t)i);
        cols[0] = (int32_t)i;
        if (vd) vd[0] = d;
        if (vf) vf[0] = (float)d;
    }
    c = 1;
    int64_t e = s->start[I + 1];
    for (int64_t j = i + 1; j < e; j++) {
        if (uniform01(kdt, (uint64_t)i, (uint64_t)j) < s->rho_diag) {
            if (cols) {
                double v = s->sigma * normal01(kval, (uint64_t)i, (uint64_t)j);
                cols[c] = (int32_t)j;
                if (vd) vd[c] = v;
                if (vf) vf[c] = (float)v;
            }
            c++;
        }
    }
    for (int64_t t = s->tptr[I]; t < s->tptr[I + 1]; t++) {
        int64_t J = s->tcol[t];
        for (int64_t j = s->start[J]; j < s->start[J + 1]; j++) {
            if (uniform01(ken, (uint64_t)i, (uint64_t)j) < s->rho) {
                if (cols) {
                    double v = s->sigma * normal01(kval, (uint64_t)i, (uint64_t)j);
                    cols[c] = (int32_t)j;
                    if (vd) vd[c] = v;
                    if (vf) vf[c] = (float)v;
                }
                c++;
            }
        }
    }
    return c;
}

/* counts[r-r0] = stored entries of row r, for r in [r0, r1) */
void hsg_count_rows(void *h, int64_t r0, int64_t r1, int64_t *counts) {
    hsg_struct *s = (hsg_struct *)h;
    uint64_t kdv = stream_key(s->seed, P_DIAGV), kdt = stream_key(s->seed, P_DTILE);
    uint64_t ken = stream_key(s->seed, P_ENTRY), kval = stream_key(s->seed, P_VAL);
    #pragma omp parallel for schedule(dynamic, 256)
    for (int64_t r = r0; r < r1; r++) {
        int64_t I = block_of(s, r);
        counts[r - r0] = gen_row(s, r, I, kdv, kdt, ken, kval, NULL, NULL, NULL);
    }
}

/*
 * Fill rows [r0, r1).  rowptr_local has r1-r0+1 entries, relative offsets
 * (rowptr_local[0] == 0), as produced by a prefix sum of hsg_count_rows.
 * Exactly one of vals_d / vals_f is non-NULL (fp64 or fp32 values; the fp32
 * value is the fp64 draw rounded to nearest).
 */
void hsg_fill_rows(void *h, int64_t r0, int64_t r1, const int64_t *rowptr_local,
                   int32_t *colind, double *vals_d, float *vals_f) {
    hsg_struct *s = (hsg_struct *)h;
    uint64_t kdv = stream_key(s->seed, P_DIAGV), kdt = stream_key(s->seed, P_DTILE);
    uint64_t ken = stream_key(s->seed, P_ENTRY), kval = stream_key(s->seed, P_VAL);
    #pragma omp parallel for schedule(dynamic, 256)
    for (int64_t r = r0; r < r1; r++) {
        int64_t I = block_of(s, r);
        int64_t o = rowptr_local[r - r0];
        gen_row(s, r, I, kdv, kdt, ken, kval, colind + o,
                vals_d ? vals_d + o : NULL, vals_f ? vals_f + o : NULL);
    }
}

/* Gaussian n x m block, row-major, entry (i,k) from stream (seed, purpose) */
static void gauss_block(uint64_t seed, int purpose, int64_t n, int64_t m, double *out) {
    uint64_t k = stream_key(seed, (uint64_t)purpose);
    #pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n; i++)
        for (int64_t j = 0; j < m; j++)
            out[i * m + j] = normal01(k, (uint64_t)i, (uint64_t)j);
}

void hsg_gauss_x0(uint64_t seed, int64_t n, int64_t m, double *out) { gauss_block(seed, P_X0, n, m, out); }
void hsg_gauss_v0(uint64_t seed, int64_t n, double *out) { gauss_block(seed, P_V0, n, 1, out); }
