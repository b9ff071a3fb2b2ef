// Launchers of the block-vector kernels (dense.hip) and the small dense
// kernels (small.hip).
#pragma once
#include "hsym_internal.h"

namespace hsym {

struct GramArgs {
    const double *a[3];
    const double *b[6];
    int na, nb;       // number of n x m blocks on each side
    int m;
    int64_t n;
    // 1: b = [a, A a] (the Rayleigh-Ritz Gram [S^T S | S^T A S]) and only the
    // blocks on and above the diagonal of each half are needed; with
    // na * m a multiple of 16 the 16 x 16 tiles below them are left zero
    int sym;
};
// out (na*m x nb*m, row-major) = [a]^T [b]; scratch >= gram_scratch_bytes
void gram(const GramArgs &g, double *out, double *scratch, hipStream_t s);
size_t gram_scratch_bytes(int64_t n, int K1, int K2);

struct LincombArgs {
    const double *in[6];   // set 0: in[0..nin), set 1: in[3..3+nin) (not an output of set 0)
    double *out[4];        // set 0: out[0..nout), set 1: out[2..2+nout)
    const double *coef;    // (nin*m) x (nout*m), row stride ldc, device
    int ldc;
    int nin, nout, nsets, m;
    int64_t n;
    const double *theta;   // optional: residual of (set1 out0) - (set0 out0) diag(theta)
    double *res;
    double *norm_part;     // lincomb_norm_parts(n) x m
    const int *skip;       // optional device flag: nonzero -> the launch writes nothing
};
void lincomb(const LincombArgs &a, hipStream_t s);
// workgroups of a linear combination over n rows (also its residual-norm
// partials): at most HSYM_LINCOMB_WGS, each over lincomb_tiles_per_wg(n) tiles
// of 64 rows
#ifndef HSYM_LINCOMB_WGS
#define HSYM_LINCOMB_WGS 1536
#endif
__host__ __device__ inline int64_t lincomb_tiles_per_wg(int64_t n) {
    const int64_t nt = (n + 63) / 64;
    const int64_t wgs = nt < HSYM_LINCOMB_WGS ? nt : HSYM_LINCOMB_WGS;
    return wgs > 0 ? (nt + wgs - 1) / wgs : 1;
}
__host__ __device__ inline int64_t lincomb_norm_parts(int64_t n) {
    const int64_t tpw = lincomb_tiles_per_wg(n);
    return ((n + 63) / 64 + tpw - 1) / tpw;
}
void colsum_final(const double *part, int64_t nparts, int m, double *out, hipStream_t s);
void precond_apply(hsym_matrix *H, int kind, double *W, const double *mu, double delta, int m, hipStream_t s,
                   int fom_iters = 3);
void to_f32(const double *x, float *y, int64_t cnt, hipStream_t s);

// Gaussian block from the counter-based generator (SplitMix64 over a Weyl
// sequence, Box-Muller cosine branch): entry (i, j) of the stream (seed,
// purpose).  Only the columns set in `mask` are written (mask = -1: all).
void gauss_fill(double *V, int64_t n, int m, int64_t ld, uint64_t seed, uint64_t purpose, int mask,
                hipStream_t s);
// evecs[:, j] = sign_j X[:, j] for j < nev (ld nev), sign_j making the
// largest-magnitude entry of column j positive (first such row on ties).
void sign_fix_copy(const double *X, int m, int nev, int64_t n, double *evecs, double *scratch, hipStream_t s);
size_t sign_fix_scratch_bytes(int64_t n, int m);

// h[0..k) = V_j . w (V_j = V + j*ldv, n long); scratch >= dots_scratch_bytes(n, k)
void dots(const double *V, int64_t ldv, int k, const double *w, int64_t n, double *h, double *scratch,
          hipStream_t s);
size_t dots_scratch_bytes(int64_t n, int k);
void sub_vh(const double *V, int64_t ldv, const double *h, int k, double *w, int64_t n, hipStream_t s);
void axpby2(double *w, const double *v1, const double *ab, const double *v0, int64_t n, hipStream_t s);
void scale_to(const double *w, const double *nrm2, double *v, int64_t n, hipStream_t s);

// ---------------------------------------------------------------------------
// small dense kernels (one workgroup per problem, batched over problems)
// ---------------------------------------------------------------------------
// Orthonormalisation of W against B = [X P] (kb = number of basis blocks) and
// itself, driven by Gram matrices G = [B W]^T W ((kb+1)m x m):
//   stage 0: coef = [-G_B D; D], D = diag of inverse projected column norms
//   stage 1: coef = [-G_B L^-T; L^-T] with L L^T = W^T W - G_B^T G_B
//   stage 2: coef = L^-T with L L^T = W^T W   (second Cholesky-QR pass)
// flag[0] receives a bit mask of deficient columns (stage 0/1) or 1 when the
// Cholesky factorisation failed.
struct OrthArgs {
    const double *gram;   // (kb+1)m x m
    double *coef;         // (kb+1)m x m  (stage 2: m x m)
    int *flag;
    int kb, m, stage;
};
void small_orth(const OrthArgs *a, int count, hipStream_t s);

// Rayleigh-Ritz on the projected matrix A = S^T (H S) (k x k, k = nblk*m,
// S = [X W P] orthonormal): eigenvalues ascending; coef = [C_X | C_P]
// (k x 2m): C_X = the m lowest Ritz vectors, C_P an orthonormal basis of the
// W,P-components of C_X made orthogonal to C_X; theta[0..m).
struct RRArgs {
    // k x 2k (k = nblk*m): [S^T S | S^T A S] for the basis S of nblk blocks
    const double *gram;
    double *coef;         // k x 2m: C_X and C_P for the stored basis
    double *theta;        // m
    double *evals_all;    // k (diagnostics), or null: then only the m lowest are computed
    int *flag;            // [0]: 1 + multisection rounds used (>0), or -1 on failure;
                          // [1]: 1 when the P block was dropped, else 0
    int nblk, m;
};
void small_rr(const RRArgs *a, int count, hipStream_t s);
void set_int(int *p, int v, hipStream_t s);

// ---- batched forms (argument tables in device memory, blockIdx.y = problem) ----
struct GramJob {
    GramArgs g;
    double *part;      // gram_scratch_bytes(n, K1, K2)
    int64_t rpw;       // rows per partial
    int parts;         // gram_parts(n)
    int kk;            // K1 * K2
    double *out;
};
// every job has the same K1 = na*m and K2 = nb*m
void gram_batched(const GramJob *jobs, int count, int K1, int K2, int max_parts, hipStream_t s);
// every table entry passes the shape checks of lincomb()
void lincomb_batched(const LincombArgs *tab, int count, int64_t max_n, hipStream_t s);
// W' = lincomb l (one set, one output W') followed by out = g (the Gram
// [A_0 .. W']^T W', with W' the last A block and the only B block), fused into
// one pass over the rows when m = 16, else the two calls
bool lincomb_gram_fusable(const LincombArgs &l, const GramArgs &g);
void lincomb_gram(const LincombArgs &l, const GramArgs &g, double *out, double *scratch, hipStream_t s);
// batched fused form (all fusable, K1 = na * 16, GramJob::rpw = gram_rows, blocks
// 16-byte aligned)
void lincomb_gram_batched(const LincombArgs *lt, const GramJob *gt, int count, int na, int max_parts,
                          hipStream_t s);
struct ColsumJob {
    const double *part;
    int64_t nparts;
    int m;
    double *out;
};
void colsum_batched(const ColsumJob *jobs, int count, int m, hipStream_t s);
struct JacobiJob {
    double *W;
    const double *diag;
    const double *mu;
    double delta;
    int64_t n;
};
void jacobi_batched(const JacobiJob *jobs, int count, int m, int64_t max_n, hipStream_t s);
void set_ints(int *const *p, int count, int v, hipStream_t s);
void gather_words(const int *const *src, int *dst, int words, int count, hipStream_t s);
int gram_parts(int64_t n);
int64_t gram_rows(int64_t n, int parts);   // rows per partial (a multiple of 64)
// Jacobi apply W[r][c] /= g(d_r - mu_c) (in place, W = the last A block and the
// only B block of g, m = 16) followed by out = g, fused into one pass
bool jacobi_gram_fusable(const GramArgs &g);
void jacobi_gram(const GramArgs &g, const double *diag, const double *mu, double delta, double *out,
                 double *scratch, hipStream_t s);

struct OrthWork {
    double *gbuf;       // >= 48*16 doubles, device
    double *coef;       // >= 48*16 doubles, device
    double *gram_scr;   // >= gram_scratch_bytes(n, 3m, m)
    int *flag_d;        // device int
    int *flag_h;        // pinned host int
};
int orthonormalize_block(int64_t n, int m, double *V, const double *const *B, int kb, uint64_t seed,
                         OrthWork &w, hipStream_t s);

}  // namespace hsym
