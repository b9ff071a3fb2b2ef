/*
 * hsym_kernels.h - step-level entry points of the LOBPCG hot path, exposed
 * so each step can be checked on its own against a plain implementation.
 * Same conventions as hsym.h: int status, device pointers, row-major n x m
 * fp64 blocks with leading dimension m (m <= 16), stream as void*, async.
 */
#ifndef HSYM_KERNELS_H
#define HSYM_KERNELS_H

#include <stdint.h>
#include "hsym.h"

#ifdef __cplusplus
extern "C" {
#endif

/*
 * Block inner product G = [A_0 .. A_{na-1}]^T [B_0 .. B_{nb-1}] (Section 4.4,
 * "block inner product"): A and B are host arrays of na (1..3), nb (1..6) device
 * pointers to n x m blocks; G is device (na*m) x (nb*m) row-major.  Reduced
 * in a fixed order (bitwise reproducible).  Scratch is allocated per call.
 * nb may be up to 6 (the Rayleigh-Ritz Gram of [X W P] against [X W P AX AW AP]).
 */
int hsym_kernel_gram(int64_t n, int m, int na, const double *const *A, int nb, const double *const *B,
                     double *G, void *stream);

/*
 * hsym_kernel_gram without allocation, for callers that cannot allocate
 * device memory (code under HIP graph capture, tight serving loops, harnesses
 * that forbid hipMalloc).  Same arguments, kernels and result (bitwise) as
 * hsym_kernel_gram, but the per-slice partials live in a static device array
 * of 36 MiB per GPU (room for K1 = na*m <= 48, K2 = nb*m <= 96 and up to 1024
 * row slices, i.e. every accepted shape), held until the process ends.  The
 * call only enqueues work on `stream` and returns: G is ready when the stream
 * is.  Every call on a GPU shares that GPU's array, so calls that overlap on
 * one GPU (other streams, other threads) race: order them on one stream.
 * Makes no hipMalloc/hipFree call.  Errors: HSYM_E_INVALID_ARG (sizes, NULL,
 * partials beyond the array), HSYM_E_DEVICE (symbol lookup failed).
 */
int hsym_kernel_gram_noalloc(int64_t n, int m, int na, const double *const *A, int nb, const double *const *B,
                             double *G, void *stream);

/*
 * Linear combination (Section 4.4, "linear combination", eq. 7):
 * Out_q = sum_i In_i C[i*m:(i+1)*m, q*m:(q+1)*m] for nin (1..3) inputs and
 * nout (1..2) outputs; C is device (nin*m) x (nout*m) with row stride ldc.
 * Outputs may alias inputs.
 */
int hsym_kernel_lincomb(int64_t n, int m, int nin, const double *const *In, int nout, double *const *Out,
                        const double *C, int ldc, void *stream);

/*
 * Rayleigh-Ritz of eq. 9 on a basis S of nblk (1..3) blocks of m columns
 * (Algorithm 1, steps 7-9), k = nblk*m: G is device k x 2k row-major,
 * [S^T S | S^T A S]; each half is read from its upper triangle (the entries
 * below the diagonal are not used).  The basis is made
 * orthonormal in coefficient space from S^T S: its Cholesky factor in the
 * block order [X W P] is Gram-Schmidt of W against X and of P against X and
 * W (a second factorisation follows when a pivot is below 1e-4); the third
 * block is dropped when a pivot of its column-normalised projection is below
 * 1e-4 or one of its columns makes an angle with a sine below 1e-5 with the
 * span of the columns before it, reported in *p_dropped (host int, may be
 * NULL).  Eigenvalues of the
 * projected matrix by bisection on Sturm counts of the Householder
 * tridiagonal form, eigenvectors by inverse iteration (accuracy: eigenvalues
 * and residuals within a small multiple of k * eps * ||A|| when S^T S = I).
 * Writes theta (device, m lowest eigenvalues ascending), evals (device, all
 * eigenvalues of the kept basis), and coef (device k x 2m, for S as given):
 * columns 0..m-1 the Ritz vectors C_X, columns m..2m-1 the coefficients of
 * the next search direction: a basis of the components of S C_X outside the
 * first block, orthonormal and orthogonal to S C_X (zero when nblk = 1);
 * rows of a dropped block are zero.
 */
int hsym_kernel_rayleigh_ritz(int nblk, int m, const double *G, double *theta, double *evals, double *coef,
                              int *p_dropped, void *stream);

/*
 * Preconditioner apply of eq. 11 in place on W (device n x m):
 * W_j <- (Htilde - mu_j I)^{-1} W_j with Htilde = diag(H) (HSYM_PRECOND_JACOBI)
 * or the 64x64 diagonal blocks (HSYM_PRECOND_BLOCK64, handle built with
 * HSYM_BUILD_BLOCK64); mu device[m]; denominators are kept >= delta in size.
 * HSYM_PRECOND_FOM (group tiles attached with hsym_attach_group_tiles) gives
 * 3 steps of the full orthogonalization method per tile and column, the
 * pivots of its small Hessenberg solve kept >= delta in size.
 */
int hsym_kernel_precond(hsym_t H, int kind, int m, double *W, const double *mu, double delta, void *stream);

/*
 * Cholesky-QR orthonormalisation of V (device n x m) against nb (0..2)
 * device blocks B with orthonormal columns, then against itself: on return
 * [B V] has orthonormal columns and span(B, V) is unchanged.  Columns found
 * numerically inside span(B) are replaced by seeded Gaussian columns
 * (*replaced counts them).  Host-synchronous on the stream.
 */
int hsym_kernel_orthonormalize(int64_t n, int m, double *V, int nb, const double *const *B, uint64_t seed,
                               int *replaced, void *stream);

#ifdef __cplusplus
}
#endif
#endif
