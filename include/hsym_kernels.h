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
 * "block inner product"): A and B are host arrays of na, nb (1..3) device
 * pointers to n x m blocks; G is device (na*m) x (nb*m) row-major.  Reduced
 * in a fixed order (bitwise reproducible).  Scratch is allocated per call.
 */
int hsym_kernel_gram(int64_t n, int m, int na, const double *const *A, int nb, const double *const *B,
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
 * Rayleigh-Ritz of eq. 9 on an orthonormal basis of nblk (1..3) blocks:
 * A is device k x k (k = nblk*m), symmetrised on input.  Eigenvalues by
 * bisection on Sturm counts of the Householder tridiagonal form, eigenvectors
 * by inverse iteration (accuracy: eigenvalues and residuals within a small
 * multiple of k * eps * ||A||).  Writes theta (device,
 * m lowest eigenvalues ascending), evals (device, all k), and coef (device
 * k x 2m): columns 0..m-1 the m lowest eigenvectors C_X, columns m..2m-1 an
 * orthonormal basis of the rows m..k-1 of C_X made orthogonal to C_X (the
 * coefficients of the next search direction; zero when nblk = 1).
 */
int hsym_kernel_rayleigh_ritz(int nblk, int m, const double *A, double *theta, double *evals, double *coef,
                              void *stream);

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
