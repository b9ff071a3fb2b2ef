// Small dense linear algebra of the LOBPCG iteration, on the GPU in fp64,
// one workgroup per problem (problems of several solves share a launch):
//   - Cholesky-QR coefficient matrices for orthonormalising W (Section 3.1:
//     orthogonalisation of the search space, step 7 of Algorithm 1);
//   - the Rayleigh-Ritz eigenproblem of eq. 9 on an orthonormal basis, solved
//     by Householder tridiagonalisation, Sturm-count bisection and inverse
//     iteration (Golub and Van Loan, Matrix Computations, Sections 8.3.1,
//     8.4.1 and 8.2.2).
#include <type_traits>

#include "dense.h"
#include "wave.h"

namespace hsym {

constexpr int KMAX = 48;   // 3 blocks of at most 16 columns

template <typename A>
struct Batch {
    A a[32];
    int count;
};

__global__ __launch_bounds__(256) void k_small_orth(Batch<OrthArgs> b) {
    __shared__ double S[16][17], Li[16][17];
    __shared__ double dsc[16];
    __shared__ double G[KMAX * 16];   // the Gram matrix, (KB + m) x m, staged from global memory
    __shared__ int bad;
    const OrthArgs a = b.a[blockIdx.x];
    const int m = a.m, kb = a.kb, KB = kb * m;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    {
        // all loads issued before any is used: the loops below read G in
        // dependent chains, which would otherwise wait on global memory per step
        const int cnt = (KB + m) * m;
        double v[3];
#pragma unroll
        for (int t = 0; t < 3; t++) v[t] = tid + 256 * t < cnt ? a.gram[tid + 256 * t] : 0.0;
#pragma unroll
        for (int t = 0; t < 3; t++)
            if (tid + 256 * t < cnt) G[tid + 256 * t] = v[t];
    }
    __syncthreads();
    if (a.stage == 0) {
        if (tid < m) {
            const int j = tid;
            double sjj = G[(KB + j) * m + j];
            double proj = 0.0;
            for (int i = 0; i < KB; i++) proj += G[i * m + j] * G[i * m + j];
            double t = sjj - proj;
            double d;
            int deficient = 0;
            if (!(sjj > 0.0) || !isfinite(sjj)) { d = 0.0; deficient = 1; }
            else if (!(t > 1e-20 * sjj)) { d = 1.0 / sqrt(sjj); deficient = 1; }
            else d = 1.0 / sqrt(t);
            dsc[j] = d;
            if (deficient) atomicOr(a.flag, 1 << j);
        }
        __syncthreads();
        for (int e = tid; e < (KB + m) * m; e += 256) {
            int i = e / m, j = e - (e / m) * m;
            double v = i < KB ? -G[i * m + j] * dsc[j] : (i - KB == j ? dsc[j] : 0.0);
            a.coef[e] = v;
        }
        return;
    }
    // stages 1 and 2: M = S - G_B^T G_B, Cholesky, coefficients [-G_B L^-T; L^-T]
    // (M is padded to 16 x 16 with the identity, as in wg_cholqr)
    {
        const int i = tid >> 4, j = tid & 15;
        double v = i == j ? 1.0 : 0.0;
        if (i < m && j < m) {
            v = 0.5 * (G[(KB + i) * m + j] + G[(KB + j) * m + i]);
            for (int k = 0; k < KB; k++) v -= G[k * m + i] * G[k * m + j];
        }
        S[i][j] = v;
    }
    __syncthreads();
    // Cholesky M = L L^T by the first wave, rows in registers (lane r & 15 holds
    // row r), column entries broadcast with readlane; the first pivot that is
    // not clearly positive marks itself and the columns after it deficient
    if (wave == 0) {
        const int r = lane & 15;
        double g[16], dmax = 0.0;
#pragma unroll
        for (int c = 0; c < 16; c++) {
            g[c] = c <= r ? S[r][c] : 0.0;
            dmax = c < m ? fmax(dmax, fabs(S[c][c])) : dmax;
        }
        int badj = -1;
#pragma unroll
        for (int j = 0; j < 16; j++) {
            const double pj = read_lane(g[j], j);
            if (j < m && badj < 0 && (!(pj > 1e-14 * dmax) || !isfinite(pj))) badj = j;
            const double dj = sqrt(fmax(pj, 1e-300));
            const double rj = 1.0 / dj;
            const double l = (r == j) ? dj : g[j] * rj;
            g[j] = l;
#pragma unroll
            for (int c = j + 1; c < 16; c++) g[c] = fma(-l, read_lane(l, c), g[c]);
            if (lane == j) dsc[j] = rj;   // reciprocal pivots for the inverse below
        }
        if (lane < 16) {
#pragma unroll
            for (int c = 0; c < 16; c++)
                if (c <= lane) S[lane][c] = g[c];
        }
        if (lane == 0) {
            bad = badj;
            if (badj >= 0) {
                int mask = 0;
                for (int jj = badj; jj < m; jj++) mask |= 1 << jj;
                atomicOr(a.flag, mask);
            }
        }
    }
    __syncthreads();
    if (bad >= 0) {
        // the block is already orthonormal to working accuracy after stage 1:
        // a failed second pass leaves it as it is
        if (a.stage == 2)
            for (int e = tid; e < m * m; e += 256) a.coef[e] = (e / m == e % m) ? 1.0 : 0.0;
        return;
    }
    // Li = L^{-1}: column c by forward substitution, one thread per column
    if (tid < m) {
        const int c = tid;
        for (int i = 0; i < c; i++) Li[i][c] = 0.0;
        Li[c][c] = dsc[c];
        for (int i = c + 1; i < m; i++) {
            double v = 0.0;
            for (int l = c; l < i; l++) v += S[i][l] * Li[l][c];
            Li[i][c] = -v * dsc[i];
        }
    }
    __syncthreads();
    // coef rows: i < KB: -(G_B L^-T)[i][j] = -sum_k G[i][k] Li[j][k];  else L^-T[i-KB][j] = Li[j][i-KB]
    for (int e = tid; e < (KB + m) * m; e += 256) {
        int i = e / m, j = e - (e / m) * m;
        double v;
        if (i < KB) {
            v = 0.0;
            for (int k = 0; k <= j; k++) v -= G[i * m + k] * Li[j][k];
        } else {
            v = Li[j][i - KB];
        }
        a.coef[e] = v;
    }
}

void small_orth(const OrthArgs *a, int count, hipStream_t s) {
    for (int c0 = 0; c0 < count; c0 += 32) {
        Batch<OrthArgs> b;
        b.count = std::min(32, count - c0);
        for (int i = 0; i < b.count; i++) b.a[i] = a[c0 + i];
        hipLaunchKernelGGL(k_small_orth, dim3(b.count), dim3(256), 0, s, b);
        HIPCHK(hipGetLastError());
    }
}

// ---------------------------------------------------------------------------
// Rayleigh-Ritz on k x k (k <= 48), one workgroup of 256 threads:
//   0. the basis S = [X W P] is made orthonormal in coefficient space from its
//      measured Gram matrix S^T S (Cholesky, twice when needed; P dropped at a
//      small pivot) and the projected matrix formed on it;
//   1. Householder reduction to tridiagonal form T = Q^T A Q (Golub and Van
//      Loan, Section 8.3.1), a quad of lanes per row for A22 v and the
//      rank-2 update, reflectors kept for step 4;
//   2. eigenvalues of T by multisection on Sturm counts (Section 8.4.1): a
//      group of lanes per eigenvalue evaluates the count at one point each
//      per round; the m lowest, or all k when they are asked for;
//   3. eigenvectors of T for the m lowest eigenvalues by inverse iteration
//      with a partially pivoted tridiagonal LU, one lane per vector; where
//      eigenvalues cluster (gap below 1e-3 of the norm of T, the rule of
//      LAPACK's stein) the vectors are orthogonalised by Cholesky-QR, refined
//      by one more solve and orthogonalised again;
//   4. back-transformation C_X = Q Y, 16 lanes per vector.
// ---------------------------------------------------------------------------
// Number of eigenvalues of the (scaled, |d|, |e| <= 1) tridiagonal T below x:
// the number of negative pivots q_i = p_i / p_{i-1} of the LDL^T
// factorisation of T - xI, carried division-free as the pair (p_i, p_{i-1})
// of leading principal minors, p_i = (d_i - x) p_{i-1} - e_{i-1}^2 p_{i-2},
// rescaled by a power of two every 4 steps.  A pivot of magnitude below PIV
// is replaced by -PIV (the LAPACK bisection convention), which also keeps
// every p_i nonzero and each step's growth within 2^62.
// d is held in registers (KM entries; padded past k with d = 4, e^2 = 0,
// steps that keep the sign, since x lies in [-1.01, 1.01]); e^2 is read from
// LDS as a broadcast.
template <int KM>
__device__ __forceinline__ int sturm_count_r(const double (&d)[KM], const double *e2, double x) {
    constexpr double PIV = 0x1p-60;
    double p = d[0] - x, q = 1.0;
    if (fabs(p) < PIV) p = -PIV;
    int n = p < 0.0;
#pragma unroll
    for (int i = 1; i < KM; i++) {
        double tt = fma(d[i] - x, p, -e2[i - 1] * q);
        if (fabs(tt) < PIV * fabs(p)) tt = -PIV * p;
        n += (tt < 0.0) != (p < 0.0);
        q = p;
        p = tt;
        if (i % 4 == 0 || i == KM - 1) {
            const int ex = __builtin_amdgcn_frexp_exp(fmax(fabs(p), fabs(q)));
            p = __builtin_amdgcn_ldexp(p, -ex);
            q = __builtin_amdgcn_ldexp(q, -ex);
        }
    }
    return n;
}

// nit steps of inverse iteration on column c of Y with the factors of T - lam_c I
// (inverse pivots in Fd, multipliers in Fl, row swaps in piv), normalising
// after each solve.
__device__ void inv_iter(int c, int k, int nit, const double (*Fd)[17], const double (*Fu)[17],
                         const double (*Fu2)[17], const double (*Fl)[17], const unsigned char (*piv)[17],
                         double (*Y)[17], int *bad) {
    for (int it = 0; it < nit; it++) {
        double cur = Y[0][c];
#pragma unroll 4
        for (int i = 0; i + 1 < k; i++) {
            double nxt = Y[i + 1][c];
            if (piv[i][c]) { const double t = cur; cur = nxt; nxt = t; }
            Y[i][c] = cur;
            cur = fma(-Fl[i][c], cur, nxt);
        }
        double y1 = cur * Fd[k - 1][c], y2 = 0.0;
        double nn = y1 * y1;
        Y[k - 1][c] = y1;
#pragma unroll 4
        for (int i = k - 2; i >= 0; i--) {
            const double yi = (Y[i][c] - Fu[i][c] * y1 - Fu2[i][c] * y2) * Fd[i][c];
            Y[i][c] = yi;
            nn = fma(yi, yi, nn);
            y2 = y1;
            y1 = yi;
        }
        if (!(nn > 0.0) || !isfinite(nn)) { *bad = 1; return; }
        const double inv = 1.0 / sqrt(nn);
#pragma unroll 4
        for (int i = 0; i < k; i++) Y[i][c] *= inv;
    }
}

// One Cholesky-QR pass on the m columns of V (k x m, V[i][c]), whole
// workgroup: with S = diag(G)^{-1/2} and G = V^T V, factor S G S + shift I =
// L L^T and set V <- V S L^{-T}.  Leaves the smallest pivot of the scaled
// factorisation (the squared sine of the smallest angle between a column and
// the span of the ones before it, plus shift) in sh[32].  sh holds >= 33
// doubles, G >= 16 x 17.
// The factorisation always runs on 16 x 16: columns m .. 15 are padded with
// the identity (their pivots are 1 + shift and they do not touch the leading
// m x m factor), so the unrolled code has no data-dependent branches.
__device__ __forceinline__ void wg_cholqr(double (*V)[17], int k, int m, double shift, double (*G)[17], double *sh) {
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    {
        const int q = tid >> 4, c = tid & 15;
        if (c <= q) {
            double s = q == c ? 1.0 : 0.0;
            if (q < m) {
                s = 0.0;
#pragma unroll 8
                for (int i = 0; i < k; i++) s = fma(V[i][q], V[i][c], s);
            }
            G[q][c] = s;
        }
    }
    __syncthreads();
    if (wave == 0) {
        const int r = lane & 15;   // lanes 16 .. 63 repeat rows 0 .. 15 (their results are not stored)
        const double gd = G[r][r];
        const double sc = gd > 0.0 ? 1.0 / sqrt(gd) : 0.0;
        double g[16];
#pragma unroll
        for (int c = 0; c < 16; c++) {
            const double scc = read_lane(sc, c);
            g[c] = c <= r ? G[r][c] * sc * scc + (c == r ? shift : 0.0) : 0.0;
        }
        double minp = 1e300;
#pragma unroll
        for (int j = 0; j < 16; j++) {
            const double pj = read_lane(g[j], j);
            minp = j < m ? fmin(minp, pj) : minp;
            const double dj = sqrt(fmax(pj, 1e-300));
            const double rj = 1.0 / dj;
            // column j of L; entries above the diagonal (lanes < j) are never read
            const double l = (r == j) ? dj : g[j] * rj;
            g[j] = l;
#pragma unroll
            for (int c = j + 1; c < 16; c++) g[c] = fma(-l, read_lane(l, c), g[c]);
            if (lane == j) sh[j] = rj;
        }
        if (lane < 16) {
#pragma unroll
            for (int c = 0; c < 16; c++)
                if (c <= lane) G[lane][c] = g[c];
            sh[16 + lane] = sc;
        }
        if (lane == 0) sh[32] = minp;
    }
    __syncthreads();
    if (tid < k) {
        double x[16];
#pragma unroll
        for (int c = 0; c < 16; c++) {
            double v = c < m ? V[tid][c] * sh[16 + c] : 0.0;
#pragma unroll
            for (int q = 0; q < c; q++) v = fma(-x[q], G[c][q], v);
            x[c] = v * sh[c];
        }
#pragma unroll
        for (int c = 0; c < 16; c++)
            if (c < m) V[tid][c] = x[c];
    }
    __syncthreads();
}

// Z <- Z - Y (Y^T Z) for the m columns of Y and Z (k rows), whole workgroup.
__device__ void proj_out(double (*Z)[17], const double (*Y)[17], int k, int m, double (*G)[17]) {
    const int tid = threadIdx.x;
    {
        const int q = tid >> 4, j = tid & 15;
        if (q < m && j < m) {
            double s = 0.0;
#pragma unroll 8
            for (int i = 0; i < k; i++) s = fma(Y[i][q], Z[i][j], s);
            G[q][j] = s;
        }
    }
    __syncthreads();
    for (int e0 = tid; e0 < KMAX * 16; e0 += 256) {
        const int i = e0 >> 4, j = e0 & 15;
        if (i < k && j < m) {
            double v = Z[i][j];
            for (int q = 0; q < m; q++) v = fma(-Y[i][q], G[q][j], v);
            Z[i][j] = v;
        }
    }
    __syncthreads();
}

// Cholesky of the k x k (k <= 48) symmetric positive definite S (LDS) after
// scaling it to unit diagonal, by the first wave alone: lane r holds row r in
// registers; columns past k are padded with the identity.  Writes the factor
// of the scaled matrix to L (lower part), the scales 1/sqrt(S_rr) to sc and
// the pivots (the squared sine of the angle between basis vector r and the
// span of the ones before it) to pv; returns nothing (other waves skip it).
template <int KM>
__device__ void wave_chol(const double (*S)[KMAX + 1], int k, double (*L)[KMAX + 1], double *sc, double *pv) {
    const int lane = threadIdx.x & 63;
    const int r = lane < KM ? lane : KM - 1;
    const double sd = r < k ? S[r][r] : 1.0;
    const double s_r = sd > 0.0 ? 1.0 / sqrt(sd) : 0.0;
    double g[KM];
#pragma unroll
    for (int c = 0; c < KM; c++) {
        const double s_c = read_lane(s_r, c);
        g[c] = c <= r ? ((r < k) ? S[r][c] * s_r * s_c : (c == r ? 1.0 : 0.0)) : 0.0;
    }
#pragma unroll
    for (int j = 0; j < KM; j++) {
        const double pj = read_lane(g[j], j);
        const double dj = sqrt(fmax(pj, 1e-300));
        const double l = (r == j) ? dj : g[j] / dj;
        g[j] = l;
#pragma unroll
        for (int c = j + 1; c < KM; c++) g[c] = fma(-l, read_lane(l, c), g[c]);
        if (lane == j) pv[j] = pj;
    }
    if (lane < k) {
#pragma unroll
        for (int c = 0; c < KM; c++)
            if (c <= lane) L[lane][c] = g[c];
        sc[lane] = s_r;
    }
}

// Li = (D^-1 Ls)^-1 = Ls^-1 D for the factor Ls of the scaled matrix and
// D = diag(sc): one lane of the first wave per column c, forward substitution
// with the column held in registers (entries above the diagonal are zero) and
// the rows of Ls read from LDS as broadcasts.  Other threads return at once.
template <int KM>
__device__ void tri_inverse(const double (*L)[KMAX + 1], const double *sc, int k, double (*Li)[KMAX + 1]) {
    const int c = threadIdx.x;
    if (c >= 64) return;
    double li[KM];
#pragma unroll
    for (int i = 0; i < KM; i++) {
        double v = i == c ? 1.0 : 0.0;
#pragma unroll
        for (int q = 0; q < i; q++) v = fma(-L[i < k ? i : 0][q], li[q], v);
        li[i] = (i >= c && i < k) ? v / L[i < k ? i : 0][i < k ? i : 0] : 0.0;
    }
    if (c < k) {
        const double s_c = sc[c];
#pragma unroll
        for (int i = 0; i < KM; i++)
            if (i < k) Li[i][c] = li[i] * s_c;
    }
}

// B <- Li S Li^T (k x k, exactly symmetric) for lower-triangular Li; T is
// scratch; B may be S.  Whole workgroup, on the matrix cores: 16 x 16 output
// tiles dealt to the four waves, v_mfma_f64_16x16x4f64 over k-steps of 4
// (lane: li = lane & 15, lk = lane >> 4; A operand A[li][lk], B operand
// B[lk][li]; accumulator v holds row lk + 4v, column li), entries past k read
// as zero.  T = Li S takes the k-steps up to the tile row's diagonal (Li is
// lower triangular); B = T Li^T forms the tiles on and above the diagonal and
// mirrors them (on a diagonal tile only row <= column is taken).
typedef double rr_double4 __attribute__((ext_vector_type(4)));
__device__ void congruence(const double (*Li)[KMAX + 1], const double (*S)[KMAX + 1], int k,
                           double (*T)[KMAX + 1], double (*B)[KMAX + 1]) {
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int li = lane & 15, lk = lane >> 4;
    const int nt = (k + 15) >> 4;
    for (int t = wave; t < nt * nt; t += 4) {
        const int ti = t / nt, tj = t - (t / nt) * nt;
        const int r = 16 * ti + li, c = 16 * tj + li;
        const int qmax = k < 16 * ti + 16 ? k : 16 * ti + 16;
        rr_double4 acc = {0.0, 0.0, 0.0, 0.0};
        for (int q0 = 0; q0 < qmax; q0 += 4) {
            const int q = q0 + lk;
            const double av = (r < k && q < k) ? Li[r][q] : 0.0;
            const double bv = (q < k && c < k) ? S[q][c] : 0.0;
            acc = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, acc, 0, 0, 0);
        }
#pragma unroll
        for (int v = 0; v < 4; v++) {
            const int row = 16 * ti + lk + 4 * v;
            if (row < k && c < k) T[row][c] = acc[v];
        }
    }
    __syncthreads();
    for (int t = wave; t < nt * nt; t += 4) {
        const int ti = t / nt, tj = t - (t / nt) * nt;
        if (ti > tj) continue;
        const int r = 16 * ti + li, c = 16 * tj + li;
        const int qmax = k < 16 * tj + 16 ? k : 16 * tj + 16;
        rr_double4 acc = {0.0, 0.0, 0.0, 0.0};
        for (int q0 = 0; q0 < qmax; q0 += 4) {
            const int q = q0 + lk;
            const double av = (r < k && q < k) ? T[r][q] : 0.0;
            const double bv = (c < k && q < k) ? Li[c][q] : 0.0;   // Li^T[q][c]
            acc = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, acc, 0, 0, 0);
        }
#pragma unroll
        for (int v = 0; v < 4; v++) {
            const int row = 16 * ti + lk + 4 * v;
            if (row < k && c < k && row <= c) {
                B[row][c] = acc[v];
                B[c][row] = acc[v];
            }
        }
    }
    __syncthreads();
}

template <int I, int N, class F>
__device__ __forceinline__ void static_for(F &&f) {
    if constexpr (I < N) {
        f(std::integral_constant<int, I>{});
        static_for<I + 1, N>(f);
    }
}

// Householder tridiagonalisation of the symmetric k x k A (LDS, k <= KMAX) by
// the first wave alone, with no barrier: lane r holds row r in registers, the
// vectors of each step are read across lanes (readlane), and the rank-2
// update keeps the matrix exactly symmetric (both products rounded, then
// added in either order).  Leaves what the barrier version left: A with its
// diagonal and first subdiagonal (T), the reflector of step j in column j
// below the subdiagonal (first entry x0 - alpha), beta[j] = 2 / v.v and
// e[j] = alpha (0 where nothing was annihilated).
template <int KM>
__device__ void tridiag_wave(double (*A)[KMAX + 1], int k, double *beta, double *e) {
    const int lane = threadIdx.x & 63;
    const int r = lane < KM ? lane : KM - 1;
    double a[KM];
#pragma unroll
    for (int c = 0; c < KM; c++) a[c] = (lane < k && c < k) ? A[r][c] : 0.0;
    static_for<0, KM - 2>([&](auto jc) {
        constexpr int j = decltype(jc)::value;
        if (j + 2 < k) {
            const bool below = lane > j && lane < k;
            const double x = below ? a[j] : 0.0;
            const double nrm2 = wave_sum(x * x);
            const double x0 = read_lane(a[j], j + 1);
            double alpha = 0.0, bt = 0.0;
            if (nrm2 > 0.0) {
                const double nrm = sqrt(nrm2);
                alpha = x0 >= 0 ? -nrm : nrm;
                bt = 1.0 / (nrm2 - alpha * x0);   // 2 / v.v with v.v = 2 (nrm2 - alpha x0)
            }
            if (lane == 0) { beta[j] = bt; e[j] = alpha; }
            if (bt != 0.0) {
                const double v = below ? (lane == j + 1 ? x - alpha : x) : 0.0;
                // p = beta A22 v
                double p = 0.0;
#pragma unroll
                for (int c = j + 1; c < KM; c++) p = fma(a[c], read_lane(v, c), p);
                p = lane < k ? bt * p : 0.0;
                const double vp = wave_sum(v * p);
                const double w = fma(-0.5 * bt * vp, v, p);
                if (below) {
#pragma unroll
                    for (int c = j + 1; c < KM; c++) {
                        const double vc = read_lane(v, c), wc = read_lane(w, c);
                        a[c] = a[c] - __dadd_rn(__dmul_rn(v, wc), __dmul_rn(w, vc));
                    }
                }
                if (lane == j + 1) a[j] = v;   // the reflector's first entry, x0 - alpha
            }
        }
    });
    if (lane < k) {
#pragma unroll
        for (int c = 0; c < KM; c++)
            if (c < k) A[r][c] = a[c];
    }
}

// KM: the register size of the unrolled steps, at least every problem's k
// (24 covers m <= 8, 48 every block width); LDS arrays keep the KMAX layout.
template <int KM>
__global__ __launch_bounds__(256) void k_small_rr(Batch<RRArgs> b) {
    __shared__ double A[KMAX][KMAX + 1];      // lower part: reflector vectors
    __shared__ double beta[KMAX], d[KMAX], e[KMAX], ds[KMAX + 4], e2s[KMAX + 4], lam[KMAX];
    __shared__ double pv[64];
    __shared__ double Y[KMAX][17];            // Y[i][c]: tridiagonal eigenvectors, then C_X
    __shared__ double Fd[KMAX][17], Fu[KMAX][17], Fu2[KMAX][17], Fl[KMAX][17];
    __shared__ unsigned char piv[KMAX][17];
    __shared__ double Z[KMAX][17];
    __shared__ double G[16][17];
    __shared__ double GS[KMAX][KMAX + 1];     // S^T S, then scratch
    __shared__ double Lf[KMAX][KMAX + 1];     // Cholesky factor, then scratch
    __shared__ double Li[KMAX][KMAX + 1];     // the basis transform: S Li^T is orthonormal
    __shared__ double scl[KMAX], pvt[KMAX];
    __shared__ double sh[40];
    __shared__ int bad, nrounds, kk, second;
    const RRArgs a = b.a[blockIdx.x];
    const int m = a.m, k0 = a.nblk * m;
    const int tid = threadIdx.x, lane = tid & 63;
    {
        // gram is k0 x 2 k0: [S^T S | S^T (A S)]; all loads in flight
        // together, then the average of the two triangles of each
        double v[18];
#pragma unroll
        for (int t = 0; t < 18; t++) v[t] = tid + 256 * t < 2 * k0 * k0 ? a.gram[tid + 256 * t] : 0.0;
#pragma unroll
        for (int t = 0; t < 18; t++) {
            const int e0 = tid + 256 * t;
            if (e0 < 2 * k0 * k0) {
                const int i = e0 / (2 * k0), j = e0 - i * (2 * k0);
                if (j < k0) GS[i][j] = v[t];
                else A[i][j - k0] = v[t];
            }
        }
    }
    __syncthreads();
    // each half is taken from its upper triangle (the Gram may leave the
    // tiles below the diagonal unformed)
    for (int e0 = tid; e0 < k0 * k0; e0 += 256) {
        const int i = e0 / k0, j = e0 - (e0 / k0) * k0;
        if (i < j) {
            A[j][i] = A[i][j];
            GS[j][i] = GS[i][j];
        }
    }
    if (tid == 0) { bad = 0; nrounds = 0; second = 0; }
    __syncthreads();
    // Orthonormalisation of S = [X W P] (Algorithm 1, step 7) in coefficient
    // space: the Cholesky factor of the measured S^T S, in the block order X,
    // W, P, is Gram-Schmidt of W against X and of P against X and W.  P is
    // dropped for this iteration when a pivot of its column-normalised
    // projection is below P_DROP (the oracle's rank test); a second pass
    // follows when the basis was far from orthonormal.
    if (tid < 64) wave_chol<KM>(GS, k0, Lf, scl, pvt);
    __syncthreads();
    if (tid < 64) {
        // one lane per basis column j (the first wave)
        const int j = lane;
        bool drop = false;
        if (a.nblk == 3 && j >= 2 * m && j < 3 * m) {
            double nn = 0.0;
            for (int c = 2 * m; c <= j; c++) nn = fma(Lf[j][c], Lf[j][c], nn);
            // the oracle's test on the normalised projection of P, and a
            // P column whose angle to span[X W, earlier P] has a sine
            // below 1e-5: the transform would amplify the rounding of the
            // basis and of A S by more than 1e5
            const double rel = Lf[j][j] / sqrt(fmax(nn, 1e-300));
            drop = !(rel >= 1e-4) || !(pvt[j] >= 1e-10);
        }
        const int k = __ballot(drop) ? 2 * m : k0;
        // smallest pivot of the kept columns (fmin passes over NaN; lanes
        // past k carry 1)
        double pmin = j < k ? pvt[j] : 1.0;
#pragma unroll
        for (int off = 32; off > 0; off >>= 1) pmin = fmin(pmin, __shfl_xor(pmin, off));
        const bool nonfinite = j < k && (!isfinite(pvt[j]) || !isfinite(scl[j]));
        const bool any_bad = __ballot(nonfinite) != 0ull;
        if (lane == 0) {
            if (any_bad) bad = 1;
            kk = k;
            second = pmin < 1e-4;
            if (a.flag) a.flag[1] = k < k0 ? 1 : 0;
        }
    }
    __syncthreads();
    const int k = kk;
    tri_inverse<KM>(Lf, scl, k, Li);
    __syncthreads();
    if (second) {
        // Li <- L2^-1 Li with L2 L2^T = Li S^T S Li^T (Cholesky-QR twice)
        congruence(Li, GS, k, Lf, GS);
        if (tid < 64) wave_chol<KM>(GS, k, Lf, scl, pvt);
        __syncthreads();
        tri_inverse<KM>(Lf, scl, k, GS);   // GS <- L2^-1 (lower)
        __syncthreads();
        for (int e0 = tid; e0 < k * k; e0 += 256) {
            const int i = e0 / k, j = e0 - (e0 / k) * k;
            double v = 0.0;
            for (int q = j; q <= i; q++) v = fma(GS[i][q], Li[q][j], v);
            Lf[i][j] = i >= j ? v : 0.0;
        }
        __syncthreads();
        for (int e0 = tid; e0 < k * k; e0 += 256) {
            const int i = e0 / k, j = e0 - (e0 / k) * k;
            Li[i][j] = Lf[i][j];
        }
        __syncthreads();
    }
    // the projected matrix Li (S^T A S) Li^T on the orthonormal basis S Li^T
    congruence(Li, A, k, Lf, A);
    // 1. tridiagonalisation, by the first wave
    __syncthreads();
    if (tid < 64) tridiag_wave<KM>(A, k, beta, e);
    __syncthreads();
    if (tid < k) d[tid] = A[tid][tid];
    if (tid == 0) {
        if (k >= 2) e[k - 2] = A[k - 1][k - 2];
        e[k - 1] = 0.0;
        for (int j = (k >= 2 ? k - 2 : 0); j < k; j++) beta[j] = 0.0;
    }
    __syncthreads();
    // Gershgorin interval and the power-of-two scale that brings T into [-1, 1]
    double glo = d[0], ghi = d[0];
    for (int i = 0; i < k; i++) {
        const double r = (i > 0 ? fabs(e[i - 1]) : 0.0) + fabs(e[i]);
        glo = fmin(glo, d[i] - r);
        ghi = fmax(ghi, d[i] + r);
    }
    const double tnorm = fmax(fabs(glo), fabs(ghi));
    const int tex = __builtin_amdgcn_frexp_exp(tnorm + 1e-300);
    if (tid < KMAX + 4) {
        const double es = tid < k ? __builtin_amdgcn_ldexp(e[tid], -tex) : 0.0;
        ds[tid] = tid < k ? __builtin_amdgcn_ldexp(d[tid], -tex) : 4.0;
        e2s[tid] = es * es;
    }
    __syncthreads();
    // 2. eigenvalues: NG lanes per eigenvalue, one point per lane per round
    const int ne = a.evals_all ? k : m;
    {
        const int NG = ne <= 16 ? 16 : (ne <= 32 ? 8 : 4);
        const int g = tid / NG, lg = tid - g * NG;
        const int gbase = lane - lg;
        const unsigned long long gmask = (1ull << NG) - 1ull;
        double lo = __builtin_amdgcn_ldexp(glo, -tex), hi = __builtin_amdgcn_ldexp(ghi, -tex);
        const double w0 = fmax(hi - lo, 1e-300);
        lo -= 1e-12 * w0 + 1e-300;
        hi += 1e-12 * w0 + 1e-300;
        const bool act = g < ne;
        double dr[KM];
#pragma unroll
        for (int i = 0; i < KM; i++) dr[i] = ds[i];
        for (int round = 0; round < 64; round++) {
            const double h = (hi - lo) / (double)(NG + 1);
            const double x = fma((double)(lg + 1), h, lo);
            const int cnt = act ? sturm_count_r<KM>(dr, e2s, x) : 0;
            const unsigned long long bal = __ballot(act && cnt > g);
            const unsigned long long msk = (bal >> gbase) & gmask;
            if (msk == 0ull) {
                lo = fma((double)NG, h, lo);
            } else {
                const int s = __builtin_ctzll(msk);
                const double nlo = s == 0 ? lo : fma((double)s, h, lo);
                hi = fma((double)(s + 1), h, lo);
                lo = nlo;
            }
            // stop when every bracket is at rounding level (uniform across the workgroup)
            const int more = act && (hi - lo) > 2.2e-16 * (fabs(lo) + fabs(hi)) + 1e-17;
            if (tid == 0) nrounds = round + 1;
            if (__syncthreads_or(more) == 0) break;
        }
        if (act && lg == 0) lam[g] = __builtin_amdgcn_ldexp(0.5 * (lo + hi), tex);
    }
    __syncthreads();
    bool clustered = false;
    for (int c = 1; c < m; c++) clustered |= (lam[c] - lam[c - 1] <= 1e-3 * tnorm);
    // 3. inverse iteration for the m lowest eigenvectors of T, one lane each
    if (tid < m) {
        const int c = tid;
        const double tiny = 1e-300 + 2.2e-16 * tnorm;
        const double sigma = lam[c];
        double dcur = d[0] - sigma, ucur = k > 1 ? e[0] : 0.0;
        for (int i = 0; i + 1 < k; i++) {
            const double li = e[i];
            const double dn = d[i + 1] - sigma;
            const double un = (i + 2 < k) ? e[i + 1] : 0.0;
            if (fabs(dcur) >= fabs(li)) {
                const double r = 1.0 / (dcur == 0.0 ? tiny : dcur);
                const double l = li * r;
                Fd[i][c] = r; Fl[i][c] = l; Fu[i][c] = ucur; Fu2[i][c] = 0.0; piv[i][c] = 0;
                dcur = fma(-l, ucur, dn);
                ucur = un;
            } else {
                const double r = 1.0 / li;
                const double l = dcur * r;
                Fd[i][c] = r; Fl[i][c] = l; Fu[i][c] = dn; Fu2[i][c] = un; piv[i][c] = 1;
                dcur = fma(-l, dn, ucur);
                ucur = -l * un;
            }
        }
        Fd[k - 1][c] = 1.0 / (dcur == 0.0 ? tiny : dcur);
        // distinct pseudo-random start vectors (hash of index and lane)
        for (int i = 0; i < k; i++) {
            unsigned h = (unsigned)(i * 2654435761u) ^ (unsigned)((c + 1) * 40503u);
            h ^= h >> 15; h *= 2246822519u; h ^= h >> 13;
            Y[i][c] = ((double)(h & 0xffff) - 32767.5) / 32768.0;
        }
        inv_iter(c, k, clustered ? 2 : 3, Fd, Fu, Fu2, Fl, piv, Y, &bad);
    }
    __syncthreads();
    if (clustered) {
        // shifted Cholesky-QR first (never breaks down), then plain; the
        // refinement solve removes what the orthogonalisation amplified
        // outside each cluster, and a last pass restores orthogonality
        wg_cholqr(Y, k, m, 2e-11, G, sh);
        wg_cholqr(Y, k, m, 0.0, G, sh);
        if (tid < m) inv_iter(tid, k, 1, Fd, Fu, Fu2, Fl, piv, Y, &bad);
        __syncthreads();
        wg_cholqr(Y, k, m, 0.0, G, sh);
    }
    // 4. back-transformation x = H_0 H_1 ... H_{k-3} y, 16 lanes per vector
    {
        const int c = tid >> 4, r = tid & 15;
        const bool own = c < m;
        double y0 = (own && r < k) ? Y[r][c] : 0.0;
        double y1 = (own && r + 16 < k) ? Y[r + 16][c] : 0.0;
        double y2 = (own && r + 32 < k) ? Y[r + 32][c] : 0.0;
        for (int j = k - 3; j >= 0; j--) {
            const double bt = beta[j];
            if (bt == 0.0) continue;
            const double a0 = (r > j && r < k) ? A[r][j] : 0.0;
            const double a1 = (r + 16 > j && r + 16 < k) ? A[r + 16][j] : 0.0;
            const double a2 = (r + 32 > j && r + 32 < k) ? A[r + 32][j] : 0.0;
            const double s = bt * row_sum(fma(a0, y0, fma(a1, y1, a2 * y2)));
            y0 = fma(-s, a0, y0);
            y1 = fma(-s, a1, y1);
            y2 = fma(-s, a2, y2);
        }
        __syncthreads();
        if (own) {
            if (r < k) Y[r][c] = y0;
            if (r + 16 < k) Y[r + 16][c] = y1;
            if (r + 32 < k) Y[r + 32][c] = y2;
        }
    }
    if (tid < ne) {
        if (a.evals_all) a.evals_all[tid] = lam[tid];
        if (tid < m) a.theta[tid] = lam[tid];
    }
    __syncthreads();
    if (tid == 0) a.flag[0] = bad ? -1 : 1 + nrounds;
    // coefficients of the basis as stored: C = Li^T Y (rows of a dropped P
    // block are zero)
    for (int e0 = tid; e0 < k0 * m; e0 += 256) {
        const int i = e0 / m, j = e0 - (e0 / m) * m;
        double v = 0.0;
        if (i < k)
            for (int r = i; r < k; r++) v = fma(Li[r][i], Y[r][j], v);
        a.coef[i * 2 * m + j] = v;
    }
    // Next search direction in coefficient space (step 10): on the
    // orthonormal basis S Li^T, whose first m vectors span the old X, the
    // components of the new X outside the old X, made orthogonal to the new X
    // and orthonormal (span{C_X, C_P} = span{C_X, Y} with Y = C_X with its X
    // rows zeroed).
    const int kr = k - m;
    if (kr == 0) {          // Rayleigh-Ritz on X alone: no search direction yet
        for (int e0 = tid; e0 < k0 * m; e0 += 256) {
            const int i = e0 / m, j = e0 - (e0 / m) * m;
            a.coef[i * 2 * m + m + j] = 0.0;
        }
        return;
    }
    for (int e0 = tid; e0 < KMAX * 16; e0 += 256) {
        const int i = e0 >> 4, j = e0 & 15;
        if (i < k && j < m) Z[i][j] = i < m ? 0.0 : Y[i][j];
    }
    __syncthreads();
    proj_out(Z, Y, k, m, G);
    proj_out(Z, Y, k, m, G);
    // Cholesky-QR twice (re-projected in between) unless some column is
    // (nearly) dependent on the others: then modified Gram-Schmidt with
    // replacement of vanishing columns
    wg_cholqr(Z, k, m, 0.0, G, sh);
    const bool deficient = !(sh[32] > 1e-14);
    __syncthreads();
    if (!deficient) {
        proj_out(Z, Y, k, m, G);
        wg_cholqr(Z, k, m, 0.0, G, sh);
    } else {
        for (int e0 = tid; e0 < KMAX * 16; e0 += 256) {
            const int i = e0 >> 4, j = e0 & 15;
            if (i < k && j < m) Z[i][j] = i < m ? 0.0 : Y[i][j];
        }
        __syncthreads();
        proj_out(Z, Y, k, m, G);
        proj_out(Z, Y, k, m, G);
        int next_unit = m;
        for (int j = 0; j < m; j++) {
            if (tid < 64) {
                const double z = lane < k ? Z[lane][j] : 0.0;
                const double n0 = wave_sum(z * z);
                if (lane == 0) sh[0] = sqrt(n0);
            }
            __syncthreads();
            double n0 = sh[0];
            for (int attempt = 0; attempt < 4; attempt++) {
                for (int pass = 0; pass < 2; pass++) {
                    if (tid < j + m) {
                        // against the previous Z columns (tid < j) and C_X (j <= tid < j + m)
                        double dsum = 0.0;
                        if (tid < j) for (int i = 0; i < k; i++) dsum = fma(Z[i][tid], Z[i][j], dsum);
                        else for (int i = 0; i < k; i++) dsum = fma(Y[i][tid - j], Z[i][j], dsum);
                        pv[tid] = dsum;
                    }
                    __syncthreads();
                    if (tid < k) {
                        double v = Z[tid][j];
                        for (int q = 0; q < j; q++) v -= pv[q] * Z[tid][q];
                        for (int q = 0; q < m; q++) v -= pv[j + q] * Y[tid][q];
                        Z[tid][j] = v;
                    }
                    __syncthreads();
                }
                if (tid < 64) {
                    const double z = lane < k ? Z[lane][j] : 0.0;
                    const double nn = wave_sum(z * z);
                    if (lane == 0) sh[1] = sqrt(nn);
                }
                __syncthreads();
                const double nn = sh[1];
                const bool ok = nn > 1e-12 * n0 && nn > 1e-300;
                if (tid < k) Z[tid][j] = ok ? Z[tid][j] / nn : ((tid == next_unit) ? 1.0 : 0.0);
                __syncthreads();
                if (ok) break;
                next_unit = (next_unit + 1 < k) ? next_unit + 1 : m;
                n0 = 1.0;
            }
        }
    }
    for (int e0 = tid; e0 < k0 * m; e0 += 256) {
        const int i = e0 / m, j = e0 - (e0 / m) * m;
        double v = 0.0;
        if (i < k)
            for (int r = i; r < k; r++) v = fma(Li[r][i], Z[r][j], v);
        a.coef[i * 2 * m + m + j] = v;
    }
}

void small_rr(const RRArgs *a, int count, hipStream_t s) {
    for (int c0 = 0; c0 < count; c0 += 32) {
        Batch<RRArgs> b;
        b.count = std::min(32, count - c0);
        for (int i = 0; i < b.count; i++) b.a[i] = a[c0 + i];
        int kmax = 0;
        for (int i = 0; i < b.count; i++) kmax = std::max(kmax, b.a[i].nblk * b.a[i].m);
        if (kmax <= 24) hipLaunchKernelGGL(k_small_rr<24>, dim3(b.count), dim3(256), 0, s, b);
        else hipLaunchKernelGGL(k_small_rr<KMAX>, dim3(b.count), dim3(256), 0, s, b);
        HIPCHK(hipGetLastError());
    }
}

}  // namespace hsym
