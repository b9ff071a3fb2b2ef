// Small dense linear algebra of the LOBPCG iteration, on the GPU in fp64,
// one workgroup per problem (problems of several solves share a launch):
//   - Cholesky-QR coefficient matrices for orthonormalising W (Section 3.1:
//     orthogonalisation of the search space, step 7 of Algorithm 1);
//   - the Rayleigh-Ritz eigenproblem of eq. 9 on an orthonormal basis, solved
//     by cyclic Jacobi rotations with the round-robin parallel ordering
//     (Golub and Van Loan, Matrix Computations, Sections 8.5.2 and 8.5.4).
#include "dense.h"

namespace hsym {

constexpr int KMAX = 48;   // 3 blocks of at most 16 columns

template <typename A>
struct Batch {
    A a[32];
    int count;
};

// In-place Cholesky of the m x m SPD matrix s (row-major, lower factor kept),
// single thread.  Returns -1 on success or the first failing column.
__device__ int chol_lower(double *s, int ld, int m) {
    double dmax = 0.0;
    for (int j = 0; j < m; j++) dmax = fmax(dmax, fabs(s[j * ld + j]));
    for (int j = 0; j < m; j++) {
        double d = s[j * ld + j];
        for (int k = 0; k < j; k++) d -= s[j * ld + k] * s[j * ld + k];
        if (!(d > 1e-14 * dmax) || !isfinite(d)) return j;
        d = sqrt(d);
        s[j * ld + j] = d;
        for (int i = j + 1; i < m; i++) {
            double v = s[i * ld + j];
            for (int k = 0; k < j; k++) v -= s[i * ld + k] * s[j * ld + k];
            s[i * ld + j] = v / d;
        }
    }
    return -1;
}

// Linv = L^{-1} (lower triangular), single thread
__device__ void tri_inv_lower(const double *L, int ld, double *Li, int ldi, int m) {
    for (int j = 0; j < m; j++) {
        Li[j * ldi + j] = 1.0 / L[j * ld + j];
        for (int i = j + 1; i < m; i++) {
            double s = 0.0;
            for (int k = j; k < i; k++) s += L[i * ld + k] * Li[k * ldi + j];
            Li[i * ldi + j] = -s / L[i * ld + i];
        }
        for (int i = 0; i < j; i++) Li[i * ldi + j] = 0.0;
    }
}

__global__ __launch_bounds__(256) void k_small_orth(Batch<OrthArgs> b) {
    __shared__ double S[16][17], Li[16][17];
    __shared__ double dsc[16];
    __shared__ int bad;
    const OrthArgs a = b.a[blockIdx.x];
    const int m = a.m, kb = a.kb, KB = kb * m;
    const double *G = a.gram;   // (KB + m) x m
    const int tid = threadIdx.x;
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
    for (int e = tid; e < m * m; e += 256) {
        int i = e / m, j = e - (e / m) * m;
        double v = 0.5 * (G[(KB + i) * m + j] + G[(KB + j) * m + i]);
        for (int k = 0; k < KB; k++) v -= G[k * m + i] * G[k * m + j];
        S[i][j] = v;
    }
    __syncthreads();
    if (tid == 0) {
        int f = chol_lower(&S[0][0], 17, m);
        bad = f;
        if (f >= 0) {
            int mask = 0;
            for (int j = f; j < m; j++) mask |= 1 << j;
            atomicOr(a.flag, mask);
        } else {
            tri_inv_lower(&S[0][0], 17, &Li[0][0], 17, m);
        }
    }
    __syncthreads();
    if (bad >= 0) return;
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
// Rayleigh-Ritz: parallel cyclic Jacobi on k x k (k <= 48)
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_small_rr(Batch<RRArgs> b) {
    __shared__ double A[KMAX][KMAX + 1], A2[KMAX][KMAX + 1];
    __shared__ double V[KMAX][KMAX + 1], V2[KMAX][KMAX + 1];
    __shared__ double rc[KMAX / 2], rs[KMAX / 2];
    __shared__ int partner[KMAX + 1], pidx[KMAX + 1], isp[KMAX + 1];
    __shared__ double offs, fro;
    __shared__ int perm[KMAX];
    __shared__ double ev[KMAX];
    __shared__ double Z[KMAX][17];
    const RRArgs a = b.a[blockIdx.x];
    const int m = a.m, k = a.nblk * m;
    const int kp = (k + 1) & ~1;          // even number of players (one dummy if k is odd)
    const int tid = threadIdx.x;
    for (int e = tid; e < k * k; e += 256) {
        int i = e / k, j = e - (e / k) * k;
        A[i][j] = 0.5 * (a.gram[i * k + j] + a.gram[j * k + i]);
        V[i][j] = (i == j) ? 1.0 : 0.0;
    }
    __syncthreads();
    if (tid == 0) {
        double f = 0.0;
        for (int i = 0; i < k; i++)
            for (int j = 0; j < k; j++) f += A[i][j] * A[i][j];
        fro = f;
    }
    __syncthreads();
    int sweeps = 0;
    for (; sweeps < 40; sweeps++) {
        if (tid == 0) {
            double o = 0.0;
            for (int i = 0; i < k; i++)
                for (int j = 0; j < k; j++)
                    if (i != j) o += A[i][j] * A[i][j];
            offs = o;
        }
        __syncthreads();
        if (offs <= 1e-30 * fro || offs == 0.0) break;
        for (int r = 0; r < kp - 1; r++) {
            // circle-method pairing of round r
            if (tid < kp / 2) {
                int p, q;
                if (tid == 0) { p = kp - 1; q = r; }
                else { p = (r + tid) % (kp - 1); q = (r - tid + (kp - 1)) % (kp - 1); }
                if (p > q) { int t = p; p = q; q = t; }
                partner[p] = q; partner[q] = p;
                pidx[p] = tid; pidx[q] = tid;
                isp[p] = 1; isp[q] = 0;
                double c = 1.0, s = 0.0;
                if (q < k) {
                    double apq = A[p][q];
                    if (apq != 0.0) {
                        double tau = (A[q][q] - A[p][p]) / (2.0 * apq);
                        double t = (tau >= 0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
                        c = 1.0 / sqrt(1.0 + t * t);
                        s = t * c;
                    }
                }
                rc[tid] = c; rs[tid] = s;
            }
            __syncthreads();
            // A' = J^T A J and V' = V J for all disjoint rotations at once.  Only the
            // upper triangle of A' is computed and mirrored, so A stays exactly
            // symmetric (rotations cannot remove an antisymmetric rounding part).
            for (int e = tid; e < k * k; e += 256) {
                int x = e / k, y = e - (e / k) * k;
                int yb = partner[y];
                double cy = rc[pidx[y]], sy = isp[y] ? -rs[pidx[y]] : rs[pidx[y]];
                double w = cy * V[x][y];
                if (yb < k) w += sy * V[x][yb];
                V2[x][y] = w;
                if (x > y) continue;
                int xb = partner[x];
                double cx = rc[pidx[x]], sx = isp[x] ? -rs[pidx[x]] : rs[pidx[x]];
                double v = cx * cy * A[x][y];
                if (yb < k) v += cx * sy * A[x][yb];
                if (xb < k) v += sx * cy * A[xb][y];
                if (xb < k && yb < k) v += sx * sy * A[xb][yb];
                A2[x][y] = v;
                A2[y][x] = v;
            }
            __syncthreads();
            for (int e = tid; e < k * k; e += 256) {
                int x = e / k, y = e - (e / k) * k;
                A[x][y] = A2[x][y];
                V[x][y] = V2[x][y];
            }
            __syncthreads();
        }
    }
    if (tid == 0) {
        for (int i = 0; i < k; i++) { perm[i] = i; ev[i] = A[i][i]; }
        for (int i = 0; i < k; i++) {          // selection sort, ascending
            int b2 = i;
            for (int j = i + 1; j < k; j++) if (ev[perm[j]] < ev[perm[b2]]) b2 = j;
            int t = perm[i]; perm[i] = perm[b2]; perm[b2] = t;
        }
        a.flag[0] = (sweeps < 40 || offs <= 1e-24 * fro) ? sweeps + 1 : -1;
    }
    __syncthreads();
    if (tid < k) a.evals_all[tid] = ev[perm[tid]];
    if (tid < m) a.theta[tid] = ev[perm[tid]];
    // C_X = first m sorted eigenvectors
    for (int e = tid; e < k * m; e += 256) {
        int i = e / m, j = e - (e / m) * m;
        a.coef[i * 2 * m + j] = V[i][perm[j]];
    }
    // Z = C_rest^T Y, Y = C_X with its X rows zeroed; (k-m) x m
    const int kr = k - m;
    if (kr == 0) {          // Rayleigh-Ritz on X alone: no search direction yet
        for (int e = tid; e < k * m; e += 256) {
            int i = e / m, j = e - (e / m) * m;
            a.coef[i * 2 * m + m + j] = 0.0;
        }
        return;
    }
    for (int e = tid; e < kr * m; e += 256) {
        int i = e / m, j = e - (e / m) * m;
        double s = 0.0;
        for (int t = m; t < k; t++) s += V[t][perm[m + i]] * V[t][perm[j]];
        Z[i][j] = s;
    }
    __syncthreads();
    if (tid == 0) {
        // modified Gram-Schmidt, two passes; a vanishing column is replaced by a unit vector
        int next_unit = 0;
        for (int j = 0; j < m; j++) {
            double n0 = 0.0;
            for (int i = 0; i < kr; i++) n0 += Z[i][j] * Z[i][j];
            n0 = sqrt(n0);
            for (int attempt = 0; attempt < 4; attempt++) {
                for (int pass = 0; pass < 2; pass++)
                    for (int q = 0; q < j; q++) {
                        double d = 0.0;
                        for (int i = 0; i < kr; i++) d += Z[i][q] * Z[i][j];
                        for (int i = 0; i < kr; i++) Z[i][j] -= d * Z[i][q];
                    }
                double nn = 0.0;
                for (int i = 0; i < kr; i++) nn += Z[i][j] * Z[i][j];
                nn = sqrt(nn);
                if (nn > 1e-12 * n0 && nn > 1e-300) {
                    for (int i = 0; i < kr; i++) Z[i][j] /= nn;
                    break;
                }
                for (int i = 0; i < kr; i++) Z[i][j] = (i == (next_unit % kr)) ? 1.0 : 0.0;
                next_unit++;
                n0 = 1.0;
            }
        }
    }
    __syncthreads();
    // C_P = C_rest Z
    for (int e = tid; e < k * m; e += 256) {
        int i = e / m, j = e - (e / m) * m;
        double s = 0.0;
        for (int t = 0; t < kr; t++) s += V[i][perm[m + t]] * Z[t][j];
        a.coef[i * 2 * m + m + j] = s;
    }
}

void small_rr(const RRArgs *a, int count, hipStream_t s) {
    for (int c0 = 0; c0 < count; c0 += 32) {
        Batch<RRArgs> b;
        b.count = std::min(32, count - c0);
        for (int i = 0; i < b.count; i++) b.a[i] = a[c0 + i];
        hipLaunchKernelGGL(k_small_rr, dim3(b.count), dim3(256), 0, s, b);
        HIPCHK(hipGetLastError());
    }
}

}  // namespace hsym
