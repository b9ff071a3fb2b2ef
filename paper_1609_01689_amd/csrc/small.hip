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
    if (tid == 0) bad = -1;
    __syncthreads();
    // right-looking Cholesky S = L L^T, in place in the lower triangle
    double dmax = 0.0;
    for (int j = 0; j < m; j++) dmax = fmax(dmax, fabs(S[j][j]));
    for (int j = 0; j < m; j++) {
        const double d = S[j][j];
        if (!(d > 1e-14 * dmax) || !isfinite(d)) {
            if (tid == 0) {
                bad = j;
                int mask = 0;
                for (int jj = j; jj < m; jj++) mask |= 1 << jj;
                atomicOr(a.flag, mask);
            }
            break;
        }
        const double sd = sqrt(d);
        __syncthreads();
        if (tid < m && tid > j) S[tid][j] /= sd;
        if (tid == 0) S[j][j] = sd;
        __syncthreads();
        for (int e = tid; e < m * m; e += 256) {
            const int i = e / m, l = e - (e / m) * m;
            if (l > j && i >= l) S[i][l] -= S[i][j] * S[l][j];
        }
        __syncthreads();
    }
    __syncthreads();
    if (bad >= 0) return;
    // Li = L^{-1}: column c by forward substitution, one thread per column
    if (tid < m) {
        const int c = tid;
        for (int i = 0; i < c; i++) Li[i][c] = 0.0;
        Li[c][c] = 1.0 / S[c][c];
        for (int i = c + 1; i < m; i++) {
            double v = 0.0;
            for (int l = c; l < i; l++) v += S[i][l] * Li[l][c];
            Li[i][c] = -v / S[i][i];
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
// Rayleigh-Ritz: parallel cyclic Jacobi on k x k (k <= 48)
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_small_rr(Batch<RRArgs> b) {
    __shared__ double A[2][KMAX][KMAX + 1];
    __shared__ double V[2][KMAX][KMAX + 1];
    __shared__ double cj[KMAX + 1], sj[KMAX + 1];   // rotation of the pair index x belongs to
    __shared__ double fro;
    __shared__ int nrot;
    __shared__ int perm[KMAX];
    __shared__ double ev[KMAX];
    __shared__ double Z[KMAX][17];
    __shared__ double dq[16];
    const RRArgs a = b.a[blockIdx.x];
    const int m = a.m, k = a.nblk * m;
    const int kp = (k + 1) & ~1;          // even number of players (one dummy if k is odd)
    const int km = kp - 1;
    const int tid = threadIdx.x;
    for (int e = tid; e < k * k; e += 256) {
        int i = e / k, j = e - (e / k) * k;
        A[0][i][j] = 0.5 * (a.gram[i * k + j] + a.gram[j * k + i]);
        V[0][i][j] = (i == j) ? 1.0 : 0.0;
    }
    if (tid == 0) fro = 0.0;
    __syncthreads();
    if (tid < 64) {
        double f = 0.0;
        for (int e = tid; e < k * k; e += 64) f += A[0][e / k][e % k] * A[0][e / k][e % k];
        for (int off = 32; off > 0; off >>= 1) f += __shfl_down(f, off, 64);
        if (tid == 0) fro = f;
    }
    __syncthreads();
    // a rotation is applied when the off-diagonal entry is above this level
    // (above the rounding floor of the rotations themselves, about k u ||A||);
    // a sweep that applies none ends the iteration
    const double tiny = 1e-14 * sqrt(fro) + 1e-300;
    int cur = 0, sweeps = 0;
    for (; sweeps < 40; sweeps++) {
        if (tid == 0) nrot = 0;
        __syncthreads();
        for (int r = 0; r < km; r++) {
            // circle-method pairing of round r: the fixed player km meets r, every
            // other x meets (2r - x) mod km
            if (tid < kp / 2) {
                int p, q;
                if (tid == 0) { p = km; q = r; }
                else { p = (r + tid) % km; q = (r - tid + km) % km; }
                if (p > q) { int t = p; p = q; q = t; }
                double c = 1.0, sn = 0.0;
                if (q < k) {
                    double apq = A[cur][p][q];
                    if (fabs(apq) > tiny) {
                        double tau = (A[cur][q][q] - A[cur][p][p]) / (2.0 * apq);
                        double t = (tau >= 0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
                        c = 1.0 / sqrt(1.0 + t * t);
                        sn = t * c;
                        atomicAdd(&nrot, 1);
                    }
                }
                // column p of J is (c at p, -s at q); column q is (s at p, c at q)
                cj[p] = c; sj[p] = -sn;
                cj[q] = c; sj[q] = sn;
            }
            __syncthreads();
            const int nx = cur ^ 1;
            // lanes own columns y, the four waves split the rows x: no integer
            // division in the loop (partner(y) = 2r - y wrapped into [0, km))
            const int y = tid & 63, xg = tid >> 6;
            if (y < k) {
                int yb = (y == km) ? r : (y == r ? km : 2 * r - y);
                if (yb < 0) yb += km;
                else if (yb >= km && y != r) yb -= km;
                const bool ybk = yb < k;
                const double cy = cj[y], sy = sj[y];
                // V' = V J: rows x = xg + 4 it, loads issued before the stores
                double v0[KMAX / 4], v1[KMAX / 4];
#pragma unroll
                for (int it = 0; it < KMAX / 4; it++) {
                    const int x = xg + 4 * it;
                    v0[it] = (x < k) ? V[cur][x][y] : 0.0;
                    v1[it] = (x < k && ybk) ? V[cur][x][yb] : 0.0;
                }
#pragma unroll
                for (int it = 0; it < KMAX / 4; it++) {
                    const int x = xg + 4 * it;
                    if (x < k) V[nx][x][y] = cy * v0[it] + sy * v1[it];
                }
                // A' = J^T A J on the upper triangle (x <= y), mirrored: A stays exactly
                // symmetric (rotations cannot remove an antisymmetric rounding part)
#pragma unroll
                for (int h = 0; h < 2; h++) {
                    double a0[KMAX / 8], a1[KMAX / 8], a2[KMAX / 8], a3[KMAX / 8], cx[KMAX / 8], sx[KMAX / 8];
#pragma unroll
                    for (int it = 0; it < KMAX / 8; it++) {
                        const int x = xg + 4 * (it + h * (KMAX / 8));
                        int xb = (x == km) ? r : (x == r ? km : 2 * r - x);
                        if (xb < 0) xb += km;
                        else if (xb >= km && x != r) xb -= km;
                        const bool ok = x <= y, xbk = ok && xb < k;
                        a0[it] = ok ? A[cur][x][y] : 0.0;
                        a1[it] = (ok && ybk) ? A[cur][x][yb] : 0.0;
                        a2[it] = xbk ? A[cur][xb][y] : 0.0;
                        a3[it] = (xbk && ybk) ? A[cur][xb][yb] : 0.0;
                        cx[it] = ok ? cj[x] : 0.0;
                        sx[it] = ok ? sj[x] : 0.0;
                    }
#pragma unroll
                    for (int it = 0; it < KMAX / 8; it++) {
                        const int x = xg + 4 * (it + h * (KMAX / 8));
                        if (x <= y) {
                            const double v = cx[it] * cy * a0[it] + cx[it] * sy * a1[it] + sx[it] * cy * a2[it] +
                                             sx[it] * sy * a3[it];
                            A[nx][x][y] = v;
                            A[nx][y][x] = v;
                        }
                    }
                }
            }
            cur = nx;
            __syncthreads();
        }
        const int none = (nrot == 0);
        __syncthreads();      // every thread has read nrot before it is reset
        if (none) break;
    }
    // ascending order by rank (ties by index)
    if (tid < k) ev[tid] = A[cur][tid][tid];
    __syncthreads();
    if (tid < k) {
        int rank = 0;
        double v = ev[tid];
        for (int j = 0; j < k; j++) rank += (ev[j] < v) || (ev[j] == v && j < tid);
        perm[rank] = tid;
    }
    if (tid == 0) a.flag[0] = sweeps < 40 ? sweeps + 1 : -1;
    __syncthreads();
    if (tid < k) a.evals_all[tid] = ev[perm[tid]];
    if (tid < m) a.theta[tid] = ev[perm[tid]];
    // C_X = first m sorted eigenvectors
    for (int e = tid; e < k * m; e += 256) {
        int i = e / m, j = e - (e / m) * m;
        a.coef[i * 2 * m + j] = V[cur][i][perm[j]];
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
        for (int t = m; t < k; t++) s += V[cur][t][perm[m + i]] * V[cur][t][perm[j]];
        Z[i][j] = s;
    }
    __syncthreads();
    // modified Gram-Schmidt on the columns of Z, two passes; a vanishing column
    // is replaced by a unit vector
    int next_unit = 0;
    for (int j = 0; j < m; j++) {
        double n0 = 0.0;
        if (tid == 0) {
            for (int i = 0; i < kr; i++) n0 += Z[i][j] * Z[i][j];
            dq[0] = sqrt(n0);
        }
        __syncthreads();
        n0 = dq[0];
        __syncthreads();
        for (int attempt = 0; attempt < 4; attempt++) {
            for (int pass = 0; pass < 2; pass++) {
                if (tid < j) {
                    double d = 0.0;
                    for (int i = 0; i < kr; i++) d += Z[i][tid] * Z[i][j];
                    dq[tid] = d;
                }
                __syncthreads();
                if (tid < kr) {
                    double v = Z[tid][j];
                    for (int q = 0; q < j; q++) v -= dq[q] * Z[tid][q];
                    Z[tid][j] = v;
                }
                __syncthreads();
            }
            __shared__ double nn_s;
            if (tid == 0) {
                double nn = 0.0;
                for (int i = 0; i < kr; i++) nn += Z[i][j] * Z[i][j];
                nn_s = sqrt(nn);
            }
            __syncthreads();
            double nn = nn_s;
            bool ok = nn > 1e-12 * n0 && nn > 1e-300;
            if (tid < kr) Z[tid][j] = ok ? Z[tid][j] / nn : ((tid == (next_unit % kr)) ? 1.0 : 0.0);
            __syncthreads();
            if (ok) break;
            next_unit++;
            n0 = 1.0;
        }
    }
    // C_P = C_rest Z
    for (int e = tid; e < k * m; e += 256) {
        int i = e / m, j = e - (e / m) * m;
        double s = 0.0;
        for (int t = 0; t < kr; t++) s += V[cur][i][perm[m + t]] * Z[t][j];
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
