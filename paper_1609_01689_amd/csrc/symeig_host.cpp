// Dense symmetric eigendecomposition on the host, used once per handle to
// factor the 64x64 diagonal blocks of the block-diagonal preconditioner
// (eq. 11 with direct solves): Householder reduction to tridiagonal form,
// then implicit symmetric QR steps with Wilkinson shifts (Golub and Van Loan,
// Matrix Computations, Sections 8.3.1-8.3.3), accumulating every reflection
// and rotation into the eigenvector matrix.
#include <algorithm>
#include <cmath>
#include <numeric>
#include <vector>

namespace hsym {

// Implicit symmetric QR steps with Wilkinson shifts on the tridiagonal matrix
// (d diagonal, e[i] couples i and i+1).  Every rotation is applied to the
// columns of Q (n x n, row-major, leading dimension ldq) when Q != nullptr.
// On return d holds the (unsorted) eigenvalues.
bool tridiag_qr(int n, double *d, double *e, double *Q, int ldq) {
    const double eps = 2.220446049250313e-16;
    int hi = n - 1, guard = 0;
    while (hi > 0) {
        if (std::fabs(e[hi - 1]) <= eps * (std::fabs(d[hi - 1]) + std::fabs(d[hi]))) {
            e[hi - 1] = 0.0;
            hi--;
            continue;
        }
        if (++guard > 60 * n) return false;
        int lo = hi - 1;
        while (lo > 0 && std::fabs(e[lo - 1]) > eps * (std::fabs(d[lo - 1]) + std::fabs(d[lo]))) lo--;
        // Wilkinson shift from the trailing 2x2 block
        double t = 0.5 * (d[hi - 1] - d[hi]);
        double b2 = e[hi - 1] * e[hi - 1];
        double den = t + (t >= 0 ? 1.0 : -1.0) * std::sqrt(t * t + b2);
        double mu = d[hi] - (den != 0.0 ? b2 / den : 0.0);
        double x = d[lo] - mu, z = e[lo], bulge = 0.0;
        for (int k = lo; k < hi; k++) {
            double r = std::hypot(x, z);
            double c = r == 0.0 ? 1.0 : x / r, s = r == 0.0 ? 0.0 : -z / r;
            if (k > lo) e[k - 1] = r;
            double a = d[k], bb = e[k], dd = d[k + 1];
            d[k] = c * c * a - 2.0 * c * s * bb + s * s * dd;
            d[k + 1] = s * s * a + 2.0 * c * s * bb + c * c * dd;
            e[k] = c * s * (a - dd) + (c * c - s * s) * bb;
            if (k + 1 < hi) {
                bulge = -s * e[k + 1];
                e[k + 1] = c * e[k + 1];
            }
            if (Q)
                for (int rr = 0; rr < n; rr++) {
                    double *row = Q + (size_t)rr * ldq;
                    double qk = row[k], qk1 = row[k + 1];
                    row[k] = c * qk - s * qk1;
                    row[k + 1] = s * qk + c * qk1;
                }
            x = e[k];
            z = bulge;
        }
    }
    return true;
}

// A: n x n row-major symmetric (upper and lower both filled).  On return the
// columns of A are orthonormal eigenvectors and w the ascending eigenvalues.
// Returns false if the QR iteration did not converge.
bool sym_eig_host(int n, double *A, double *w) {
    std::vector<double> Q((size_t)n * n, 0.0), v(n), p(n), q(n);
    for (int i = 0; i < n; i++) Q[(size_t)i * n + i] = 1.0;
    // Householder tridiagonalisation: column k below the subdiagonal is zeroed
    for (int k = 0; k + 2 < n; k++) {
        double nrm = 0.0;
        for (int i = k + 1; i < n; i++) nrm += A[(size_t)i * n + k] * A[(size_t)i * n + k];
        nrm = std::sqrt(nrm);
        if (nrm == 0.0) continue;
        double x0 = A[(size_t)(k + 1) * n + k];
        double alpha = x0 >= 0 ? -nrm : nrm;
        int len = n - k - 1;
        for (int i = 0; i < len; i++) v[i] = A[(size_t)(k + 1 + i) * n + k];
        v[0] -= alpha;
        double vn = 0.0;
        for (int i = 0; i < len; i++) vn += v[i] * v[i];
        vn = std::sqrt(vn);
        if (vn == 0.0) continue;
        for (int i = 0; i < len; i++) v[i] /= vn;
        // trailing block B = A[k+1:, k+1:]; p = B v, K = v'p, q = p - K v, B -= 2(v q' + q v')
        for (int i = 0; i < len; i++) {
            double s = 0.0;
            const double *row = A + (size_t)(k + 1 + i) * n + (k + 1);
            for (int j = 0; j < len; j++) s += row[j] * v[j];
            p[i] = s;
        }
        double K = 0.0;
        for (int i = 0; i < len; i++) K += v[i] * p[i];
        for (int i = 0; i < len; i++) q[i] = p[i] - K * v[i];
        for (int i = 0; i < len; i++) {
            double *row = A + (size_t)(k + 1 + i) * n + (k + 1);
            for (int j = 0; j < len; j++) row[j] -= 2.0 * (v[i] * q[j] + q[i] * v[j]);
        }
        A[(size_t)(k + 1) * n + k] = A[(size_t)k * n + (k + 1)] = alpha;
        for (int i = k + 2; i < n; i++) A[(size_t)i * n + k] = A[(size_t)k * n + i] = 0.0;
        // Q <- Q (I - 2 v v') on columns k+1..n-1
        for (int r = 0; r < n; r++) {
            double *row = Q.data() + (size_t)r * n + (k + 1);
            double s = 0.0;
            for (int j = 0; j < len; j++) s += row[j] * v[j];
            s *= 2.0;
            for (int j = 0; j < len; j++) row[j] -= s * v[j];
        }
    }
    std::vector<double> d(n), e(std::max(n, 1), 0.0);
    for (int i = 0; i < n; i++) d[i] = A[(size_t)i * n + i];
    for (int i = 0; i + 1 < n; i++) e[i] = A[(size_t)i * n + i + 1];
    if (!tridiag_qr(n, d.data(), e.data(), Q.data(), n)) return false;
    std::vector<int> idx(n);
    std::iota(idx.begin(), idx.end(), 0);
    std::sort(idx.begin(), idx.end(), [&](int a, int b) { return d[a] < d[b]; });
    for (int j = 0; j < n; j++) {
        w[j] = d[idx[j]];
        for (int i = 0; i < n; i++) A[(size_t)i * n + j] = Q[(size_t)i * n + idx[j]];
    }
    return true;
}

}  // namespace hsym
