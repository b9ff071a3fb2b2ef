// Single-vector Lanczos with full re-orthogonalisation: the eigensolver the
// paper replaces (Section 3, opening paragraph; MFDn's Lanczos keeps every
// basis vector and re-orthogonalises against all of them).  The three-term
// recurrence, the re-orthogonalisation (classical Gram-Schmidt applied twice)
// and the SpMV run on the GPU; the tridiagonal Ritz problem is solved on the
// host at the checks of Section 5.2, footnote 7 (every 10 iterations up to
// 100, then every 20 up to 200, every 40 up to 400, ...).
#include <chrono>
#include <cmath>
#include <cstring>
#include <numeric>

#include "dense.h"

namespace hsym {

bool tridiag_qr(int n, double *d, double *e, double *Q, int ldq);

static int check_interval(int j) {
    int iv = 10, lim = 100;
    while (j > lim) { iv *= 2; lim *= 2; }
    return iv;
}

// eigenvector of the tridiagonal (d, e) for eigenvalue theta by inverse
// iteration with a partially pivoted LU; orthogonalised against `prev`
static void tridiag_inverse_iteration(int k, const double *d, const double *e, double theta, double tnorm,
                                      const std::vector<std::vector<double>> &prev, std::vector<double> &y) {
    std::vector<double> dl(k), dd(k), du(k), du2(k), b(k);
    std::vector<int> piv(k);
    const double tiny = 1e-300 + 2.2e-16 * tnorm;
    double sigma = theta + 1e-14 * tnorm;   // keep T - sigma I away from exact singularity
    for (int i = 0; i < k; i++) {
        dd[i] = d[i] - sigma;
        du[i] = i + 1 < k ? e[i] : 0.0;
        dl[i] = i + 1 < k ? e[i] : 0.0;
        du2[i] = 0.0;
    }
    for (int i = 0; i + 1 < k; i++) {
        if (std::fabs(dd[i]) >= std::fabs(dl[i])) {
            if (dd[i] == 0.0) dd[i] = tiny;
            double l = dl[i] / dd[i];
            dl[i] = l;
            dd[i + 1] -= l * du[i];
            piv[i] = i;
        } else {
            double l = dd[i] / dl[i];
            double ddn = dd[i + 1], dun = (i + 2 < k) ? du[i + 1] : 0.0, dui = du[i];
            dd[i] = dl[i];
            dl[i] = l;
            du[i] = ddn;
            du2[i] = dun;
            dd[i + 1] = dui - l * ddn;
            if (i + 2 < k) du[i + 1] = -l * dun;
            piv[i] = i + 1;
        }
    }
    if (dd[k - 1] == 0.0) dd[k - 1] = tiny;
    y.assign(k, 1.0 / std::sqrt((double)k));
    for (int it = 0; it < 4; it++) {
        b = y;
        for (int i = 0; i + 1 < k; i++) {
            if (piv[i] != i) std::swap(b[i], b[i + 1]);
            b[i + 1] -= dl[i] * b[i];
        }
        y[k - 1] = b[k - 1] / dd[k - 1];
        if (k > 1) y[k - 2] = (b[k - 2] - du[k - 2] * y[k - 1]) / dd[k - 2];
        for (int i = k - 3; i >= 0; i--) y[i] = (b[i] - du[i] * y[i + 1] - du2[i] * y[i + 2]) / dd[i];
        for (int pass = 0; pass < 2; pass++)
            for (const auto &q : prev) {
                double dot = 0.0;
                for (int i = 0; i < k; i++) dot += q[i] * y[i];
                for (int i = 0; i < k; i++) y[i] -= dot * q[i];
            }
        double nrm = 0.0;
        for (double v : y) nrm += v * v;
        nrm = std::sqrt(nrm);
        if (!(nrm > 0.0)) { y.assign(k, 0.0); y[it % k] = 1.0; continue; }
        for (double &v : y) v /= nrm;
    }
}

__global__ void k_vts(const double *__restrict__ V, int64_t n, int k, const double *__restrict__ S, int nev,
                      double *__restrict__ out) {
    int64_t r = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (r >= n) return;
    double acc[HSYM_MAX_BLOCK];
    for (int c = 0; c < nev; c++) acc[c] = 0.0;
    for (int i = 0; i < k; i++) {
        double v = V[(int64_t)i * n + r];
        for (int c = 0; c < nev; c++) acc[c] = fma(v, S[i * nev + c], acc[c]);
    }
    for (int c = 0; c < nev; c++) out[r * nev + c] = acc[c];
}

__global__ void k_axpy_dev(double *__restrict__ w, const double *__restrict__ v, const double *__restrict__ coef,
                           int64_t n) {
    int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i < n) w[i] -= coef[0] * v[i];
}

__global__ void k_sqrt_to(const double *__restrict__ x, double *__restrict__ y) { y[0] = sqrt(x[0]); }

}  // namespace hsym

using namespace hsym;

extern "C" int lanczos_solve(hsym_t H, int nev, double tol, const double *v0, const lanczos_opts *opts,
                             double *evals, double *evecs, lanczos_report *rep, void *stream) {
    std::vector<void *> allocs;
    std::vector<hipEvent_t> evs;
    auto cleanup = [&] {
        for (void *p : allocs) (void)hipFree(p);
        for (auto e : evs) (void)hipEventDestroy(e);
    };
    try {
        if (!H || !H->ready) fail(HSYM_E_INVALID_ARG, "invalid handle");
        if (nev < 1 || nev > HSYM_MAX_BLOCK || nev > H->n) fail(HSYM_E_INVALID_ARG, "need 1 <= nev <= min(16, n)");
        if (!(tol > 0.0)) fail(HSYM_E_INVALID_ARG, "tol must be > 0");
        if (!evals) fail(HSYM_E_INVALID_ARG, "NULL evals");
        hipStream_t s = (hipStream_t)stream;
        const int64_t n = H->n;
        int maxit = (opts && opts->maxit > 0) ? opts->maxit : 2000;
        uint64_t seed = opts ? opts->seed : 0;
        const int kmax = (int)std::min<int64_t>(maxit, n);
        auto dal = [&](size_t b) {
            void *p = nullptr;
            if (hipMalloc(&p, std::max<size_t>(b, 256)) != hipSuccess) {
                (void)hipGetLastError();
                fail(HSYM_E_OUT_OF_MEMORY, "Lanczos allocation of " + std::to_string(b) + " bytes");
            }
            allocs.push_back(p);
            return p;
        };
        double *V = (double *)dal(sizeof(double) * (size_t)(kmax + 1) * n);
        double *w = (double *)dal(sizeof(double) * n);
        double *h = (double *)dal(sizeof(double) * (kmax + 1));
        double *dscr = (double *)dal(dots_scratch_bytes(n, kmax + 1));
        double *alpha = (double *)dal(sizeof(double) * (kmax + 1));
        double *beta2 = (double *)dal(sizeof(double) * (kmax + 1));   // squared norms
        double *beta = (double *)dal(sizeof(double) * (kmax + 1));
        const unsigned gb = (unsigned)((n + 255) / 256);
        auto t0 = std::chrono::steady_clock::now();
        // v_1 = v0 / ||v0||
        if (v0) HIPCHK(hipMemcpyAsync(w, v0, sizeof(double) * n, hipMemcpyDeviceToDevice, s));
        else gauss_fill(w, n, 1, 1, seed, 9, -1, s);
        dots(w, n, 1, w, n, beta2, dscr, s);
        scale_to(w, beta2, V, n, s);
        const int NEV = 512;
        for (int i = 0; i < 2 * NEV; i++) {
            hipEvent_t e;
            HIPCHK(hipEventCreate(&e));
            evs.push_back(e);
        }
        int nev_rec = 0;
        double spmv_ms = 0.0;
        std::vector<double> ha, hb;
        std::vector<double> theta;
        std::vector<std::vector<double>> S;
        bool conv = false;
        int j = 0;
        double normH = H->norm1;
        for (j = 1; j <= kmax; j++) {
            double *vj = V + (int64_t)(j - 1) * n;
            if (nev_rec < NEV) HIPCHK(hipEventRecord(evs[2 * nev_rec], s));
            spmm_launch(H, 1, vj, T_F64, 1, w, T_F64, 1, s);
            if (nev_rec < NEV) { HIPCHK(hipEventRecord(evs[2 * nev_rec + 1], s)); nev_rec++; }
            if (j > 1) {
                hipLaunchKernelGGL(k_axpy_dev, dim3(gb), dim3(256), 0, s, w, vj - n, beta + (j - 2), n);
                HIPCHK(hipGetLastError());
            }
            dots(vj, n, 1, w, n, alpha + (j - 1), dscr, s);
            hipLaunchKernelGGL(k_axpy_dev, dim3(gb), dim3(256), 0, s, w, vj, alpha + (j - 1), n);
            HIPCHK(hipGetLastError());
            for (int pass = 0; pass < 2; pass++) {
                dots(V, n, j, w, n, h, dscr, s);
                sub_vh(V, n, h, j, w, n, s);
            }
            dots(w, n, 1, w, n, beta2 + (j - 1), dscr, s);
            hipLaunchKernelGGL(k_sqrt_to, dim3(1), dim3(1), 0, s, beta2 + (j - 1), beta + (j - 1));
            HIPCHK(hipGetLastError());
            scale_to(w, beta2 + (j - 1), V + (int64_t)j * n, n, s);
            if (j % check_interval(j) != 0 && j != kmax) continue;
            // check: Ritz values of T_j and residuals beta_j |s_{j,i}|
            ha.resize(j);
            hb.resize(j);
            HIPCHK(hipMemcpyAsync(ha.data(), alpha, sizeof(double) * j, hipMemcpyDeviceToHost, s));
            HIPCHK(hipMemcpyAsync(hb.data(), beta, sizeof(double) * j, hipMemcpyDeviceToHost, s));
            HIPCHK(hipStreamSynchronize(s));
            for (int q = 0; q < nev_rec; q++) {
                float ms = 0.f;
                HIPCHK(hipEventElapsedTime(&ms, evs[2 * q], evs[2 * q + 1]));
                spmv_ms += ms;
            }
            nev_rec = 0;
            int kk = j;
            bool invariant = false;
            for (int i = 0; i < j; i++)
                if (!std::isfinite(ha[i]) || !std::isfinite(hb[i])) fail(HSYM_E_NUMERIC, "NaN/Inf in Lanczos");
            for (int i = 0; i < j; i++)
                if (hb[i] < 1e-14 * normH) { kk = i + 1; invariant = true; break; }
            std::vector<double> d(ha.begin(), ha.begin() + kk), e(kk, 0.0);
            for (int i = 0; i + 1 < kk; i++) e[i] = hb[i];
            std::vector<double> dcopy = d, ecopy = e;
            if (!tridiag_qr(kk, dcopy.data(), ecopy.data(), nullptr, 0))
                fail(HSYM_E_NUMERIC, "tridiagonal QR did not converge");
            std::sort(dcopy.begin(), dcopy.end());
            int want = std::min(nev, kk);
            double tnorm = 0.0;
            for (int i = 0; i < kk; i++)
                tnorm = std::max(tnorm, std::fabs(d[i]) + (i ? std::fabs(e[i - 1]) : 0.0) + std::fabs(e[i]));
            theta.assign(dcopy.begin(), dcopy.begin() + want);
            S.clear();
            bool all = want == nev;
            std::vector<double> res(want);
            for (int i = 0; i < want; i++) {
                std::vector<std::vector<double>> prev;
                for (int q = 0; q < i; q++)
                    if (std::fabs(theta[q] - theta[i]) < 1e-8 * tnorm) prev.push_back(S[q]);
                std::vector<double> y;
                tridiag_inverse_iteration(kk, d.data(), e.data(), theta[i], tnorm, prev, y);
                S.push_back(y);
                res[i] = hb[kk - 1] * std::fabs(y[kk - 1]);
                if (!(res[i] <= tol * normH)) all = false;
            }
            if (rep) {
                rep->iters = j;
                for (int i = 0; i < want; i++) rep->resnorm[i] = res[i] / normH;
            }
            if (all || invariant || j == kmax) {
                conv = all;
                j = kk;
                break;
            }
        }
        if (j > kmax) j = kmax;
        for (int i = 0; i < (int)theta.size() && i < nev; i++) evals[i] = theta[i];
        for (int i = (int)theta.size(); i < nev; i++) evals[i] = NAN;
        if (evecs && (int)S.size() == nev) {
            int k = (int)S[0].size();
            std::vector<double> Sh((size_t)k * nev);
            for (int i = 0; i < k; i++)
                for (int c = 0; c < nev; c++) Sh[(size_t)i * nev + c] = S[c][i];
            double *Sd = (double *)dal(sizeof(double) * Sh.size());
            double *tmp = (double *)dal(sizeof(double) * (size_t)n * nev);
            double *scr = (double *)dal(sign_fix_scratch_bytes(n, nev));
            HIPCHK(hipMemcpyAsync(Sd, Sh.data(), sizeof(double) * Sh.size(), hipMemcpyHostToDevice, s));
            hipLaunchKernelGGL(k_vts, dim3(gb), dim3(256), 0, s, V, n, k, Sd, nev, tmp);
            HIPCHK(hipGetLastError());
            sign_fix_copy(tmp, nev, nev, n, evecs, scr, s);
        }
        HIPCHK(hipStreamSynchronize(s));
        if (rep) {
            rep->iters = j;
            rep->converged = conv ? 1 : 0;
            rep->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
            rep->spmv_ms = spmv_ms;
            rep->orth_ms = 0.0;
        }
        cleanup();
        set_error("");
        return conv ? HSYM_OK : HSYM_NOT_CONVERGED;
    } catch (Error &e) {
        cleanup();
        set_error(e.msg);
        return e.status;
    } catch (std::bad_alloc &) {
        cleanup();
        set_error("host allocation failed");
        return HSYM_E_OUT_OF_MEMORY;
    }
}
