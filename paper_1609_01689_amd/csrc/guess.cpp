// Multi-level initial guess (Section 3.3.1): the lowest eigenvectors of the
// Hamiltonian restricted to a smaller configuration space, padded with zeros
// (eq. 12), start the solve on the next larger space; applied recursively
// over a sequence of level caps.
#include <algorithm>
#include <cstring>
#include <vector>

#include "hsym_internal.h"

using namespace hsym;

namespace {

template <class F>
int guess_guard(F &&f) {
    try {
        f();
        set_error("");
        return HSYM_OK;
    } catch (Error &e) {
        set_error(e.msg);
        return e.status;
    } catch (std::bad_alloc &) {
        set_error("host allocation failed");
        return HSYM_E_OUT_OF_MEMORY;
    } catch (std::exception &e) {
        set_error(e.what());
        return HSYM_E_DEVICE;
    }
}

struct DevBlock {
    double *p = nullptr;
    ~DevBlock() { if (p) (void)hipFree(p); }
};

// upper CSR of the principal submatrix on the rows with keep[i] (renumbered
// in order); pos[i] is the new index of a kept row
void restrict_upper(int64_t n, const int64_t *rp, const int32_t *ci, const void *vals, int vprec,
                    const std::vector<int64_t> &pos, std::vector<int64_t> &srp, std::vector<int32_t> &sci,
                    std::vector<double> &sv64, std::vector<float> &sv32) {
    srp.assign(1, 0);
    sci.clear(); sv64.clear(); sv32.clear();
    for (int64_t i = 0; i < n; i++) {
        if (pos[(size_t)i] < 0) continue;
        for (int64_t p = rp[i]; p < rp[i + 1]; p++) {
            const int64_t c = ci[p];
            if (c < i || c >= n) fail(HSYM_E_INVALID_ARG, "column outside [row, n) in row " + std::to_string(i));
            if (pos[(size_t)c] < 0) continue;
            sci.push_back((int32_t)pos[(size_t)c]);
            if (vprec == HSYM_FP64) sv64.push_back(((const double *)vals)[p]);
            else sv32.push_back(((const float *)vals)[p]);
        }
        srp.push_back((int64_t)sci.size());
    }
}

}  // namespace

extern "C" int lobpcg_guess_multilevel(int64_t n, const int64_t *rowptr, const int32_t *colind,
                                       const void *values, int values_prec, const int32_t *level, int ncaps,
                                       const int32_t *caps, int storage, int m, double tol, int precond,
                                       const lobpcg_opts *opts, double *X0, int *iters, void *stream) {
    return guess_guard([&] {
        if (!rowptr || !colind || !values || !level || !caps || !X0) fail(HSYM_E_INVALID_ARG, "NULL argument");
        if (n < 1 || n >= ((int64_t)1 << 31)) fail(HSYM_E_INVALID_ARG, "n must be in [1, 2^31)");
        if (ncaps < 1 || ncaps > 16) fail(HSYM_E_INVALID_ARG, "need 1 <= ncaps <= 16");
        if (m < 1 || m > HSYM_MAX_BLOCK) fail(HSYM_E_INVALID_ARG, "block width must be in [1, 16]");
        if (values_prec != HSYM_FP64 && values_prec != HSYM_FP32) fail(HSYM_E_INVALID_ARG, "bad values precision");
        if (precond == HSYM_PRECOND_FOM)
            fail(HSYM_E_INVALID_ARG, "the sub-solves take the none, Jacobi or block64 preconditioner");
        for (int k = 1; k < ncaps; k++)
            if (caps[k] <= caps[k - 1]) fail(HSYM_E_INVALID_ARG, "level caps must be strictly ascending");
        if (rowptr[0] != 0) fail(HSYM_E_INVALID_ARG, "rowptr[0] != 0");
        for (int64_t i = 0; i < n; i++)
            if (rowptr[i + 1] < rowptr[i]) fail(HSYM_E_INVALID_ARG, "rowptr decreases at row " + std::to_string(i));
        hipStream_t s = (hipStream_t)stream;
        const int flags = HSYM_GEOM_M(m) | (precond == HSYM_PRECOND_BLOCK64 ? HSYM_BUILD_BLOCK64 : 0);

        std::vector<int64_t> prev_rows;          // rows of the previous level, in order
        std::vector<double> prev_X;              // its eigenvectors, |prev| x m row-major
        for (int k = 0; k < ncaps; k++) {
            // the smaller configuration space: rows with level <= cap
            std::vector<int64_t> pos((size_t)n, -1), rows;
            for (int64_t i = 0; i < n; i++)
                if (level[i] <= caps[k]) {
                    pos[(size_t)i] = (int64_t)rows.size();
                    rows.push_back(i);
                }
            const int64_t ns = (int64_t)rows.size();
            if (ns < 3 * (int64_t)m)
                fail(HSYM_E_INVALID_ARG, "level cap " + std::to_string(caps[k]) + " keeps fewer than 3m rows");
            std::vector<int64_t> srp;
            std::vector<int32_t> sci;
            std::vector<double> sv64;
            std::vector<float> sv32;
            restrict_upper(n, rowptr, colind, values, values_prec, pos, srp, sci, sv64, sv32);
            hsym_t H = nullptr;
            const void *sv = values_prec == HSYM_FP64 ? (const void *)sv64.data() : (const void *)sv32.data();
            int st = hsym_create(&H, ns, srp.data(), sci.data(), sv, values_prec, storage, flags, stream);
            if (st != HSYM_OK) fail(st, hsym_last_error());
            DevBlock Xs, V;
            try {
                // start: seeded Gaussian (first level) or eq. 12 padding of the previous level
                const double *x0 = nullptr;
                if (!prev_rows.empty()) {
                    std::vector<double> h((size_t)ns * m, 0.0);
                    for (size_t r = 0; r < prev_rows.size(); r++) {
                        const int64_t q = pos[(size_t)prev_rows[r]];
                        if (q < 0) fail(HSYM_E_INVALID_ARG, "level sets are not nested");
                        memcpy(&h[(size_t)q * m], &prev_X[r * m], sizeof(double) * m);
                    }
                    HIPCHK(hipMalloc((void **)&Xs.p, sizeof(double) * h.size()));
                    HIPCHK(hipMemcpy(Xs.p, h.data(), sizeof(double) * h.size(), hipMemcpyHostToDevice));
                    x0 = Xs.p;
                }
                HIPCHK(hipMalloc((void **)&V.p, sizeof(double) * (size_t)ns * m));
                std::vector<double> ev(m);
                lobpcg_report rep;
                st = lobpcg_solve(H, m, m, tol, x0, precond, opts, ev.data(), V.p, &rep, stream);
                if (st != HSYM_OK && st != HSYM_NOT_CONVERGED) fail(st, hsym_last_error());
                if (iters) iters[k] = rep.iters;
                prev_X.assign((size_t)ns * m, 0.0);
                HIPCHK(hipStreamSynchronize(s));
                HIPCHK(hipMemcpy(prev_X.data(), V.p, sizeof(double) * prev_X.size(), hipMemcpyDeviceToHost));
            } catch (...) {
                hsym_destroy(H);
                throw;
            }
            hsym_destroy(H);
            prev_rows.swap(rows);
        }
        // eq. 12 on the full space
        std::vector<double> h((size_t)n * m, 0.0);
        for (size_t r = 0; r < prev_rows.size(); r++)
            memcpy(&h[(size_t)prev_rows[r] * m], &prev_X[r * m], sizeof(double) * m);
        HIPCHK(hipMemcpyAsync(X0, h.data(), sizeof(double) * h.size(), hipMemcpyHostToDevice, s));
        HIPCHK(hipStreamSynchronize(s));
    });
}
