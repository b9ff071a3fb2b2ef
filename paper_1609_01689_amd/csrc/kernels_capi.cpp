// Step-level C ABI (include/hsym_kernels.h): thin wrappers over the kernels
// the solver uses, with per-call scratch.
#include <cstring>

#include "../../include/hsym_kernels.h"
#include "dense.h"

using namespace hsym;

namespace {

struct DevBuf {
    void *p = nullptr;
    explicit DevBuf(size_t b) {
        if (hipMalloc(&p, std::max<size_t>(b, 256)) != hipSuccess) {
            (void)hipGetLastError();
            p = nullptr;
            fail(HSYM_E_OUT_OF_MEMORY, "scratch allocation");
        }
    }
    ~DevBuf() { if (p) (void)hipFree(p); }
};

template <class F>
int guarded(F &&f) {
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
    }
}

void check_nm(int64_t n, int m) {
    if (n < 1 || m < 1 || m > HSYM_MAX_BLOCK) fail(HSYM_E_INVALID_ARG, "need n >= 1 and 1 <= m <= 16");
}

}  // namespace

extern "C" {

int hsym_kernel_gram(int64_t n, int m, int na, const double *const *A, int nb, const double *const *B, double *G,
                     void *stream) {
    return guarded([&] {
        check_nm(n, m);
        if (na < 1 || na > 3 || nb < 1 || nb > 6 || !A || !B || !G) fail(HSYM_E_INVALID_ARG, "bad gram arguments");
        hipStream_t s = (hipStream_t)stream;
        GramArgs g{};
        for (int i = 0; i < na; i++) g.a[i] = A[i];
        for (int i = 0; i < nb; i++) g.b[i] = B[i];
        g.na = na; g.nb = nb; g.m = m; g.n = n;
        DevBuf scr(gram_scratch_bytes(n, na * m, nb * m));
        gram(g, G, (double *)scr.p, s);
        HIPCHK(hipStreamSynchronize(s));
    });
}

int hsym_kernel_lincomb(int64_t n, int m, int nin, const double *const *In, int nout, double *const *Out,
                        const double *C, int ldc, void *stream) {
    return guarded([&] {
        check_nm(n, m);
        if (nin < 1 || nin > 3 || nout < 1 || nout > 2 || !In || !Out || !C || ldc < nout * m)
            fail(HSYM_E_INVALID_ARG, "bad lincomb arguments");
        LincombArgs l{};
        for (int i = 0; i < nin; i++) l.in[i] = In[i];
        for (int i = 0; i < nout; i++) l.out[i] = Out[i];
        l.coef = C; l.ldc = ldc; l.nin = nin; l.nout = nout; l.nsets = 1; l.m = m; l.n = n;
        lincomb(l, (hipStream_t)stream);
    });
}

int hsym_kernel_rayleigh_ritz(int nblk, int m, const double *G, double *theta, double *evals, double *coef,
                              int *p_dropped, void *stream) {
    return guarded([&] {
        if (nblk < 1 || nblk > 3 || m < 1 || m > HSYM_MAX_BLOCK || !G || !theta || !evals || !coef)
            fail(HSYM_E_INVALID_ARG, "bad Rayleigh-Ritz arguments");
        hipStream_t s = (hipStream_t)stream;
        DevBuf flag(2 * sizeof(int));
        RRArgs r{};
        r.gram = G; r.coef = coef; r.theta = theta; r.evals_all = evals; r.flag = (int *)flag.p;
        r.nblk = nblk; r.m = m;
        small_rr(&r, 1, s);
        int f[2] = {0, 0};
        HIPCHK(hipMemcpyAsync(f, flag.p, 2 * sizeof(int), hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        if (f[0] < 0) fail(HSYM_E_NUMERIC, "Rayleigh-Ritz eigensolver broke down (non-finite inverse iterate)");
        if (p_dropped) *p_dropped = f[1];
    });
}

int hsym_kernel_precond(hsym_t H, int kind, int m, double *W, const double *mu, double delta, void *stream) {
    return guarded([&] {
        if (!H || !H->ready) fail(HSYM_E_INVALID_ARG, "invalid handle");
        check_nm(H->n, m);
        if (!W || !mu) fail(HSYM_E_INVALID_ARG, "NULL block");
        if (kind != HSYM_PRECOND_JACOBI && kind != HSYM_PRECOND_BLOCK64 && kind != HSYM_PRECOND_FOM)
            fail(HSYM_E_INVALID_ARG, "bad kind");
        if (kind == HSYM_PRECOND_BLOCK64 && !H->pre_q) fail(HSYM_E_INVALID_ARG, "block64 factors not built");
        precond_apply(H, kind, W, mu, delta, m, (hipStream_t)stream);
    });
}

int hsym_kernel_orthonormalize(int64_t n, int m, double *V, int nb, const double *const *B, uint64_t seed,
                               int *replaced, void *stream) {
    return guarded([&] {
        check_nm(n, m);
        if (nb < 0 || nb > 2 || !V || (nb > 0 && !B)) fail(HSYM_E_INVALID_ARG, "bad orthonormalize arguments");
        if ((int64_t)(nb + 1) * m > n) fail(HSYM_E_INVALID_ARG, "more columns than rows");
        hipStream_t s = (hipStream_t)stream;
        DevBuf g(48 * 48 * 8), c(48 * 32 * 8), scr(gram_scratch_bytes(n, 3 * m, m)), fl(sizeof(int));
        int *fh = nullptr;
        HIPCHK(hipHostMalloc((void **)&fh, sizeof(int), hipHostMallocDefault));
        OrthWork w{(double *)g.p, (double *)c.p, (double *)scr.p, (int *)fl.p, fh};
        int r = 0;
        try {
            r = orthonormalize_block(n, m, V, B, nb, seed, w, s);
            HIPCHK(hipStreamSynchronize(s));
        } catch (...) {
            (void)hipHostFree(fh);
            throw;
        }
        (void)hipHostFree(fh);
        if (replaced) *replaced = r;
    });
}

}  // extern "C"
