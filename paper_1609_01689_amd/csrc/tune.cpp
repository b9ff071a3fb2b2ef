// Tile-shape autotuner: time the SpMM of a row sample of H under each panel
// geometry that fits the LDS at the requested block width, keep the fastest.
#include <algorithm>
#include <cstring>
#include <vector>

#include "hsym_internal.h"

using namespace hsym;

namespace {

// Rows [a, a + k) of the stored triangle as a k x k matrix: entries whose
// column leaves the window are dropped.
struct Sample {
    std::vector<int64_t> rp;
    std::vector<int32_t> ci;
    std::vector<double> v64;
    std::vector<float> v32;
};

Sample take_sample(int64_t a, int64_t k, const int64_t *rowptr, const int32_t *colind, const void *values,
                   int vprec) {
    Sample S;
    S.rp.assign((size_t)k + 1, 0);
    for (int64_t i = 0; i < k; i++) {
        const int64_t row = a + i;
        for (int64_t p = rowptr[row]; p < rowptr[row + 1]; p++) {
            const int64_t c = colind[p];
            if (c < row) fail(HSYM_E_INVALID_ARG, "column " + std::to_string(c) + " below the diagonal in row " +
                                                      std::to_string(row));
            if (c >= a + k) continue;
            S.ci.push_back((int32_t)(c - a));
            if (vprec == HSYM_FP64) S.v64.push_back(((const double *)values)[p]);
            else S.v32.push_back(((const float *)values)[p]);
        }
        S.rp[(size_t)i + 1] = (int64_t)S.ci.size();
    }
    return S;
}

struct DevBuf {
    void *p = nullptr;
    ~DevBuf() { if (p) (void)hipFree(p); }
};

struct Handle {
    hsym_t h = nullptr;
    ~Handle() { if (h) (void)hsym_destroy(h); }
};

struct Stream {
    hipStream_t s = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    ~Stream() {
        if (e0) (void)hipEventDestroy(e0);
        if (e1) (void)hipEventDestroy(e1);
        if (s) (void)hipStreamDestroy(s);
    }
};

template <class F>
int tune_guard(F &&f) {
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

}  // namespace

extern "C" int hsym_autotune_geometry(int64_t n, const int64_t *rowptr, const int32_t *colind, const void *values,
                                      int values_prec, int storage, int m, int64_t sample_rows, int *out_flags,
                                      hsym_tune_entry *table, int cap, int *ntried) {
    if (out_flags) *out_flags = 0;
    if (ntried) *ntried = 0;
    return tune_guard([&] {
    if (!rowptr || !colind || !values || !out_flags) fail(HSYM_E_INVALID_ARG, "NULL argument");
    if (n < 1 || n >= ((int64_t)1 << 31)) fail(HSYM_E_INVALID_ARG, "n must be in [1, 2^31)");
    if (m < 1 || m > HSYM_MAX_BLOCK) fail(HSYM_E_INVALID_ARG, "block width must be in [1, 16]");
    if (values_prec != HSYM_FP64 && values_prec != HSYM_FP32) fail(HSYM_E_INVALID_ARG, "bad values precision");
    if (storage != HSYM_FP64 && storage != HSYM_FP32) fail(HSYM_E_INVALID_ARG, "bad storage precision");
    if (rowptr[0] != 0) fail(HSYM_E_INVALID_ARG, "rowptr[0] != 0");
    for (int64_t i = 0; i < n; i++)
        if (rowptr[i + 1] < rowptr[i]) fail(HSYM_E_INVALID_ARG, "rowptr decreases at row " + std::to_string(i));
    const int64_t k = std::min<int64_t>(n, sample_rows > 0 ? sample_rows : 262144);
    const int64_t a = (n - k) / 2;
    Sample S = take_sample(a, k, rowptr, colind, values, values_prec);
    const void *sv = values_prec == HSYM_FP64 ? (const void *)S.v64.data() : (const void *)S.v32.data();

    Stream st;
    HIPCHK(hipStreamCreate(&st.s));
    HIPCHK(hipEventCreate(&st.e0));
    HIPCHK(hipEventCreate(&st.e1));
    DevBuf X, Y;
    HIPCHK(hipMalloc(&X.p, (size_t)k * m * sizeof(double)));
    HIPCHK(hipMalloc(&Y.p, (size_t)k * m * sizeof(double)));
    // the SpMM's time does not depend on the values of X
    HIPCHK(hipMemsetAsync(X.p, 0, (size_t)k * m * sizeof(double), st.s));

    double best = -1.0;
    int used = 0;
    // candidates: panel rows a multiple of 64 from 256 to 2048, chunks of
    // 64 or 128 columns dividing them, those that fit the LDS at width m
    for (int r64 = 4; r64 <= 32; r64 += (r64 < 8 ? 1 : r64 < 16 ? 2 : 4)) {
        for (int lc = 6; lc <= 7; lc++) {
            const int R = 64 * r64, C = 1 << lc;
            if (R % C) continue;
            Geom gt;
            try {
                gt = geometry_for(storage, m, k, r64, lc);
            } catch (Error &) {
                continue;
            }
            if (spmm_lds_bytes(storage, m, gt) > 160 * 1024) continue;
            const int flags = HSYM_GEOM_M(m) | HSYM_GEOM_PANEL(r64, lc);
            double ms = -1.0;
            Handle hg;   // destroyed on every path, errors included
            int rc = hsym_create(&hg.h, k, S.rp.data(), S.ci.data(), sv, values_prec, storage, flags, st.s);
            hsym_t H = hg.h;
            if (rc == HSYM_OK) {
                for (int w = 0; w < 3 && rc == HSYM_OK; w++)
                    rc = spmm_sym(H, m, (const double *)X.p, m, (double *)Y.p, m, st.s);
                if (rc == HSYM_OK) {
                    HIPCHK(hipEventRecord(st.e0, st.s));
                    for (int t = 0; t < 5 && rc == HSYM_OK; t++)
                        rc = spmm_sym(H, m, (const double *)X.p, m, (double *)Y.p, m, st.s);
                    HIPCHK(hipEventRecord(st.e1, st.s));
                    HIPCHK(hipEventSynchronize(st.e1));
                    float f = 0.0f;
                    HIPCHK(hipEventElapsedTime(&f, st.e0, st.e1));
                    if (rc == HSYM_OK) ms = f / 5.0;
                }
            }
            // a geometry the device cannot hold (memory) is skipped, not fatal
            if (rc == HSYM_E_DEVICE) fail(rc, std::string("autotune: ") + hsym_last_error());
            if (table && used < cap) table[used] = hsym_tune_entry{R, C, ms};
            used++;
            if (ms > 0.0 && (best < 0.0 || ms < best)) {
                best = ms;
                *out_flags = flags;
            }
        }
    }
    if (ntried) *ntried = used;
    if (best < 0.0) fail(HSYM_E_UNSUPPORTED, "no panel geometry could be timed at this block width");
    });
}
