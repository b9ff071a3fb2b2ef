// C ABI entry points: argument checks, error capture, handle lifetime.
#include <algorithm>
#include <cstring>
#include <mutex>

#include <vector>

#include "hsym_internal.h"

namespace hsym {

static thread_local std::string g_last_error;

void set_error(const std::string &msg) { g_last_error = msg; }


void fail(int status, const std::string &msg) { throw Error{status, msg}; }

void check_hip(hipError_t e, const char *what) {
    if (e == hipSuccess) return;
    (void)hipGetLastError();
    int st = (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation) ? HSYM_E_OUT_OF_MEMORY : HSYM_E_DEVICE;
    fail(st, std::string(what) + ": " + hipGetErrorString(e));
}

Scratch::~Scratch() { if (p) (void)hipFree(p); }

void *Scratch::get(size_t b) {
    if (b <= bytes && p) return p;
    if (p) { (void)hipFree(p); p = nullptr; bytes = 0; }
    if (hipMalloc(&p, std::max<size_t>(b, 256)) != hipSuccess) {
        (void)hipGetLastError();
        p = nullptr;
        fail(HSYM_E_OUT_OF_MEMORY, "scratch allocation of " + std::to_string(b) + " bytes");
    }
    bytes = b;
    return p;
}

void builder_begin(hsym_matrix *H, int64_t nnz_hint);
void builder_append(hsym_matrix *H, int64_t nrows, const int64_t *rp, const int32_t *ci, const void *vals,
                    int vprec);
void builder_finish(hsym_matrix *H);
void builder_discard(hsym_matrix *H);

}  // namespace hsym

using namespace hsym;

#define API_BEGIN try {
#define API_END                                              \
    }                                                        \
    catch (Error & e) {                                      \
        set_error(e.msg);                                    \
        return e.status;                                     \
    }                                                        \
    catch (std::bad_alloc &) {                               \
        set_error("host allocation failed");                 \
        return HSYM_E_OUT_OF_MEMORY;                         \
    }                                                        \
    catch (std::exception & e) {                             \
        set_error(e.what());                                 \
        return HSYM_E_DEVICE;                                \
    }                                                        \
    set_error("");                                           \
    return HSYM_OK;

static void destroy_matrix(hsym_matrix *H) {
    if (!H) return;
    builder_discard(H);
    free_tiles(&H->tiles);
    if (H->diag64) (void)hipFree(H->diag64);
    if (H->diag32) (void)hipFree(H->diag32);
    if (H->pre_q) (void)hipFree(H->pre_q);
    if (H->pre_lam) (void)hipFree(H->pre_lam);
    if (H->tg_start) (void)hipFree(H->tg_start);
    if (H->tg_off) (void)hipFree(H->tg_off);
    if (H->tg_dense) (void)hipFree(H->tg_dense);
    delete H;
}

extern "C" {

const char *hsym_last_error(void) { return g_last_error.c_str(); }

static int geom_from_flags(int flags) {
    int g = (flags >> 8) & 0xff;
    return g ? g : 16;
}

int hsym_create_begin(hsym_t *out, int64_t n, int storage, int flags, void *stream) {
    if (out) *out = nullptr;
    hsym_matrix *H = nullptr;
    API_BEGIN
    if (flags & HSYM_DEVICE_PTRS) fail(HSYM_E_INVALID_ARG, "the streaming create takes host arrays");
    if (!out) fail(HSYM_E_INVALID_ARG, "NULL handle pointer");
    if (n < 1 || n >= ((int64_t)1 << 31)) fail(HSYM_E_INVALID_ARG, "n must be in [1, 2^31)");
    if (storage != HSYM_FP64 && storage != HSYM_FP32) fail(HSYM_E_INVALID_ARG, "storage must be HSYM_FP64 or HSYM_FP32");
    H = new hsym_matrix();
    H->n = n;
    H->storage = storage;
    H->flags = flags;
    H->geom_m = geom_from_flags(flags);
    H->geom_r64 = (flags >> 16) & 0xff;
    H->geom_lc = (flags >> 24) & 0xf;
    if (H->geom_r64 && !H->geom_lc) fail(HSYM_E_INVALID_ARG, "explicit panel geometry needs the chunk exponent");
    H->stream = (hipStream_t)stream;
    HIPCHK(hipGetDevice(&H->device));
    try {
        builder_begin(H, 0);
    } catch (...) {
        destroy_matrix(H);
        throw;
    }
    *out = H;
    API_END
}

int hsym_create_append(hsym_t H, int64_t nrows, const int64_t *rowptr_local, const int32_t *colind,
                       const void *values, int values_prec) {
    API_BEGIN
    if (!H) fail(HSYM_E_INVALID_ARG, "NULL handle");
    if (values_prec != HSYM_FP64 && values_prec != HSYM_FP32) fail(HSYM_E_INVALID_ARG, "bad values precision");
    try {
        builder_append(H, nrows, rowptr_local, colind, values, values_prec);
    } catch (...) {
        destroy_matrix(H);
        throw;
    }
    API_END
}

int hsym_create_finish(hsym_t H) {
    API_BEGIN
    if (!H) fail(HSYM_E_INVALID_ARG, "NULL handle");
    try {
        builder_finish(H);
    } catch (...) {
        destroy_matrix(H);
        throw;
    }
    API_END
}

int hsym_create(hsym_t *out, int64_t n, const int64_t *rowptr, const int32_t *colind, const void *values,
                int values_prec, int storage, int flags, void *stream) {
    if (out) *out = nullptr;
    API_BEGIN
    if (!out) fail(HSYM_E_INVALID_ARG, "NULL handle pointer");
    if (!rowptr) fail(HSYM_E_INVALID_ARG, "NULL rowptr");
    if (n < 1 || n >= ((int64_t)1 << 31)) fail(HSYM_E_INVALID_ARG, "n must be in [1, 2^31)");
    if (values_prec != HSYM_FP64 && values_prec != HSYM_FP32) fail(HSYM_E_INVALID_ARG, "bad values precision");
    // device-resident CSR: staged to the host, where the tiles are built
    std::vector<int64_t> rp_h;
    std::vector<int32_t> ci_h;
    std::vector<char> v_h;
    if (flags & HSYM_DEVICE_PTRS) {
        rp_h.resize((size_t)n + 1);
        if (hipMemcpy(rp_h.data(), rowptr, sizeof(int64_t) * rp_h.size(), hipMemcpyDeviceToHost) != hipSuccess) {
            (void)hipGetLastError();
            fail(HSYM_E_INVALID_ARG, "rowptr is not readable device memory");
        }
        const int64_t nnz = rp_h[(size_t)n];
        if (rp_h[0] != 0 || nnz < 0) fail(HSYM_E_INVALID_ARG, "rowptr[0] != 0 or rowptr[n] < 0");
        if (nnz > 0) {
            if (!colind || !values) fail(HSYM_E_INVALID_ARG, "NULL CSR array");
            const size_t vs = values_prec == HSYM_FP64 ? 8 : 4;
            ci_h.resize((size_t)nnz);
            v_h.resize((size_t)nnz * vs);
            if (hipMemcpy(ci_h.data(), colind, sizeof(int32_t) * ci_h.size(), hipMemcpyDeviceToHost) != hipSuccess ||
                hipMemcpy(v_h.data(), values, v_h.size(), hipMemcpyDeviceToHost) != hipSuccess) {
                (void)hipGetLastError();
                fail(HSYM_E_INVALID_ARG, "colind or values is not readable device memory");
            }
        }
        rowptr = rp_h.data();
        colind = ci_h.data();
        values = v_h.data();
        flags &= ~HSYM_DEVICE_PTRS;
    }
    if (rowptr[0] != 0) fail(HSYM_E_INVALID_ARG, "rowptr[0] != 0");
    hsym_t H = nullptr;
    int st = hsym_create_begin(&H, n, storage, flags, stream);
    if (st) return st;
    try {
        builder_append(H, n, rowptr, colind, values, values_prec);
        builder_finish(H);
    } catch (...) {
        destroy_matrix(H);
        throw;
    }
    *out = H;
    API_END
}

int hsym_attach_group_tiles(hsym_t H, int64_t ngroups, const int64_t *group_start, const int64_t *rowptr,
                            const int32_t *colind, const void *values, int values_prec) {
    API_BEGIN
    if (!H || !H->ready) fail(HSYM_E_INVALID_ARG, "invalid handle");
    if (!group_start || !rowptr || !colind || !values) fail(HSYM_E_INVALID_ARG, "NULL argument");
    if (values_prec != HSYM_FP64 && values_prec != HSYM_FP32) fail(HSYM_E_INVALID_ARG, "bad values precision");
    const int64_t n = H->n;
    if (ngroups < 1 || group_start[0] != 0 || group_start[ngroups] != n)
        fail(HSYM_E_INVALID_ARG, "group boundaries must run from 0 to n");
    if (rowptr[0] != 0) fail(HSYM_E_INVALID_ARG, "rowptr[0] != 0");
    // tiles: the groups, cut into pieces of at most 64 rows
    std::vector<int64_t> st{0};
    for (int64_t g = 0; g < ngroups; g++) {
        if (group_start[g + 1] <= group_start[g]) fail(HSYM_E_INVALID_ARG, "group boundaries must ascend");
        for (int64_t a = group_start[g]; a < group_start[g + 1]; a += 64)
            st.push_back(std::min(group_start[g + 1], a + 64));
    }
    const int64_t nt = (int64_t)st.size() - 1;
    std::vector<int64_t> off((size_t)nt + 1, 0);
    for (int64_t t = 0; t < nt; t++) {
        const int64_t sz = st[(size_t)t + 1] - st[(size_t)t];
        off[(size_t)t + 1] = off[(size_t)t] + sz * sz;
    }
    std::vector<double> dense((size_t)off[(size_t)nt], 0.0);
    parallel_for(nt, 64, [&](int64_t t0, int64_t t1) {
        for (int64_t t = t0; t < t1; t++) {
            const int64_t a = st[(size_t)t], b = st[(size_t)t + 1], sz = b - a;
            double *D = dense.data() + off[(size_t)t];
            for (int64_t r = a; r < b; r++) {
                if (rowptr[r + 1] < rowptr[r]) fail(HSYM_E_INVALID_ARG, "rowptr decreases at row " + std::to_string(r));
                for (int64_t p = rowptr[r]; p < rowptr[r + 1]; p++) {
                    const int64_t c = colind[p];
                    if (c < r || c >= n) fail(HSYM_E_INVALID_ARG, "column outside [row, n) in row " + std::to_string(r));
                    if (c >= b) break;
                    const double v = values_prec == HSYM_FP64 ? ((const double *)values)[p]
                                                              : (double)((const float *)values)[p];
                    D[(r - a) * sz + (c - a)] = v;
                    D[(c - a) * sz + (r - a)] = v;
                }
            }
        }
    });
    int64_t *d_st = nullptr, *d_off = nullptr;
    double *d_dense = nullptr;
    auto cleanup = [&] {
        if (d_st) (void)hipFree(d_st);
        if (d_off) (void)hipFree(d_off);
        if (d_dense) (void)hipFree(d_dense);
    };
    try {
        HIPCHK(hipMalloc((void **)&d_st, sizeof(int64_t) * st.size()));
        HIPCHK(hipMalloc((void **)&d_off, sizeof(int64_t) * off.size()));
        HIPCHK(hipMalloc((void **)&d_dense, sizeof(double) * std::max<size_t>(1, dense.size())));
        HIPCHK(hipMemcpy(d_st, st.data(), sizeof(int64_t) * st.size(), hipMemcpyHostToDevice));
        HIPCHK(hipMemcpy(d_off, off.data(), sizeof(int64_t) * off.size(), hipMemcpyHostToDevice));
        HIPCHK(hipMemcpy(d_dense, dense.data(), sizeof(double) * dense.size(), hipMemcpyHostToDevice));
    } catch (...) {
        cleanup();
        throw;
    }
    if (H->tg_start) (void)hipFree(H->tg_start);
    if (H->tg_off) (void)hipFree(H->tg_off);
    if (H->tg_dense) (void)hipFree(H->tg_dense);
    H->bytes -= H->tg_bytes;
    H->ntg = nt;
    H->tg_start = d_st;
    H->tg_off = d_off;
    H->tg_dense = d_dense;
    H->tg_bytes = (int64_t)(sizeof(int64_t) * (st.size() + off.size()) + sizeof(double) * dense.size());
    H->bytes += H->tg_bytes;
    API_END
}

int hsym_destroy(hsym_t H) {
    API_BEGIN
    if (!H) fail(HSYM_E_INVALID_ARG, "NULL handle");
    destroy_matrix(H);
    API_END
}

int hsym_info(hsym_t H, hsym_info_t *o) {
    API_BEGIN
    if (!H || !o) fail(HSYM_E_INVALID_ARG, "NULL argument");
    if (!H->ready) fail(HSYM_E_INVALID_ARG, "handle not finished");
    memset(o, 0, sizeof(*o));
    o->n = H->n;
    o->nnz_stored = H->nnz;
    o->norm1 = H->norm1;
    o->storage = H->storage;
    o->panel_rows = H->tiles.g.R;
    o->chunk_cols = H->tiles.g.C;
    o->npanels = H->tiles.npanels;
    o->ntiles = H->tiles.ntiles;
    o->nslots = H->tiles.next;
    o->padded_entries = H->tiles.nentries;
    o->device_bytes = H->bytes;
    o->has_block64 = H->pre_q != nullptr;
    o->index_bytes = H->tiles.g.idx_bytes;
    o->npieces = H->tiles.npieces;
    o->piece_entries = H->tiles.g.maxe;
    API_END
}

static void check_block(hsym_t H, int m, const void *X, int64_t ldx, const void *Y, int64_t ldy) {
    if (!H || !H->ready) fail(HSYM_E_INVALID_ARG, "invalid handle");
    if (m < 1 || m > HSYM_MAX_BLOCK) fail(HSYM_E_INVALID_ARG, "m must be in [1, 16]");
    if (!X || !Y) fail(HSYM_E_INVALID_ARG, "NULL block");
    if (ldx < m || ldy < m) fail(HSYM_E_INVALID_ARG, "leading dimension < m");
}

int spmm_sym(hsym_t H, int m, const double *X, int64_t ldx, double *Y, int64_t ldy, void *stream) {
    API_BEGIN
    check_block(H, m, X, ldx, Y, ldy);
    spmm_launch(H, m, X, T_F64, ldx, Y, T_F64, ldy, (hipStream_t)stream);
    API_END
}

int spmm_sym_f32(hsym_t H, int m, const float *X, int64_t ldx, float *Y, int64_t ldy, void *stream) {
    API_BEGIN
    check_block(H, m, X, ldx, Y, ldy);
    if (H->storage != HSYM_FP32) fail(HSYM_E_INVALID_ARG, "spmm_sym_f32 needs fp32 storage");
    spmm_launch(H, m, X, T_F32, ldx, Y, T_F32, ldy, (hipStream_t)stream);
    API_END
}

}  // extern "C"
