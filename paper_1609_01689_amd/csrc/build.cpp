// Host-side construction of the device tile format from upper-triangle CSR.
//
// The stored triangle is cut into row panels and column chunks (the CSB
// blocking of Sections 2.2 and 4.2: independently addressable blocks of the
// half-stored matrix) and uploaded in batches of panels, so a matrix larger
// than host memory can be streamed slab by slab.
#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstring>
#include <mutex>
#include <thread>

#include "hsym_internal.h"

namespace hsym {

int host_threads() {
    static int t = [] {
        const char *e = getenv("HSYM_HOST_THREADS");
        int v = e ? atoi(e) : (int)std::thread::hardware_concurrency();
        if (v < 1) v = 1;
        if (v > 64) v = 64;
        return v;
    }();
    return t;
}

void parallel_for(int64_t n, int64_t grain, const std::function<void(int64_t, int64_t)> &fn) {
    if (n <= 0) return;
    int nt = host_threads();
    if (nt == 1 || n <= grain) { fn(0, n); return; }
    std::atomic<int64_t> next(0);
    std::vector<std::thread> th;
    std::mutex em;
    std::string err;
    int errst = 0;
    auto body = [&] {
        for (;;) {
            int64_t a = next.fetch_add(grain);
            if (a >= n) break;
            int64_t b = std::min(n, a + grain);
            try { fn(a, b); } catch (Error &e) {
                std::lock_guard<std::mutex> g(em);
                if (!errst) { errst = e.status; err = e.msg; }
                next.store(n);
            }
        }
    };
    for (int t = 0; t < nt - 1; t++) th.emplace_back(body);
    body();
    for (auto &t : th) t.join();
    if (errst) fail(errst, err);
}

void geometry_for(int storage, int m, int64_t n, int lr, int lc, int *R, int *C, int *G) {
    // Panel rows R and chunk columns C = R/4: the largest power-of-two R for
    // which the panel accumulator, the panel's X rows, the staged X chunk and
    // the chunk's transposed accumulator fit the 160 KB LDS of a gfx950 CU.
    const size_t budget = 160 * 1024;
    int r = 65536;
    while (r > 64 && spmm_lds_bytes(storage, m, r, r / 4) > budget) r /= 2;
    // keep at least one panel per CU (256 CUs) when n allows
    while (r > 256 && (int64_t)r * 256 > n) r /= 2;
    int c = r / 4;
    if (lr > 0) {
        // explicit geometry (hsym_create flags, e.g. from the autotuner)
        if (lr > 16 || lc < 3 || lc > 16) fail(HSYM_E_INVALID_ARG, "panel geometry exponents out of range");
        r = 1 << lr;
        c = 1 << lc;
    } else {
        const char *er = getenv("HSYM_PANEL_ROWS");
        const char *ec = getenv("HSYM_CHUNK_COLS");
        if (er) r = atoi(er);
        if (ec) c = atoi(ec);
    }
    // the SpMM relies on chunks tiling panels and on chunk rows sharing the
    // LDS swizzle of their panel rows (a multiple of 8)
    if (r < 64 || r > 65536 || c < 8 || c % 8 || r % c)
        fail(HSYM_E_INVALID_ARG, "panel geometry must have 64 <= R <= 65536, C a multiple of 8 dividing R");
    *R = r;
    *C = c;
    // one segment per lane group of the 1024-thread workgroup at this width
    *G = 1024 / spmm_lanes_per_entry(storage, m);
}

// ---------------------------------------------------------------------------
// one panel
// ---------------------------------------------------------------------------
struct PanelOut {
    std::vector<TileDesc> tiles;      // base relative to the panel
    std::vector<uint32_t> idx;
    std::vector<double> v64;
    std::vector<float> v32;
    std::vector<int32_t> ext_chunks;  // chunk of every external tile, in order
    std::vector<double> colsum;       // |a| summed per column, window [r0, r0 + size)
    double rowsum_max = 0.0;
    int64_t nnz = 0;                  // stored entries incl. diagonal
    std::vector<double> preq, prelam; // block-64 factors of the panel's 64-row chunks
};

bool sym_eig_host(int n, double *A, double *w);

// Dense diagonal block of the 64 rows starting at c0 (sz rows), factored as
// Q diag(lambda) Q^T; Q is stored row-major and padded to 64x64 with the
// identity, lambda padded with ones.
static void block64_factor(int64_t c0, int sz, int64_t slab_row0, const int64_t *rp, const int32_t *ci,
                           const double *vin64, const float *vin32, PanelOut &out) {
    std::vector<double> B((size_t)sz * sz, 0.0), w(sz);
    for (int i = 0; i < sz; i++) {
        int64_t row = c0 + i;
        for (int64_t p = rp[row - slab_row0]; p < rp[row - slab_row0 + 1]; p++) {
            int64_t j = ci[p];
            if (j >= c0 + sz) break;
            double v = vin64 ? vin64[p] : (double)vin32[p];
            B[(size_t)i * sz + (j - c0)] = v;
            B[(size_t)(j - c0) * sz + i] = v;
        }
    }
    if (!sym_eig_host(sz, B.data(), w.data()))
        fail(HSYM_E_NUMERIC, "block-64 eigendecomposition did not converge at row " + std::to_string(c0));
    size_t q0 = out.preq.size();
    out.preq.resize(q0 + 64 * 64, 0.0);
    for (int i = 0; i < 64; i++)
        for (int j = 0; j < 64; j++)
            out.preq[q0 + (size_t)i * 64 + j] = (i < sz && j < sz) ? B[(size_t)i * sz + j] : (i == j ? 1.0 : 0.0);
    for (int j = 0; j < 64; j++) out.prelam.push_back(j < sz ? w[j] : 1.0);
}

// Rows [r0, r1) of the matrix; rp/ci/v index the caller's slab whose first row
// is slab_row0.  dg receives the diagonal of the panel rows.
static void build_panel(int64_t n, int64_t r0, int64_t r1, int R, int C, int G, int cs, int storage, bool b64,
                        int64_t slab_row0, const int64_t *rp, const int32_t *ci,
                        const double *vin64, const float *vin32, double *dg, PanelOut &out) {
    const int nr = (int)(r1 - r0);
    std::vector<int64_t> cur(nr), end(nr);
    int64_t maxcol = r0;
    std::vector<double> rowsum(nr, 0.0);
    for (int i = 0; i < nr; i++) {
        int64_t row = r0 + i;
        int64_t a = rp[row - slab_row0], b = rp[row - slab_row0 + 1];
        if (b < a) fail(HSYM_E_INVALID_ARG, "rowptr decreases at row " + std::to_string(row));
        out.nnz += b - a;
        dg[i] = 0.0;
        int64_t prev = -1;
        for (int64_t p = a; p < b; p++) {
            int64_t c = ci[p];
            double v = vin64 ? vin64[p] : (double)vin32[p];
            if (c < row || c >= n)
                fail(HSYM_E_INVALID_ARG, "column " + std::to_string(c) + " outside [row, n) in row " +
                                             std::to_string(row));
            if (c <= prev)
                fail(HSYM_E_INVALID_ARG, "columns not strictly increasing in row " + std::to_string(row));
            if (!std::isfinite(v)) fail(HSYM_E_INVALID_ARG, "non-finite value in row " + std::to_string(row));
            prev = c;
            rowsum[i] += std::fabs(v);
        }
        if (b > a && ci[a] == row) { dg[i] = vin64 ? vin64[a] : (double)vin32[a]; a++; }
        cur[i] = a;
        end[i] = b;
        if (b > a) maxcol = std::max<int64_t>(maxcol, ci[b - 1]);
    }
    // the window covers every row of the panel and every column it touches
    out.colsum.assign((size_t)(std::max<int64_t>(maxcol, r1 - 1) - r0 + 1), 0.0);
    for (int i = 0; i < nr; i++)
        for (int64_t p = cur[i]; p < end[i]; p++)
            out.colsum[ci[p] - r0] += std::fabs(vin64 ? vin64[p] : (double)vin32[p]);
    for (int i = 0; i < nr; i++) out.rowsum_max = std::max(out.rowsum_max, rowsum[i]);
    // rowsum is combined with column sums by the caller: keep per-row values in colsum too
    for (int i = 0; i < nr; i++) out.colsum[i] += rowsum[i];

    if (b64)
        for (int64_t c0 = r0; c0 < r1; c0 += 64)
            block64_factor(c0, (int)std::min<int64_t>(64, r1 - c0), slab_row0, rp, ci, vin64, vin32, out);

    const int64_t gmin = r0 / C, gmax = maxcol / C;
    std::vector<int> cnt(nr);
    for (int64_t g = gmin; g <= gmax; g++) {
        const int64_t cend = (g + 1) * (int64_t)C;
        int64_t nnz = 0;
        int last = -1;
        for (int i = 0; i < nr; i++) {
            int64_t p = cur[i];
            while (p < end[i] && ci[p] < cend) p++;
            cnt[i] = (int)(p - cur[i]);
            nnz += cnt[i];
            if (cnt[i]) last = i;
        }
        if (!nnz) continue;
        TileDesc td;
        td.base = (int64_t)out.idx.size();
        td.len = (int32_t)((nnz + G - 1) / G);
        td.chunk = (int32_t)g;
        bool ext = g * (int64_t)C >= r0 + R;
        td.slot = ext ? (int32_t)out.ext_chunks.size() : -1;
        td.pad = 0;
        if (ext) out.ext_chunks.push_back((int32_t)g);
        out.tiles.push_back(td);
        const size_t sz = (size_t)td.len * G;
        const size_t b0 = out.idx.size();
        // padding: zero values on the last row (keeps a segment's row run unbroken)
        out.idx.resize(b0 + sz, (uint32_t)last << cs);
        if (storage == HSYM_FP64) out.v64.resize(b0 + sz, 0.0);
        else out.v32.resize(b0 + sz, 0.0f);
        int64_t logical = 0;
        for (int i = 0; i < nr; i++) {
            for (int e = 0; e < cnt[i]; e++, logical++) {
                int64_t p = cur[i] + e;
                const int64_t seg = logical / td.len, pos = logical - seg * td.len;
                const size_t at = b0 + (size_t)pos * G + (size_t)seg;
                out.idx[at] = ((uint32_t)i << cs) | (uint32_t)(ci[p] - g * (int64_t)C);
                if (storage == HSYM_FP64) out.v64[at] = vin64 ? vin64[p] : (double)vin32[p];
                else out.v32[at] = vin64 ? (float)vin64[p] : vin32[p];
            }
        }
        for (int i = 0; i < nr; i++) cur[i] += cnt[i];
    }
}

// ---------------------------------------------------------------------------
// growable device arrays
// ---------------------------------------------------------------------------
template <class T>
struct DevVec {
    T *p = nullptr;
    int64_t size = 0, cap = 0;
    void reserve(int64_t c) {
        if (c <= cap) return;
        T *q = nullptr;
        if (hipMalloc(&q, sizeof(T) * (size_t)std::max<int64_t>(c, 1)) != hipSuccess) {
            (void)hipGetLastError();
            fail(HSYM_E_OUT_OF_MEMORY, "device allocation of " + std::to_string(sizeof(T) * c) + " bytes");
        }
        if (size) HIPCHK(hipMemcpy(q, p, sizeof(T) * size, hipMemcpyDeviceToDevice));
        if (p) HIPCHK(hipFree(p));
        p = q;
        cap = c;
    }
    void append(const T *h, int64_t k) {
        if (!k) return;
        if (size + k > cap) reserve(std::max<int64_t>(size + k, cap + cap / 4 + 1024));
        HIPCHK(hipMemcpy(p + size, h, sizeof(T) * k, hipMemcpyHostToDevice));
        size += k;
    }
    void release() { if (p) (void)hipFree(p); p = nullptr; size = cap = 0; }
};

struct Builder {
    int R = 0, C = 0, G = 256;
    bool idx16 = false;             // 16-bit index codes (shift log2 C)
    int cs = 16;                    // code shift: local row << cs | local column
    int storage = HSYM_FP64;
    bool b64 = false;
    DevVec<double> preq, prelam;
    int64_t n = 0;
    int64_t next_row = 0;          // first row not yet turned into panels
    int64_t npanels_done = 0;
    int64_t nnz = 0;
    // carried rows of an incomplete panel
    std::vector<int64_t> carry_rp{0};
    std::vector<int32_t> carry_ci;
    std::vector<double> carry_v64;
    std::vector<float> carry_v32;
    // device arrays
    DevVec<TileDesc> tiles;
    DevVec<uint32_t> idx;
    DevVec<uint16_t> idx16v;
    DevVec<double> v64;
    DevVec<float> v32;
    std::vector<int64_t> panel_tile_ptr{0};
    std::vector<int64_t> panel_weight;  // per panel: padded entries + a per-tile cost, in entry units
    std::vector<int32_t> slot_chunk;   // chunk of every slot
    std::vector<double> diag;          // n
    std::vector<double> abssum;        // n: row+column absolute sums
    double norm1 = 0.0;
    int64_t nentries = 0, ntiles = 0;

    void release() {
        tiles.release(); idx.release(); idx16v.release(); v64.release(); v32.release();
        preq.release(); prelam.release();
    }

    // turn complete panels [p0, p1) whose rows lie in the given slab into device data
    void panels(int64_t p0, int64_t p1, int64_t slab_row0, const int64_t *rp, const int32_t *ci,
                const double *vin64, const float *vin32) {
        const int64_t BATCH = 4 * host_threads();
        for (int64_t b0 = p0; b0 < p1; b0 += BATCH) {
            int64_t b1 = std::min(p1, b0 + BATCH);
            std::vector<PanelOut> outs((size_t)(b1 - b0));
            parallel_for(b1 - b0, 1, [&](int64_t a, int64_t b) {
                for (int64_t k = a; k < b; k++) {
                    int64_t p = b0 + k;
                    int64_t r0 = p * R, r1 = std::min(n, r0 + R);
                    build_panel(n, r0, r1, R, C, G, cs, storage, b64, slab_row0, rp, ci, vin64, vin32,
                                diag.data() + r0, outs[(size_t)k]);
                }
            });
            // concatenate in panel order
            std::vector<TileDesc> t;
            std::vector<uint32_t> c;
            std::vector<double> d64;
            std::vector<float> d32;
            std::vector<double> pq, pl;
            for (int64_t k = 0; k < b1 - b0; k++) {
                PanelOut &o = outs[(size_t)k];
                int64_t r0 = (b0 + k) * R;
                int64_t entry_off = nentries + (int64_t)c.size();
                int32_t slot_off = (int32_t)slot_chunk.size();
                for (auto td : o.tiles) {
                    td.base += entry_off;
                    if (td.slot >= 0) td.slot += slot_off;
                    t.push_back(td);
                }
                c.insert(c.end(), o.idx.begin(), o.idx.end());
                d64.insert(d64.end(), o.v64.begin(), o.v64.end());
                d32.insert(d32.end(), o.v32.begin(), o.v32.end());
                for (int32_t g : o.ext_chunks) slot_chunk.push_back(g);
                pq.insert(pq.end(), o.preq.begin(), o.preq.end());
                pl.insert(pl.end(), o.prelam.begin(), o.prelam.end());
                panel_tile_ptr.push_back(panel_tile_ptr.back() + (int64_t)o.tiles.size());
                {
                    // a tile's fixed cost (staging its X chunk, barriers, writing its sums)
                    // is about that of 1,200 entries at m = 16
                    int64_t wgt = 1200 * (int64_t)o.tiles.size();
                    for (const auto &td : o.tiles) wgt += (int64_t)td.len * G;
                    panel_weight.push_back(wgt);
                }
                for (size_t w = 0; w < o.colsum.size(); w++) abssum[(size_t)r0 + w] += o.colsum[w];
                nnz += o.nnz;
                PanelOut().tiles.swap(o.tiles);
            }
            tiles.append(t.data(), (int64_t)t.size());
            if (idx16) {
                std::vector<uint16_t> c16(c.begin(), c.end());
                idx16v.append(c16.data(), (int64_t)c16.size());
            } else {
                idx.append(c.data(), (int64_t)c.size());
            }
            if (storage == HSYM_FP64) v64.append(d64.data(), (int64_t)d64.size());
            else v32.append(d32.data(), (int64_t)d32.size());
            if (b64) { preq.append(pq.data(), (int64_t)pq.size()); prelam.append(pl.data(), (int64_t)pl.size()); }
            ntiles += (int64_t)t.size();
            nentries += (int64_t)c.size();
            npanels_done = b1;
        }
    }

    void carry_rows(int64_t k, const int64_t *rp, const int32_t *ci, const double *vd, const float *vf) {
        for (int64_t i = 0; i < k; i++) {
            for (int64_t p = rp[i]; p < rp[i + 1]; p++) {
                carry_ci.push_back(ci[p]);
                if (vd) carry_v64.push_back(vd[p]); else carry_v32.push_back(vf[p]);
            }
            carry_rp.push_back((int64_t)carry_ci.size());
        }
    }

    // Rows arrive in order; complete panels are built as soon as all their
    // rows are present, the rows of an incomplete panel are carried over.
    void append(int64_t nrows, const int64_t *rp, const int32_t *ci, const void *vals, int vprec) {
        int64_t carried = (int64_t)carry_rp.size() - 1;
        if (nrows < 0 || next_row + carried + nrows > n) fail(HSYM_E_INVALID_ARG, "appended rows exceed n");
        if (nrows == 0) return;
        if (!rp || (rp[nrows] > rp[0] && (!ci || !vals))) fail(HSYM_E_INVALID_ARG, "NULL CSR array");
        if (rp[0] != 0) fail(HSYM_E_INVALID_ARG, "rowptr[0] != 0");
        for (int64_t i = 0; i < nrows; i++)
            if (rp[i + 1] < rp[i])
                fail(HSYM_E_INVALID_ARG, "rowptr decreases at row " + std::to_string(next_row + carried + i));
        const double *vd = vprec == HSYM_FP64 ? (const double *)vals : nullptr;
        const float *vf = vprec == HSYM_FP32 ? (const float *)vals : nullptr;
        int64_t slab_row0 = next_row + carried;
        if (carried > 0) {
            int64_t pc = npanels_done;
            int64_t pend_row = std::min(n, (pc + 1) * (int64_t)R);
            int64_t take = std::min(nrows, pend_row - slab_row0);
            carry_rows(take, rp, ci, vd, vf);
            rp += take; nrows -= take; slab_row0 += take;
            if (slab_row0 == pend_row) {
                panels(pc, pc + 1, next_row, carry_rp.data(), carry_ci.data(),
                       vd ? carry_v64.data() : nullptr, vf ? carry_v32.data() : nullptr);
                carry_rp.assign(1, 0); carry_ci.clear(); carry_v64.clear(); carry_v32.clear();
                std::vector<double>().swap(carry_v64); std::vector<float>().swap(carry_v32);
                next_row = pend_row;
            }
            if (nrows == 0) return;
        }
        // slab now starts on a panel boundary (next_row == slab_row0)
        int64_t last = slab_row0 + nrows;
        int64_t pbeg = npanels_done;
        int64_t pend = (last == n) ? (n + R - 1) / R : last / R;
        if (pend > pbeg) {
            panels(pbeg, pend, slab_row0, rp, ci, vd, vf);
            int64_t done = std::min(n, pend * (int64_t)R) - slab_row0;
            next_row = slab_row0 + done;
            rp += done; nrows -= done;
        }
        if (nrows > 0) {
            // rebase the leftover rows' pointers: carry_rows copies entries by index
            carry_rows(nrows, rp, ci, vd, vf);
        }
    }
};

}  // namespace hsym

using namespace hsym;

// The builder lives behind the handle while a streaming create is open.
static std::mutex g_builders_mu;
static std::vector<std::pair<hsym_matrix *, Builder *>> g_builders;

static Builder *builder_of(hsym_matrix *H) {
    std::lock_guard<std::mutex> g(g_builders_mu);
    for (auto &p : g_builders) if (p.first == H) return p.second;
    return nullptr;
}

namespace hsym {

void builder_begin(hsym_matrix *H, int64_t nnz_hint) {
    Builder *b = new Builder();
    b->n = H->n;
    b->storage = H->storage;
    b->b64 = (H->flags & HSYM_BUILD_BLOCK64) != 0;
    geometry_for(H->storage, H->geom_m, H->n, H->geom_lr, H->geom_lc, &b->R, &b->C, &b->G);
    if (b->G < 1) fail(HSYM_E_INVALID_ARG, "bad segment count");
    if (b->R % b->C != 0 || b->C > 65536 || b->R > 65535)
        fail(HSYM_E_INVALID_ARG, "panel rows must be a multiple of chunk columns (<= 65535)");
    // 16-bit codes on request, when a tile's local row and column fit in 16 bits together
    if ((H->flags & HSYM_INDEX16) && (b->C & (b->C - 1)) == 0 && (int64_t)b->R * b->C <= 65536) {
        b->idx16 = true;
        b->cs = 0;
        while ((1 << b->cs) < b->C) b->cs++;
    }
    b->diag.assign((size_t)H->n, 0.0);
    b->abssum.assign((size_t)H->n, 0.0);
    if (nnz_hint > 0) {
        int64_t est = nnz_hint + nnz_hint / 8 + 4096;
        if (b->idx16) b->idx16v.reserve(est); else b->idx.reserve(est);
        if (H->storage == HSYM_FP64) b->v64.reserve(est); else b->v32.reserve(est);
    }
    std::lock_guard<std::mutex> g(g_builders_mu);
    g_builders.push_back({H, b});
}

void builder_append(hsym_matrix *H, int64_t nrows, const int64_t *rp, const int32_t *ci,
                    const void *vals, int vprec) {
    Builder *b = builder_of(H);
    if (!b) fail(HSYM_E_INVALID_ARG, "no streaming create open on this handle");
    b->append(nrows, rp, ci, vals, vprec);
}

void builder_discard(hsym_matrix *H) {
    std::lock_guard<std::mutex> g(g_builders_mu);
    for (size_t i = 0; i < g_builders.size(); i++)
        if (g_builders[i].first == H) {
            g_builders[i].second->release();
            delete g_builders[i].second;
            g_builders.erase(g_builders.begin() + (long)i);
            return;
        }
}

void builder_finish(hsym_matrix *H) {
    Builder *b = builder_of(H);
    if (!b) fail(HSYM_E_INVALID_ARG, "no streaming create open on this handle");
    if (b->next_row != H->n || b->carry_rp.size() != 1)
        fail(HSYM_E_INVALID_ARG, "streaming create finished before all n rows were appended");
    DeviceTiles &dt = H->tiles;
    dt.R = b->R; dt.C = b->C; dt.G = b->G;
    dt.npanels = (H->n + b->R - 1) / b->R;
    dt.nchunks = (H->n + b->C - 1) / b->C;
    dt.ntiles = b->ntiles; dt.nentries = b->nentries;
    dt.nslots = (int64_t)b->slot_chunk.size();
    dt.tiles = b->tiles.p;
    dt.idx = b->idx16 ? (void *)b->idx16v.p : (void *)b->idx.p;
    dt.idx_bytes = b->idx16 ? 2 : 4;
    dt.idx_shift = b->cs;
    dt.vals = H->storage == HSYM_FP64 ? (void *)b->v64.p : (void *)b->v32.p;
    const int64_t idx_cap_bytes = b->idx16 ? b->idx16v.cap * 2 : b->idx.cap * 4;
    b->tiles.p = nullptr; b->idx.p = nullptr; b->idx16v.p = nullptr;
    b->v64.p = nullptr; b->v32.p = nullptr;
    int vs = H->storage == HSYM_FP64 ? 8 : 4;
    dt.bytes = b->tiles.cap * (int64_t)sizeof(TileDesc) + idx_cap_bytes +
               (H->storage == HSYM_FP64 ? b->v64.cap : b->v32.cap) * vs;
    // panel pointers
    HIPCHK(hipMalloc(&dt.panel_tile_ptr, sizeof(int64_t) * b->panel_tile_ptr.size()));
    HIPCHK(hipMemcpy(dt.panel_tile_ptr, b->panel_tile_ptr.data(), sizeof(int64_t) * b->panel_tile_ptr.size(),
                     hipMemcpyHostToDevice));
    dt.bytes += (int64_t)(sizeof(int64_t) * b->panel_tile_ptr.size());
    // workgroup -> panel.  The dispatcher deals workgroups round-robin to the
    // 8 XCDs (workgroup b to XCD b mod 8).  XCD x gets a contiguous run of
    // panels, so the X chunks that neighbouring panels share stay in its L2.
    // With few panels per CU it takes them heaviest first, so that its CUs
    // end on light panels (list scheduling; the panels' loads differ by up to
    // 2x); with many, in row order, which keeps more chunk reuse in L2.
    {
        const int64_t P = dt.npanels, q = P >> 3, rem = P & 7;
        const bool heavy_first = P < 16 * 256;
        std::vector<int32_t> order((size_t)P);
        for (int64_t x = 0; x < 8; x++) {
            const int64_t lo = x * q + std::min<int64_t>(x, rem), cnt = q + (x < rem ? 1 : 0);
            std::vector<int32_t> ps((size_t)cnt);
            for (int64_t i = 0; i < cnt; i++) ps[(size_t)i] = (int32_t)(lo + i);
            if (heavy_first)
                std::stable_sort(ps.begin(), ps.end(), [&](int32_t u, int32_t v) {
                    return b->panel_weight[(size_t)u] > b->panel_weight[(size_t)v];
                });
            for (int64_t i = 0; i < cnt; i++) order[(size_t)(8 * i + x)] = ps[(size_t)i];
        }
        HIPCHK(hipMalloc(&dt.panel_order, sizeof(int32_t) * std::max<size_t>(1, order.size())));
        if (!order.empty())
            HIPCHK(hipMemcpy(dt.panel_order, order.data(), sizeof(int32_t) * order.size(), hipMemcpyHostToDevice));
        dt.bytes += (int64_t)(sizeof(int32_t) * order.size());
    }
    // reduction lists: slots per output chunk in panel order
    std::vector<int64_t> rptr((size_t)dt.nchunks + 1, 0);
    for (int32_t g : b->slot_chunk) rptr[(size_t)g + 1]++;
    for (int64_t g = 0; g < dt.nchunks; g++) rptr[(size_t)g + 1] += rptr[(size_t)g];
    std::vector<int32_t> rs(b->slot_chunk.size());
    std::vector<int64_t> fill(rptr.begin(), rptr.end() - 1);
    for (size_t s = 0; s < b->slot_chunk.size(); s++) rs[(size_t)fill[(size_t)b->slot_chunk[s]]++] = (int32_t)s;
    std::vector<int32_t> rc;
    for (int64_t g = 0; g < dt.nchunks; g++) if (rptr[(size_t)g + 1] > rptr[(size_t)g]) rc.push_back((int32_t)g);
    dt.nred_chunks = (int64_t)rc.size();
    HIPCHK(hipMalloc(&dt.red_ptr, sizeof(int64_t) * rptr.size()));
    HIPCHK(hipMemcpy(dt.red_ptr, rptr.data(), sizeof(int64_t) * rptr.size(), hipMemcpyHostToDevice));
    HIPCHK(hipMalloc(&dt.red_slot, sizeof(int32_t) * std::max<size_t>(1, rs.size())));
    if (!rs.empty()) HIPCHK(hipMemcpy(dt.red_slot, rs.data(), sizeof(int32_t) * rs.size(), hipMemcpyHostToDevice));
    HIPCHK(hipMalloc(&dt.red_chunks, sizeof(int32_t) * std::max<size_t>(1, rc.size())));
    if (!rc.empty()) HIPCHK(hipMemcpy(dt.red_chunks, rc.data(), sizeof(int32_t) * rc.size(), hipMemcpyHostToDevice));
    dt.bytes += (int64_t)(sizeof(int64_t) * rptr.size() + 4 * rs.size() + 4 * rc.size());
    // diagonal in both precisions and ||H||_1
    H->d_host = b->diag;
    std::vector<float> d32(b->diag.size());
    for (size_t i = 0; i < d32.size(); i++) d32[i] = (float)b->diag[i];
    HIPCHK(hipMalloc(&H->diag64, sizeof(double) * (size_t)H->n));
    HIPCHK(hipMalloc(&H->diag32, sizeof(float) * (size_t)H->n));
    HIPCHK(hipMemcpy(H->diag64, b->diag.data(), sizeof(double) * (size_t)H->n, hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(H->diag32, d32.data(), sizeof(float) * (size_t)H->n, hipMemcpyHostToDevice));
    if (b->b64) {
        H->pre_q = b->preq.p; H->pre_lam = b->prelam.p;
        H->pre_nchunks = (H->n + 63) / 64;
        dt.bytes += b->preq.cap * 8 + b->prelam.cap * 8;
        b->preq.p = nullptr; b->prelam.p = nullptr;
    }
    double nm = 0.0;
    for (double v : b->abssum) nm = std::max(nm, v);
    H->norm1 = nm;
    H->nnz = b->nnz;
    H->bytes = dt.bytes + 12 * H->n;
    builder_discard(H);
    H->ready = true;
}

void free_tiles(DeviceTiles *dt) {
    void *ptrs[] = {dt->panel_tile_ptr, dt->panel_order, dt->tiles, dt->idx, dt->vals,
                    dt->red_ptr, dt->red_slot, dt->red_chunks};
    for (void *p : ptrs) if (p) (void)hipFree(p);
    *dt = DeviceTiles();
}

}  // namespace hsym
