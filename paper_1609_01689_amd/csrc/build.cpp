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
#include <memory>
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

// LDS of the SpMM at block width m (spmm.hip): fp64 accumulators for the
// panel rows and the chunk rows, the panel's and the chunk's X rows in the
// arithmetic precision (that of the storage), and the staged codes, perm and
// values of one piece.
size_t spmm_lds_bytes(int storage, int m, const Geom &g) {
    const size_t M = (size_t)round_m(m), sa = storage == HSYM_FP64 ? 8 : 4;
    auto r16 = [](size_t b) { return (b + 15) & ~(size_t)15; };
    const size_t xs = M + (size_t)spmm_xpad((int)M);   // staged X row stride
    return (size_t)(g.R + g.C) * (M * 8 + xs * sa) + r16((size_t)g.maxe * g.idx_bytes) + r16((size_t)g.maxe * 2) +
           r16((size_t)g.maxe * sa);
}

// Lane groups of the 1024-thread SpMM workgroup at block width M: a group
// holds spmm_lane_elems(M) elements of an X row per lane, so the number of
// groups (segments per piece) is 1024 divided by the lanes one row needs.
static int segments_for(int storage, int M) {
    (void)storage;
    const int mw = spmm_lane_elems(M);
    return 1024 / (M / mw);
}

Geom geometry_for(int storage, int m, int64_t n, int r64, int lc) {
    const int M = round_m(m);
    const size_t budget = 160 * 1024;
    const int sa = storage == HSYM_FP64 ? 8 : 4;
    Geom g;
    g.G = segments_for(storage, M);
    auto fill = [&](int R, int C) -> bool {
        g.R = R;
        g.C = C;
        g.cb = 0;
        while ((1 << g.cb) < C) g.cb++;
        g.idx_bytes = (int64_t)R * C <= 65536 ? 2 : 4;
        g.maxe = 0;
        const size_t fixed = spmm_lds_bytes(storage, M, g);
        if (fixed + 64 > budget) return false;
        // entries per piece: what is left of the LDS, a multiple of 8, and the
        // perm codes of a piece index at most 2^16 positions
        const size_t eb = (size_t)g.idx_bytes + 2 + sa;
        int64_t e = (int64_t)((budget - fixed - 64) / eb);
        // a piece is staged through registers: at most spmm_stage_units(M)
        // units of 16 bytes per thread of the workgroup, three streams each
        // rounded up to 16 bytes
        e = std::min<int64_t>(e, ((int64_t)spmm_stage_units(M) * 1024 - 3) * 16 / (int64_t)eb);
        e = std::min<int64_t>(e, 16384) & ~(int64_t)7;
        g.maxe = (int)e;
        return spmm_lds_bytes(storage, M, g) <= budget;
    };
    if (r64 > 0) {
        // explicit geometry (hsym_create flags, e.g. from the autotuner)
        const int R = 64 * r64, C = 1 << lc;
        if (lc < 3 || lc > 12 || C > R || R % C || (int64_t)C * M > 4096)
            fail(HSYM_E_INVALID_ARG, "panel geometry must have C = 2^lc (3 <= lc <= 12) dividing R = 64 * r64");
        if (!fill(R, C) || g.maxe < 256)
            fail(HSYM_E_INVALID_ARG, "panel geometry does not fit the LDS at the geometry block width");
        return g;
    }
    // Chunks of 128 columns first, then the tallest panels whose pieces still
    // hold about 4,000 entries (measured on CI-shaped matrices at m = 1, 8, 16
    // in both storages: 128-column chunks beat 64 by 8-25%, and full pieces
    // beat taller panels with smaller pieces), at least one panel per CU
    // (256) when n allows, 16-bit codes at block widths of 4 and more.  Then
    // the same with 64-column chunks and at least 2,048 entries per piece.
    const int64_t rmax = std::max<int64_t>(64, std::min<int64_t>(2048, (n / 256) / 64 * 64));
    for (int pass = 0; pass < 2; pass++) {
        for (int C : {128, 64}) {
            for (int64_t R = rmax; R >= C; R -= 64) {
                if (R % C) continue;
                if (M >= 4 && R * C > 65536) continue;
                if ((int64_t)C * M > 4096) continue;
                if (fill((int)R, C) && g.maxe >= (pass == 0 ? 4000 : 2048)) return g;
            }
        }
    }
    if (!fill(64, 64) || g.maxe < 256) fail(HSYM_E_UNSUPPORTED, "no panel geometry fits the LDS at this block width");
    return g;
}

// ---------------------------------------------------------------------------
// one panel
// ---------------------------------------------------------------------------
struct PanelOut {
    std::vector<TileDesc> tiles;      // pieces, base (bytes) relative to the panel
    std::vector<unsigned char> blob;  // the pieces' codes, perm and values
    int64_t positions = 0;            // padded entries of the pieces
    int64_t next = 0;                 // external tiles
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
static void build_panel(int64_t n, int64_t r0, int64_t r1, const Geom &geo, int storage, bool b64,
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

    const int C = geo.C, G = geo.G, cb = geo.cb;
    const int64_t gmin = r0 / C, gmax = maxcol / C;
    std::vector<int> cnt(nr);
    std::vector<int32_t> tr, tc;      // one tile's entries: local row, local column
    std::vector<int64_t> tp;          // and their positions in the slab
    std::vector<int32_t> colcnt((size_t)C + 1), order;
    std::vector<uint32_t> pcode;      // one piece: codes, perm and values by position
    std::vector<uint16_t> pperm;
    std::vector<double> pval;
    for (int64_t g = gmin; g <= gmax; g++) {
        const int64_t cend = (g + 1) * (int64_t)C;
        tr.clear(); tc.clear(); tp.clear();
        for (int i = 0; i < nr; i++) {
            int64_t p = cur[i];
            for (; p < end[i] && ci[p] < cend; p++) {
                tr.push_back(i);
                tc.push_back((int32_t)(ci[p] - g * (int64_t)C));
                tp.push_back(p);
            }
            cnt[i] = (int)(p - cur[i]);
        }
        for (int i = 0; i < nr; i++) cur[i] += cnt[i];
        const int64_t tcnt = (int64_t)tr.size();
        if (!tcnt) continue;
        const bool ext = g * (int64_t)C >= r0 + geo.R;
        if (ext) out.next++;
        // pieces of consecutive row-major entries, at most maxe positions
        // after padding to a whole, even number of steps of G segments
        const int64_t cut = (int64_t)((geo.maxe / G) & ~(SPMM_STEP - 1)) * G;
        if (cut < 1) fail(HSYM_E_INVALID_ARG, "panel geometry leaves no room for a piece");
        const int ib = geo.idx_bytes, sv = storage == HSYM_FP64 ? 8 : 4;
        for (int64_t q0 = 0; q0 < tcnt; q0 += cut) {
            const int pc = (int)std::min<int64_t>(cut, tcnt - q0);
            const int len = ((pc + G - 1) / G + SPMM_STEP - 1) / SPMM_STEP * SPMM_STEP;
            const int64_t E = (int64_t)G * len;
            const PieceParts pp = piece_parts(E, ib, sv);
            const int64_t base = (int64_t)out.blob.size();
            out.blob.resize((size_t)(base + pp.bytes), 0);
            unsigned char *bp = out.blob.data() + base;
            // row-major codes and values at their positions; padding positions
            // repeat the last code with value 0
            const int64_t last = q0 + pc - 1;
            const uint32_t lastcode = ((uint32_t)tr[(size_t)last] << cb) | (uint32_t)tc[(size_t)last];
            pcode.assign((size_t)E, lastcode);
            pval.assign((size_t)E, 0.0);
            for (int64_t q = 0; q < pc; q++) {
                const int64_t at = piece_pos(q % len, q / len, G);
                const int64_t k = q0 + q;
                pcode[(size_t)at] = ((uint32_t)tr[(size_t)k] << cb) | (uint32_t)tc[(size_t)k];
                const int64_t p = tp[(size_t)k];
                pval[(size_t)at] = vin64 ? vin64[p] : (double)vin32[p];
            }
            // column-major order of the piece (a stable counting sort by
            // column keeps rows ascending within a column)
            std::fill(colcnt.begin(), colcnt.end(), 0);
            for (int q = 0; q < pc; q++) colcnt[(size_t)tc[(size_t)(q0 + q)] + 1]++;
            for (int c = 0; c < C; c++) colcnt[(size_t)c + 1] += colcnt[(size_t)c];
            order.assign((size_t)pc, 0);
            for (int q = 0; q < pc; q++) order[(size_t)colcnt[(size_t)tc[(size_t)(q0 + q)]]++] = q;
            // padding positions of the column order point at a padding
            // position of the row order (value 0), which exists when E > pc
            const int64_t padpos = E > pc ? piece_pos(pc % len, pc / len, G) : 0;
            pperm.assign((size_t)E, (uint16_t)padpos);
            for (int64_t q = 0; q < pc; q++) {
                const int64_t o = order[(size_t)q];
                pperm[(size_t)piece_pos(q % len, q / len, G)] = (uint16_t)piece_pos(o % len, o / len, G);
            }
            // the piece's bytes (piece_parts)
            for (int64_t at = 0; at < E; at++) {
                const uint32_t c = pcode[(size_t)at];
                const uint16_t pm = pperm[(size_t)at];
                const double v = pval[(size_t)at];
                if (ib == 2) {
                    const uint32_t w = c << 16 | pm;
                    if (sv == 4) {
                        const float f = (float)v;
                        memcpy(bp + at * 8, &w, 4);
                        memcpy(bp + at * 8 + 4, &f, 4);
                    } else {
                        memcpy(bp + at * 4, &w, 4);
                        memcpy(bp + pp.val + at * 8, &v, 8);
                    }
                } else {
                    memcpy(bp + at * 4, &c, 4);
                    memcpy(bp + pp.perm + at * 2, &pm, 2);
                    if (sv == 8) memcpy(bp + pp.val + at * 8, &v, 8);
                    else { const float f = (float)v; memcpy(bp + pp.val + at * 4, &f, 4); }
                }
            }
            out.positions += E;
            TileDesc td;
            td.base = base;
            td.len = len;
            td.chunk = (int32_t)g;
            td.ext = ext ? 1 : 0;
            td.flags = (q0 == 0 ? TILE_FIRST : 0) | (q0 + pc == tcnt ? TILE_LAST : 0);
            out.tiles.push_back(td);
        }
    }
}

// Pieces and tiles of the strictly-upper entries of rows [0, rows) under a
// geometry (only panels wholly inside the rows are counted).
static void count_tiles(const Geom &g, int64_t n, int64_t rows, const int64_t *rp, const int32_t *ci,
                        int64_t &pieces, int64_t &tiles) {
    pieces = tiles = 0;
    const int64_t cut = (int64_t)((g.maxe / g.G) & ~(SPMM_STEP - 1)) * g.G;
    if (cut < 1) return;
    std::vector<int32_t> cnt((size_t)((n + g.C - 1) / g.C), 0);
    std::vector<int64_t> touched;
    for (int64_t p = 0; (p + 1) * g.R <= rows; p++) {
        touched.clear();
        for (int64_t r = p * g.R; r < (p + 1) * g.R; r++)
            for (int64_t q = rp[r]; q < rp[r + 1]; q++) {
                if (ci[q] <= r || ci[q] >= n) continue;   // the panel builder reports bad columns
                const int64_t c = ci[q] / g.C;
                if (cnt[(size_t)c]++ == 0) touched.push_back(c);
            }
        for (int64_t c : touched) {
            tiles++;
            pieces += (cnt[(size_t)c] + cut - 1) / cut;
            cnt[(size_t)c] = 0;
        }
    }
}

// Panel geometry from the first rows of the matrix when none was given: the
// default rule's (geometry_for), or the tallest shorter panels with the same
// chunks whose pieces hold at least 1.5 times as many entries, when on these
// rows the taller panels cut enough tiles into several pieces.  In the SpMM a
// piece costs about twice a tile (the per-piece staging and barriers against
// the X chunk and transposed sums of an external tile; measured on CI-shaped
// matrices of 2 * 10^6 rows with 150 to 800 entries per row, fp32 storage,
// m = 16), so the shorter panels are taken when
// 2 * (pieces_tall - pieces_short) > tiles_short - tiles_tall.
static Geom choose_geometry(int storage, int m, int64_t n, int64_t rows, const int64_t *rp, const int32_t *ci) {
    const Geom a = geometry_for(storage, m, n, 0, 0);
    const int64_t sample = std::min<int64_t>(rows, 131072);
    Geom b;
    bool have_b = false;
    for (int R = a.R - a.C; R >= a.C && !have_b; R -= a.C) {
        if (R % 64) continue;
        try {
            b = geometry_for(storage, m, n, R / 64, a.cb);
        } catch (Error &) {
            continue;
        }
        have_b = 2 * (int64_t)b.maxe >= 3 * (int64_t)a.maxe;
    }
    if (!have_b || sample < 2 * (int64_t)a.R) return a;
    int64_t pa, ta, pb, tb;
    count_tiles(a, n, sample, rp, ci, pa, ta);
    count_tiles(b, n, sample, rp, ci, pb, tb);
    // compare per row: the two geometries count different numbers of whole panels
    const double ra = (double)(sample / a.R * a.R), rb = (double)(sample / b.R * b.R);
    const double cost_a = (2.0 * (double)pa + (double)ta) / ra, cost_b = (2.0 * (double)pb + (double)tb) / rb;
    return cost_b < cost_a ? b : a;
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
    Geom geo;
    int R = 0;
    int m = 16;
    bool geo_pending = false;    // geometry still to be chosen from the first rows
    int storage = HSYM_FP64;
    bool b64 = false;
    DevVec<double> preq, prelam;
    DevVec<float> preq32;          // the factors Q at fp32 storage
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
    DevVec<unsigned char> blob;
    std::vector<int64_t> panel_tile_ptr{0};
    std::vector<int64_t> panel_weight;  // per panel: padded entries + a per-piece cost, in entry units
    std::vector<double> diag;          // n
    std::vector<double> abssum;        // n: row+column absolute sums
    double norm1 = 0.0;
    int64_t nentries = 0, npieces = 0, ntiles = 0, next = 0, nbytes = 0;

    void release() {
        tiles.release(); blob.release();
        preq.release(); prelam.release(); preq32.release();
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
                    build_panel(n, r0, r1, geo, storage, b64, slab_row0, rp, ci, vin64, vin32,
                                diag.data() + r0, outs[(size_t)k]);
                }
            });
            // concatenate in panel order
            std::vector<TileDesc> t;
            std::vector<unsigned char> bl;
            std::vector<double> pq, pl;
            int64_t pos = 0;
            for (int64_t k = 0; k < b1 - b0; k++) {
                PanelOut &o = outs[(size_t)k];
                int64_t r0 = (b0 + k) * R;
                const int64_t byte_off = nbytes + (int64_t)bl.size();
                for (auto td : o.tiles) {
                    td.base += byte_off;
                    t.push_back(td);
                    if (td.flags & TILE_FIRST) ntiles++;
                }
                bl.insert(bl.end(), o.blob.begin(), o.blob.end());
                pos += o.positions;
                next += o.next;
                pq.insert(pq.end(), o.preq.begin(), o.preq.end());
                pl.insert(pl.end(), o.prelam.begin(), o.prelam.end());
                panel_tile_ptr.push_back(panel_tile_ptr.back() + (int64_t)o.tiles.size());
                {
                    // a piece's fixed cost (two barriers, staging, the transposed
                    // sums of an external tile) is about that of 600 entries
                    int64_t wgt = 600 * (int64_t)o.tiles.size();
                    for (const auto &td : o.tiles) wgt += (int64_t)td.len * geo.G;
                    panel_weight.push_back(wgt);
                }
                for (size_t w = 0; w < o.colsum.size(); w++) abssum[(size_t)r0 + w] += o.colsum[w];
                nnz += o.nnz;
                PanelOut().tiles.swap(o.tiles);
                std::vector<unsigned char>().swap(o.blob);
            }
            tiles.append(t.data(), (int64_t)t.size());
            blob.append(bl.data(), (int64_t)bl.size());
            if (b64) {
                if (storage == HSYM_FP32) {
                    // the preconditioner's factors in the storage precision
                    std::vector<float> q32(pq.begin(), pq.end());
                    preq32.append(q32.data(), (int64_t)q32.size());
                } else {
                    preq.append(pq.data(), (int64_t)pq.size());
                }
                prelam.append(pl.data(), (int64_t)pl.size());
            }
            npieces += (int64_t)t.size();
            nentries += pos;
            nbytes += (int64_t)bl.size();
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
        if (geo_pending) {
            // the first rows of the matrix (nothing is built or carried yet)
            geo = choose_geometry(storage, m, n, nrows, rp, ci);
            R = geo.R;
            geo_pending = false;
        }
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
    const Geom geo = geometry_for(H->storage, H->geom_m, H->n, H->geom_r64, H->geom_lc);
    std::unique_ptr<Builder> b(new Builder());
    b->n = H->n;
    b->storage = H->storage;
    b->m = H->geom_m;
    b->b64 = (H->flags & HSYM_BUILD_BLOCK64) != 0;
    b->geo = geo;
    b->R = geo.R;
    // without an explicit geometry the first appended rows decide the panels
    b->geo_pending = H->geom_r64 == 0;
    b->diag.assign((size_t)H->n, 0.0);
    b->abssum.assign((size_t)H->n, 0.0);
    if (nnz_hint > 0) {
        int64_t est = nnz_hint + nnz_hint / 8 + 4096;
        b->blob.reserve(est * ((int64_t)geo.idx_bytes + 2 + (H->storage == HSYM_FP64 ? 8 : 4)));
    }
    std::lock_guard<std::mutex> g(g_builders_mu);
    g_builders.push_back({H, b.release()});
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
    dt.g = b->geo;
    dt.npanels = (H->n + b->R - 1) / b->R;
    dt.nchunks = (H->n + b->geo.C - 1) / b->geo.C;
    dt.ntiles = b->ntiles; dt.npieces = b->npieces; dt.nentries = b->nentries; dt.next = b->next;
    dt.nbytes = b->nbytes;
    dt.tiles = b->tiles.p;
    dt.blob = b->blob.p;
    b->tiles.p = nullptr; b->blob.p = nullptr;
    dt.bytes = b->tiles.cap * (int64_t)sizeof(TileDesc) + b->blob.cap;
    // panel pointers
    HIPCHK(hipMalloc(&dt.panel_tile_ptr, sizeof(int64_t) * b->panel_tile_ptr.size()));
    HIPCHK(hipMemcpy(dt.panel_tile_ptr, b->panel_tile_ptr.data(), sizeof(int64_t) * b->panel_tile_ptr.size(),
                     hipMemcpyHostToDevice));
    dt.bytes += (int64_t)(sizeof(int64_t) * b->panel_tile_ptr.size());
    // workgroup -> panel.  The dispatcher deals workgroups round-robin to the
    // 8 XCDs (workgroup b to XCD b mod 8).  XCD x gets a contiguous run of
    // panels, so the X chunks and the rows of Y that neighbouring panels share
    // stay in its L2.  With few panels per CU it takes them heaviest first, so
    // that its CUs end on light panels (list scheduling; the panels' loads
    // differ by up to 2x); with many, in row order, which keeps more reuse in L2.
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
    // diagonal in both precisions and ||H||_1
    H->d_host = b->diag;
    std::vector<float> d32(b->diag.size());
    for (size_t i = 0; i < d32.size(); i++) d32[i] = (float)b->diag[i];
    HIPCHK(hipMalloc(&H->diag64, sizeof(double) * (size_t)H->n));
    HIPCHK(hipMalloc(&H->diag32, sizeof(float) * (size_t)H->n));
    HIPCHK(hipMemcpy(H->diag64, b->diag.data(), sizeof(double) * (size_t)H->n, hipMemcpyHostToDevice));
    HIPCHK(hipMemcpy(H->diag32, d32.data(), sizeof(float) * (size_t)H->n, hipMemcpyHostToDevice));
    if (b->b64) {
        H->pre_q32 = H->storage == HSYM_FP32;
        H->pre_q = H->pre_q32 ? (void *)b->preq32.p : (void *)b->preq.p;
        H->pre_lam = b->prelam.p;
        H->pre_nchunks = (H->n + 63) / 64;
        dt.bytes += b->preq.cap * 8 + b->preq32.cap * 4 + b->prelam.cap * 8;
        b->preq.p = nullptr; b->preq32.p = nullptr; b->prelam.p = nullptr;
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
    void *ptrs[] = {dt->panel_tile_ptr, dt->panel_order, dt->tiles, dt->blob};
    for (void *p : ptrs) if (p) (void)hipFree(p);
    *dt = DeviceTiles();
}

}  // namespace hsym
