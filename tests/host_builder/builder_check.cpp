// Host check of the tile builder (paper_1609_01689_amd/csrc/build.cpp), built
// with g++ against a host stand-in of the HIP runtime so that it runs under
// AddressSanitizer and UBSan without a GPU.  It builds a handle's tile streams
// from upper CSR (whole or in slabs), checks the invariants the SpMM kernel
// relies on, and replays the kernel's two passes over the streams on the CPU
// (same staged indexing, same run logic) to compare H X with the product
// computed from the CSR directly.
//
// usage: builder_check <case> <n> <N> <seed> <storage 0|1> <m> <slab> <r64> <lc>
//   case: gen (synthetic CI-shaped matrix), diag (diagonal only), holes (empty
//   rows, missing diagonals, a trailing empty stretch), dense (full upper
//   triangle); slab 0 = one append; r64/lc 0 = automatic geometry.
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "hsym_internal.h"

extern "C" {
void *hsg_create(int64_t n, double target_nnz_row, uint64_t seed, int64_t window, double rho, double rho_diag,
                 double sigma, int variant);
void hsg_destroy(void *h);
void hsg_count_rows(void *h, int64_t r0, int64_t r1, int64_t *counts);
void hsg_fill_rows(void *h, int64_t r0, int64_t r1, const int64_t *rowptr_local, int32_t *colind, double *vals_d,
                   float *vals_f);
}

namespace hsym {
void set_error(const std::string &) {}
void fail(int status, const std::string &msg) { throw Error{status, msg}; }
void check_hip(hipError_t e, const char *what) {
    if (e != hipSuccess) fail(HSYM_E_DEVICE, what);
}
void builder_begin(hsym_matrix *H, int64_t nnz_hint);
void builder_append(hsym_matrix *H, int64_t nrows, const int64_t *rp, const int32_t *ci, const void *vals,
                    int vprec);
void builder_finish(hsym_matrix *H);
void builder_discard(hsym_matrix *H);
}  // namespace hsym

using namespace hsym;

static int g_bad = 0;
#define REQUIRE(c, ...)                                 \
    do {                                                \
        if (!(c)) {                                     \
            if (g_bad < 10) {                           \
                std::printf("violation: " __VA_ARGS__); \
                std::printf("\n");                      \
            }                                           \
            g_bad++;                                    \
        }                                               \
    } while (0)

struct CSR {
    int64_t n = 0;
    std::vector<int64_t> rp;
    std::vector<int32_t> ci;
    std::vector<double> v;
};

static CSR make(const std::string &kind, int64_t n, double N, uint64_t seed) {
    CSR A;
    A.n = n;
    A.rp.assign((size_t)n + 1, 0);
    if (kind == "gen") {
        void *h = hsg_create(n, N, seed, 64, 0.24, 0.5, 0.3, 0);
        std::vector<int64_t> cnt((size_t)n);
        hsg_count_rows(h, 0, n, cnt.data());
        for (int64_t i = 0; i < n; i++) A.rp[(size_t)i + 1] = A.rp[(size_t)i] + cnt[(size_t)i];
        A.ci.resize((size_t)A.rp[(size_t)n]);
        A.v.resize(A.ci.size());
        hsg_fill_rows(h, 0, n, A.rp.data(), A.ci.data(), A.v.data(), nullptr);
        hsg_destroy(h);
        return A;
    }
    // small deterministic patterns with values from a fixed LCG
    uint64_t s = seed * 6364136223846793005ULL + 1442695040888963407ULL;
    auto val = [&]() {
        s = s * 6364136223846793005ULL + 1442695040888963407ULL;
        return ((double)(s >> 11) / 9007199254740992.0) - 0.5;
    };
    for (int64_t i = 0; i < n; i++) {
        if (kind == "diag") {
            A.ci.push_back((int32_t)i);
            A.v.push_back(1.0 + val());
        } else if (kind == "holes") {
            // rows i % 5 == 3 empty; no diagonal on odd rows; the last quarter empty
            if (i % 5 != 3 && i < n - n / 4) {
                if (i % 2 == 0) { A.ci.push_back((int32_t)i); A.v.push_back(2.0 + val()); }
                for (int64_t j = i + 1 + (i % 7); j < n; j += 3 + (i % 11)) {
                    A.ci.push_back((int32_t)j);
                    A.v.push_back(val());
                }
            }
        } else if (kind == "dense") {
            for (int64_t j = i; j < n; j++) {
                A.ci.push_back((int32_t)j);
                A.v.push_back(j == i ? 4.0 + val() : val());
            }
        } else {
            std::printf("unknown case %s\n", kind.c_str());
            std::exit(2);
        }
        A.rp[(size_t)i + 1] = (int64_t)A.ci.size();
    }
    return A;
}

template <typename A_t, typename T, typename IT>
static void replay(const hsym_matrix *H, const std::vector<double> &X, int m, std::vector<double> &Y) {
    const DeviceTiles &dt = H->tiles;
    const Geom &g = dt.g;
    const int64_t n = H->n;
    const int M = round_m(m);
    const T *diag = H->storage == HSYM_FP64 ? (const T *)(const void *)H->diag64 : (const T *)(const void *)H->diag32;
    const int64_t total = dt.nbytes;
    Y.assign((size_t)(n * m), 0.0);
    std::vector<char> seen((size_t)dt.npanels, 0);
    for (int64_t b = 0; b < dt.npanels; b++) {
        const int64_t p = dt.panel_order[b];
        REQUIRE(p >= 0 && p < dt.npanels && !seen[(size_t)p], "panel order is not a permutation at %ld", (long)b);
        if (p < 0 || p >= dt.npanels) continue;
        seen[(size_t)p] = 1;
        const int64_t row0 = p * g.R;
        const int nrow = (int)std::min<int64_t>(g.R, n - row0);
        std::vector<A_t> xp((size_t)g.R * M, (A_t)0), xs((size_t)g.C * M, (A_t)0);
        std::vector<double> acc((size_t)g.R * M, 0.0), ts((size_t)g.C * M, 0.0);
        for (int r = 0; r < nrow; r++)
            for (int k = 0; k < m; k++) xp[(size_t)r * M + k] = (A_t)X[(size_t)((row0 + r) * m + k)];
        bool open_ext = false;
        for (int64_t t = dt.panel_tile_ptr[p]; t < dt.panel_tile_ptr[p + 1]; t++) {
            const TileDesc td = dt.tiles[t];
            const int64_t E = (int64_t)g.G * td.len;
            const int64_t col0 = (int64_t)td.chunk * g.C;
            const PieceParts pp = piece_parts(E, (int)sizeof(IT), (int)sizeof(T));
            const int64_t bytes = pp.bytes;
            REQUIRE(td.base % 16 == 0, "piece base %ld not a multiple of 16", (long)td.base);
            REQUIRE(td.len >= 1 && td.len % SPMM_STEP == 0 && E <= g.maxe, "piece of %ld positions (%d steps) exceeds %d",
                    (long)E, td.len, g.maxe);
            REQUIRE(td.base + bytes <= total, "piece at %ld overruns the stream", (long)td.base);
            REQUIRE(td.ext == (col0 >= row0 + g.R ? 1 : 0), "external flag of chunk %d in panel %ld", td.chunk, (long)p);
            REQUIRE(col0 >= row0 && col0 < n, "chunk %d outside the panel's column range", td.chunk);
            if (!(td.base % 16 == 0 && E <= g.maxe && td.base + bytes <= total)) return;
            const unsigned char *pb = dt.blob + td.base;
            if (td.flags & TILE_FIRST) {
                REQUIRE(!open_ext, "first piece inside an open tile");
                if (td.ext) {
                    for (int r = 0; r < g.C; r++)
                        for (int k = 0; k < M; k++)
                            xs[(size_t)r * M + k] =
                                (k < m && col0 + r < n) ? (A_t)X[(size_t)((col0 + r) * m + k)] : (A_t)0;
                }
            }
            open_ext = !(td.flags & TILE_LAST);
            const A_t *xsrc = td.ext ? xs.data() : xp.data() + (size_t)(col0 - row0) * M;
            // staged copies of the piece
            std::vector<uint32_t> sc((size_t)E);
            std::vector<int> sp((size_t)E);
            std::vector<T> sv((size_t)E);
            std::vector<int> hits((size_t)E, 0);
            for (int64_t e = 0; e < E; e++) {
                // the layouts of the piece format: 16-bit codes share a word
                // (code << 16 | perm) with the perm, fp32 values sit next to it
                if (sizeof(IT) == 2) {
                    uint32_t w;
                    std::memcpy(&w, pb + (sizeof(T) == 4 ? 8 : 4) * e, 4);
                    sc[(size_t)e] = w >> 16;
                    sp[(size_t)e] = (int)(w & 0xFFFFu);
                } else {
                    uint32_t c;
                    uint16_t pm;
                    std::memcpy(&c, pb + 4 * e, 4);
                    std::memcpy(&pm, pb + pp.perm + 2 * e, 2);
                    sc[(size_t)e] = c;
                    sp[(size_t)e] = pm;
                }
                std::memcpy(&sv[(size_t)e], pb + pp.val + (sizeof(IT) == 2 && sizeof(T) == 4 ? 8 : sizeof(T)) * e,
                            sizeof(T));
                const int r = (int)(sc[(size_t)e] >> g.cb), c = (int)(sc[(size_t)e] & (g.C - 1));
                REQUIRE(r < nrow && col0 + c < n && col0 + c > row0 + r, "code %u outside the tile", sc[(size_t)e]);
                REQUIRE(sp[(size_t)e] < E, "perm %d outside the piece", sp[(size_t)e]);
                if (sp[(size_t)e] < E) hits[(size_t)sp[(size_t)e]]++;
            }
            // every nonzero position appears exactly once in the column order
            for (int64_t e = 0; e < E; e++)
                if (sv[(size_t)e] != (T)0) REQUIRE(hits[(size_t)e] == 1, "position %ld in the column order %d times", (long)e, hits[(size_t)e]);
            // row pass
            for (int seg = 0; seg < g.G; seg++) {
                int cur = -1;
                std::vector<A_t> ra((size_t)M, (A_t)0);
                for (int s = 0; s < td.len; s++) {
                    const int64_t e = piece_pos(s, seg, g.G);
                    const int r = (int)(sc[(size_t)e] >> g.cb), c = (int)(sc[(size_t)e] & (g.C - 1));
                    if (r != cur) {
                        if (cur >= 0)
                            for (int k = 0; k < M; k++) { acc[(size_t)cur * M + k] += (double)ra[(size_t)k]; ra[(size_t)k] = 0; }
                        cur = r;
                    }
                    for (int k = 0; k < M; k++)
                        ra[(size_t)k] = std::fma((A_t)sv[(size_t)e], xsrc[(size_t)c * M + k], ra[(size_t)k]);
                }
                if (cur >= 0)
                    for (int k = 0; k < M; k++) acc[(size_t)cur * M + k] += (double)ra[(size_t)k];
            }
            // column pass
            double *tgt = td.ext ? ts.data() : acc.data() + (size_t)(col0 - row0) * M;
            int prevc = -1, prevr = -1;
            for (int seg = 0; seg < g.G; seg++) {
                int cur = -1;
                std::vector<A_t> ca((size_t)M, (A_t)0);
                for (int s = 0; s < td.len; s++) {
                    const int64_t q = (int64_t)seg * td.len + s;   // position in the column order
                    const int pe = sp[(size_t)piece_pos(s, seg, g.G)];
                    const int r = (int)(sc[(size_t)pe] >> g.cb), c = (int)(sc[(size_t)pe] & (g.C - 1));
                    if (sv[(size_t)pe] != (T)0) {
                        REQUIRE(c > prevc || (c == prevc && r > prevr), "column order broken at %ld", (long)q);
                        prevc = c;
                        prevr = r;
                    }
                    if (c != cur) {
                        if (cur >= 0)
                            for (int k = 0; k < M; k++) { tgt[(size_t)cur * M + k] += (double)ca[(size_t)k]; ca[(size_t)k] = 0; }
                        cur = c;
                    }
                    for (int k = 0; k < M; k++)
                        ca[(size_t)k] = std::fma((A_t)sv[(size_t)pe], xp[(size_t)r * M + k], ca[(size_t)k]);
                }
                if (cur >= 0)
                    for (int k = 0; k < M; k++) tgt[(size_t)cur * M + k] += (double)ca[(size_t)k];
            }
            if (td.ext && (td.flags & TILE_LAST)) {
                for (int r = 0; r < g.C; r++)
                    for (int k = 0; k < m; k++)
                        if (col0 + r < n) Y[(size_t)((col0 + r) * m + k)] += ts[(size_t)r * M + k];
                std::fill(ts.begin(), ts.end(), 0.0);
            }
        }
        REQUIRE(!open_ext, "panel %ld ends inside a tile", (long)p);
        for (int r = 0; r < nrow; r++)
            for (int k = 0; k < m; k++)
                Y[(size_t)((row0 + r) * m + k)] +=
                    acc[(size_t)r * M + k] + (double)diag[row0 + r] * (double)xp[(size_t)r * M + k];
    }
}

int main(int argc, char **argv) {
    if (argc != 10) {
        std::printf("usage: builder_check case n N seed storage m slab r64 lc\n");
        return 2;
    }
    const std::string kind = argv[1];
    const int64_t n = std::atoll(argv[2]);
    const double N = std::atof(argv[3]);
    const uint64_t seed = (uint64_t)std::atoll(argv[4]);
    const int storage = std::atoi(argv[5]), m = std::atoi(argv[6]);
    const int64_t slab = std::atoll(argv[7]);
    const int r64 = std::atoi(argv[8]), lc = std::atoi(argv[9]);
    CSR A = make(kind, n, N, seed);
    hsym_matrix H;
    H.n = n;
    H.storage = storage;
    H.geom_m = m;
    H.geom_r64 = r64;
    H.geom_lc = lc;
    try {
        builder_begin(&H, 0);
        if (slab <= 0) {
            builder_append(&H, n, A.rp.data(), A.ci.data(), A.v.data(), HSYM_FP64);
        } else {
            // uneven slabs: rebased row pointers per slab
            int64_t r = 0, k = 0;
            while (r < n) {
                const int64_t len = std::min<int64_t>(n - r, slab + (k++ % 3) * 17);
                std::vector<int64_t> rp((size_t)len + 1);
                for (int64_t i = 0; i <= len; i++) rp[(size_t)i] = A.rp[(size_t)(r + i)] - A.rp[(size_t)r];
                builder_append(&H, len, rp.data(), A.ci.data() + A.rp[(size_t)r], A.v.data() + A.rp[(size_t)r],
                               HSYM_FP64);
                r += len;
            }
        }
        builder_finish(&H);
    } catch (Error &e) {
        std::printf("builder error %d: %s\n", e.status, e.msg.c_str());
        return 1;
    }
    const Geom &g = H.tiles.g;
    std::printf("geometry R=%d C=%d G=%d maxe=%d code bytes %d; panels %ld, tiles %ld, pieces %ld, external %ld, "
                "positions %ld\n",
                g.R, g.C, g.G, g.maxe, g.idx_bytes, (long)H.tiles.npanels, (long)H.tiles.ntiles,
                (long)H.tiles.npieces, (long)H.tiles.next, (long)H.tiles.nentries);
    // X and the reference product from the CSR (both halves, diagonal once)
    std::vector<double> X((size_t)(n * m)), Yref((size_t)(n * m), 0.0), Yabs((size_t)(n * m), 0.0);
    for (size_t i = 0; i < X.size(); i++) X[i] = std::sin(0.37 * (double)i + 0.11) + 0.25;
    double maxabsH = 0.0;
    for (int64_t i = 0; i < n; i++) {
        for (int64_t q = A.rp[(size_t)i]; q < A.rp[(size_t)i + 1]; q++) {
            const int64_t j = A.ci[(size_t)q];
            const double a = storage == HSYM_FP64 ? A.v[(size_t)q] : (double)(float)A.v[(size_t)q];
            maxabsH = std::max(maxabsH, std::fabs(a));
            for (int k = 0; k < m; k++) {
                Yref[(size_t)(i * m + k)] += a * X[(size_t)(j * m + k)];
                Yabs[(size_t)(i * m + k)] += std::fabs(a * X[(size_t)(j * m + k)]);
                if (j != i) {
                    Yref[(size_t)(j * m + k)] += a * X[(size_t)(i * m + k)];
                    Yabs[(size_t)(j * m + k)] += std::fabs(a * X[(size_t)(i * m + k)]);
                }
            }
        }
    }
    // the diagonal the handle keeps
    for (int64_t i = 0; i < n; i++) {
        double d = 0.0;
        if (A.rp[(size_t)i + 1] > A.rp[(size_t)i] && A.ci[(size_t)A.rp[(size_t)i]] == i) d = A.v[(size_t)A.rp[(size_t)i]];
        REQUIRE(H.d_host[(size_t)i] == d, "diagonal of row %ld", (long)i);
    }
    int64_t offdiag = 0;
    for (int64_t i = 0; i < n; i++)
        for (int64_t q = A.rp[(size_t)i]; q < A.rp[(size_t)i + 1]; q++) offdiag += A.ci[(size_t)q] != i;
    std::vector<double> Y;
    const bool i16 = g.idx_bytes == 2;
    if (storage == HSYM_FP64) {
        if (i16) replay<double, double, uint16_t>(&H, X, m, Y);
        else replay<double, double, uint32_t>(&H, X, m, Y);
    } else {
        if (i16) replay<float, float, uint16_t>(&H, X, m, Y);
        else replay<float, float, uint32_t>(&H, X, m, Y);
    }
    // componentwise bound gamma_k(|H||X|) with k = the longest full row, in the
    // arithmetic precision (fp32 X staging adds one rounding of X)
    int64_t kmax = 1;
    {
        std::vector<int64_t> full((size_t)n, 0);
        for (int64_t i = 0; i < n; i++)
            for (int64_t q = A.rp[(size_t)i]; q < A.rp[(size_t)i + 1]; q++) {
                full[(size_t)i]++;
                if (A.ci[(size_t)q] != i) full[(size_t)A.ci[(size_t)q]]++;
            }
        for (int64_t f : full) kmax = std::max(kmax, f);
    }
    const double u = storage == HSYM_FP64 ? std::ldexp(1.0, -53) : std::ldexp(1.0, -24);
    const double gam = (double)(kmax + 2) * u / (1.0 - (double)(kmax + 2) * u);
    double worst = 0.0;
    for (size_t i = 0; i < Y.size(); i++) {
        const double err = std::fabs(Y[i] - Yref[i]);
        const double lim = gam * Yabs[i] + 1e-300;
        worst = std::max(worst, err / lim);
    }
    std::printf("off-diagonal entries %ld, longest row %ld, worst error / bound %.3f, violations %d\n",
                (long)offdiag, (long)kmax, worst, g_bad);
    builder_discard(&H);
    hsym::free_tiles(&H.tiles);
    std::free(H.diag64);
    std::free(H.diag32);
    std::free(H.pre_q);
    std::free(H.pre_lam);
    if (g_bad || !(worst <= 1.0)) {
        std::printf("FAIL\n");
        return 1;
    }
    std::printf("OK\n");
    return 0;
}
