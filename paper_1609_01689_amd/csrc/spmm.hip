// Symmetric SpMM from one stored triangle: Y = D X + U X + U^T X.
//
// Each stored off-diagonal entry is used twice, once as itself (row half,
// U X) and once transposed (U^T X): the two local products per stored block of
// Section 4.1.  The diagonal D is applied separately so it is counted once.
//
// One 1024-thread workgroup owns one row panel of R rows and walks its tiles
// (panel x chunk of C columns, Section 4.2) in column order, as the CSB
// traversal of Section 4.4 does.  LDS holds the panel's X rows and fp64
// accumulator, the current chunk's X rows and fp64 accumulator, and the staged
// entries of the current piece (codes, values and the column-order perm).
// Every piece is processed in two passes over its staged entries, each
// accumulating in registers:
//   - row pass: the entries in row-major order, cut into one segment per lane
//     group; a group keeps the sum of its current row run and gathers the X
//     row of each entry's column;
//   - column pass: the same entries in column-major order (through the perm);
//     a group keeps the sum of its current column run and gathers the X row of
//     each entry's row.
// A run's sum is added to its LDS accumulator row when the run ends, with
// fp64 LDS atomics (runs cut by a segment boundary have two owners); no
// per-entry atomics remain, and the X rows are read as whole rows by the
// lanes of a group (two elements per lane), which keeps the LDS banks free of
// conflicts.  While a piece runs, the next piece's entries and X chunk are
// already in flight into registers.
// Output: Y is cleared first; every panel adds its own rows and its external
// chunks' sums into Y with device-scope atomic adds.
// Precision: the arithmetic (X staged in LDS, products and run sums) is that
// of the storage: fp64, or fp32 for fp32 storage (the mixed form of Section
// 4.4, footnote 5).  Run sums are accumulated across runs in fp64.
#include <mutex>

#include "hsym_internal.h"

namespace hsym {

constexpr int SPMM_NT = 1024;
constexpr int SPMM_XE = 4;   // X chunk elements per thread (C * M <= 4096)

template <int M, typename A>
struct Lay {
    static constexpr int SA = (int)sizeof(A);
    static constexpr int MW = spmm_lane_elems(M);            // elements per lane
    static constexpr int L = M / MW;                         // lanes per row
    static constexpr int GK = SPMM_NT / L;                   // lane groups
};

struct SpmmArgs {
    const int64_t *ptp;
    const int32_t *porder;
    const TileDesc *tiles;
    const unsigned char *blob;
    const void *diag;
    const void *X;
    int64_t ldx;
    void *Y;
    int64_t ldy;
    int64_t n;
    int64_t npanels;
    Geom g;
    int m;
};

// MW consecutive elements of an LDS row (32, 16, 8 or 4 bytes)
template <int MW, typename A>
__device__ __forceinline__ void lds_get(const A *p, A *o) {
    if constexpr (MW * sizeof(A) == 32 && sizeof(A) == 8) {
        const double2 v = *reinterpret_cast<const double2 *>(p);
        const double2 w = *reinterpret_cast<const double2 *>(p + 2);
        o[0] = v.x; o[1] = v.y; o[2] = w.x; o[3] = w.y;
    } else if constexpr (MW * sizeof(A) == 32) {
        const float4 v = *reinterpret_cast<const float4 *>(p);
        const float4 w = *reinterpret_cast<const float4 *>(p + 4);
        o[0] = v.x; o[1] = v.y; o[2] = v.z; o[3] = v.w;
        o[4] = w.x; o[5] = w.y; o[6] = w.z; o[7] = w.w;
    } else if constexpr (MW * sizeof(A) == 16 && sizeof(A) == 8) {
        const double2 v = *reinterpret_cast<const double2 *>(p);
        o[0] = v.x; o[1] = v.y;
    } else if constexpr (MW * sizeof(A) == 16) {
        const float4 v = *reinterpret_cast<const float4 *>(p);
        o[0] = v.x; o[1] = v.y; o[2] = v.z; o[3] = v.w;
    } else if constexpr (MW == 2 && sizeof(A) == 4) {
        const float2 v = *reinterpret_cast<const float2 *>(p);
        o[0] = v.x; o[1] = v.y;
    } else {
#pragma unroll
        for (int j = 0; j < MW; j++) o[j] = p[j];
    }
}

template <int MW, typename A>
__device__ __forceinline__ void run_flush(double *row, A *s) {
#pragma unroll
    for (int j = 0; j < MW; j++) {
        __hip_atomic_fetch_add(row + j, (double)s[j], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
        s[j] = (A)0;
    }
}

template <typename YT>
__device__ __forceinline__ void y_add(YT *p, double v) {
    unsafeAtomicAdd(p, (YT)v);
}

// Reads of a staged piece in LDS (the three layouts of the piece format):
// entry2(e) gives the words holding the codes of row-major positions e and
// e + 1 (e even; the code sits CS bits up in a word) and their values;
// perm2(k) the row-major positions of column-major positions k and k + 1;
// word(e) the word of one position.
template <typename T, typename IT>
struct Staged;
template <>
struct Staged<float, uint16_t> {   // 8-byte records {code << 16 | perm, value}
    static constexpr int CS = 16;
    const uint2 *rec;
    __device__ Staged(const unsigned char *s, int) : rec(reinterpret_cast<const uint2 *>(s)) {}
    __device__ __forceinline__ void entry2(int e, uint32_t *w, float *v) const {
        const uint4 r = *reinterpret_cast<const uint4 *>(rec + e);
        w[0] = r.x; v[0] = __uint_as_float(r.y);
        w[1] = r.z; v[1] = __uint_as_float(r.w);
    }
    __device__ __forceinline__ void entry(int e, uint32_t &w, float &v) const {
        const uint2 r = rec[e];
        w = r.x;
        v = __uint_as_float(r.y);
    }
    __device__ __forceinline__ uint32_t word(int e) const { return rec[e].x; }
    __device__ __forceinline__ void perm2(int k, int *p) const {
        p[0] = (int)(rec[k].x & 0xFFFFu);
        p[1] = (int)(rec[k + 1].x & 0xFFFFu);
    }
};
template <>
struct Staged<double, uint16_t> {  // words code << 16 | perm, then the values
    static constexpr int CS = 16;
    const uint32_t *wd;
    const double *val;
    __device__ Staged(const unsigned char *s, int E)
        : wd(reinterpret_cast<const uint32_t *>(s)),
          val(reinterpret_cast<const double *>(s + piece_parts(E, 2, 8).val)) {}
    __device__ __forceinline__ void entry2(int e, uint32_t *w, double *v) const {
        const uint2 r = *reinterpret_cast<const uint2 *>(wd + e);
        const double2 d = *reinterpret_cast<const double2 *>(val + e);
        w[0] = r.x; w[1] = r.y;
        v[0] = d.x; v[1] = d.y;
    }
    __device__ __forceinline__ void entry(int e, uint32_t &w, double &v) const {
        w = wd[e];
        v = val[e];
    }
    __device__ __forceinline__ uint32_t word(int e) const { return wd[e]; }
    __device__ __forceinline__ void perm2(int k, int *p) const {
        const uint2 r = *reinterpret_cast<const uint2 *>(wd + k);
        p[0] = (int)(r.x & 0xFFFFu);
        p[1] = (int)(r.y & 0xFFFFu);
    }
};
template <typename T>
struct Staged<T, uint32_t> {       // codes, perm (16-bit), values
    static constexpr int CS = 0;
    const uint32_t *code;
    const uint16_t *pm;
    const T *val;
    __device__ Staged(const unsigned char *s, int E) {
        const PieceParts pp = piece_parts(E, 4, (int)sizeof(T));
        code = reinterpret_cast<const uint32_t *>(s);
        pm = reinterpret_cast<const uint16_t *>(s + pp.perm);
        val = reinterpret_cast<const T *>(s + pp.val);
    }
    __device__ __forceinline__ void entry2(int e, uint32_t *w, T *v) const {
        const uint2 r = *reinterpret_cast<const uint2 *>(code + e);
        w[0] = r.x; w[1] = r.y;
        v[0] = val[e]; v[1] = val[e + 1];
    }
    __device__ __forceinline__ void entry(int e, uint32_t &w, T &v) const {
        w = code[e];
        v = val[e];
    }
    __device__ __forceinline__ uint32_t word(int e) const { return code[e]; }
    __device__ __forceinline__ void perm2(int k, int *p) const {
        const uint32_t r = *reinterpret_cast<const uint32_t *>(pm + k);
        p[0] = (int)(r & 0xFFFFu);
        p[1] = (int)(r >> 16);
    }
};

// Load a piece into registers: 16-byte units of its bytes (thread tid takes
// units tid, tid + 1024, ...), and the X chunk of an external tile's first
// piece (element i = tid + k * 1024 of the C x M chunk).
template <int M, typename XT, int KU>
__device__ __forceinline__ void spmm_fetch(const SpmmArgs &a, const TileDesc &td, int nunits, uint4 &u0, uint4 &u1,
                                           uint4 &u2, uint4 &u3, uint4 &u4, uint4 &u5, uint4 &u6, uint4 &u7, XT &x0,
                                           XT &x1, XT &x2, XT &x3) {
    const int tid = threadIdx.x;
    const uint4 *g = reinterpret_cast<const uint4 *>(a.blob + td.base);
    if (tid < nunits) u0 = g[tid];
    if (tid + SPMM_NT < nunits) u1 = g[tid + SPMM_NT];
    if (tid + 2 * SPMM_NT < nunits) u2 = g[tid + 2 * SPMM_NT];
    if (tid + 3 * SPMM_NT < nunits) u3 = g[tid + 3 * SPMM_NT];
    if constexpr (KU > 4) {
        if (tid + 4 * SPMM_NT < nunits) u4 = g[tid + 4 * SPMM_NT];
        if (tid + 5 * SPMM_NT < nunits) u5 = g[tid + 5 * SPMM_NT];
        if (tid + 6 * SPMM_NT < nunits) u6 = g[tid + 6 * SPMM_NT];
        if (tid + 7 * SPMM_NT < nunits) u7 = g[tid + 7 * SPMM_NT];
    }
    if (td.ext && (td.flags & TILE_FIRST)) {
        const XT *X = reinterpret_cast<const XT *>(a.X);
        const int C = a.g.C, m = a.m;
        const int64_t col0 = (int64_t)td.chunk * C;
        auto getx = [&](int i, XT &d) {
            const int r = i / M, c = i - r * M;
            d = (XT)0;
            if (i < C * M && c < m && col0 + r < a.n) d = X[(col0 + r) * a.ldx + c];
        };
        getx(tid, x0);
        getx(tid + SPMM_NT, x1);
        getx(tid + 2 * SPMM_NT, x2);
        getx(tid + 3 * SPMM_NT, x3);
    }
}

template <int M, typename T, typename A, typename XT, typename YT, typename IT, int KU>
__device__ __forceinline__ void spmm_panel_body(const SpmmArgs &a, int64_t blk, unsigned char *smem) {
    using Ly = Lay<M, A>;
    constexpr int MW = Ly::MW, L = Ly::L, GK = Ly::GK, SA = Ly::SA;
    constexpr int IB = (int)sizeof(IT), SV = (int)sizeof(T);
    const int R = a.g.R, C = a.g.C, G = a.g.G, cb = a.g.cb, m = a.m;
    const uint32_t cm = (uint32_t)C - 1u;
    const int tid = threadIdx.x, grp = tid / L, q = tid - grp * L;
    // LDS layout (byte offsets): acc, ts (fp64), xp, xs (A), codes, perm, values
    double *acc = reinterpret_cast<double *>(smem);
    double *ts = acc + (size_t)R * M;
    constexpr int XS = M + spmm_xpad(M);   // staged X row stride (padded)
    A *xp = reinterpret_cast<A *>(ts + (size_t)C * M);
    A *xs = xp + (size_t)R * XS;
    // the staged piece: its bytes as stored (codes, perm, values; the offsets
    // of the last two depend on the piece's size)
    unsigned char *stg = smem + (size_t)(R + C) * ((size_t)M * 8 + (size_t)XS * SA);
    // 16-byte units of a piece of len steps
    auto units = [&](int len) { return (int)(piece_parts((int64_t)G * len, IB, SV).bytes >> 4); };

    const XT *X = reinterpret_cast<const XT *>(a.X);
    YT *Y = reinterpret_cast<YT *>(a.Y);
    const int64_t p = a.porder[blk];
    const int64_t row0 = p * (int64_t)R;
    const int nrow = (int)((a.n - row0) < R ? (a.n - row0) : R);

    for (int i = tid; i < R * M; i += SPMM_NT) {
        const int r = i / M, k = i - r * M;
        A v = (A)0;
        if (r < nrow && k < m) v = (A)X[(row0 + r) * a.ldx + k];
        xp[r * XS + k] = v;
        acc[i] = 0.0;
    }
    for (int i = tid; i < C * M; i += SPMM_NT) ts[i] = 0.0;

    const int64_t t0 = a.ptp[p], t1 = a.ptp[p + 1];
    // registers holding the next piece: 16-byte units of its three streams,
    // and (first piece of an external tile) its X chunk
    // (the first KU of the eight are used; named registers, not an array,
    // which the compiler would place in scratch memory)
    uint4 su0, su1, su2, su3, su4, su5, su6, su7;
    XT xr0 = (XT)0, xr1 = (XT)0, xr2 = (XT)0, xr3 = (XT)0;
    static_assert(SPMM_XE == 4, "X chunk registers are unrolled by hand");
    // descriptors travel one piece ahead of the data they describe, so that
    // no wait on memory sits between two pieces
    // (scalar loads through the constant address space: they do not wait
    // behind the vector loads of the staged pieces)
    typedef __attribute__((address_space(4))) const TileDesc ConstTile;
    ConstTile *ctiles = (ConstTile *)a.tiles;
    auto tile_at = [&](int64_t t) {
        TileDesc r;
        r.base = ctiles[t].base;
        r.len = ctiles[t].len;
        r.chunk = ctiles[t].chunk;
        r.ext = ctiles[t].ext;
        r.flags = ctiles[t].flags;
        return r;
    };
    TileDesc tdc{}, tdn{};
    if (t0 < t1) {
        tdc = tile_at(t0);
        spmm_fetch<M, XT, KU>(a, tdc, units(tdc.len), su0, su1, su2, su3, su4, su5, su6, su7, xr0, xr1, xr2, xr3);
        if (t0 + 1 < t1) tdn = tile_at(t0 + 1);
    }

    // the chunk's transposed sums go into Y; each thread clears what it read,
    // for the next external tile
    int64_t flush_col0 = -1;
    auto flush_ts = [&](int64_t c0) {
        for (int i = tid; i < C * M; i += SPMM_NT) {
            const int r = i / M, k = i - r * M;
            const double v = ts[i];
            if (k < m && c0 + r < a.n) y_add<YT>(Y + (c0 + r) * a.ldy + k, v);
            ts[i] = 0.0;
        }
    };

    for (int64_t t = t0; t < t1; t++) {
        const TileDesc td = tdc;
        // the staged piece's loads, issued one piece ago, and the previous
        // tile's atomics are complete here on every path (s_waitcnt vmcnt(0),
        // gfx9 encoding): the loads of the next piece then need no further
        // wait before the barrier
        __builtin_amdgcn_s_waitcnt(0x0F70);
        if (flush_col0 >= 0) {
            flush_ts(flush_col0);
            flush_col0 = -1;
        }
        const int len = td.len;
        const int64_t col0 = (int64_t)td.chunk * C;
        const int nunits = units(len);
        {
            uint4 *sdst = reinterpret_cast<uint4 *>(stg);
            if (tid < nunits) sdst[tid] = su0;
            if (tid + SPMM_NT < nunits) sdst[tid + SPMM_NT] = su1;
            if (tid + 2 * SPMM_NT < nunits) sdst[tid + 2 * SPMM_NT] = su2;
            if (tid + 3 * SPMM_NT < nunits) sdst[tid + 3 * SPMM_NT] = su3;
            if constexpr (KU > 4) {
                if (tid + 4 * SPMM_NT < nunits) sdst[tid + 4 * SPMM_NT] = su4;
                if (tid + 5 * SPMM_NT < nunits) sdst[tid + 5 * SPMM_NT] = su5;
                if (tid + 6 * SPMM_NT < nunits) sdst[tid + 6 * SPMM_NT] = su6;
                if (tid + 7 * SPMM_NT < nunits) sdst[tid + 7 * SPMM_NT] = su7;
            }
            if (td.ext && (td.flags & TILE_FIRST)) {
                // element i of the chunk (row i / M, column i % M) at its padded place
                auto xput = [&](int i, XT v) {
                    if (i < C * M) xs[(i / M) * XS + i % M] = (A)v;
                };
                xput(tid, xr0);
                xput(tid + SPMM_NT, xr1);
                xput(tid + 2 * SPMM_NT, xr2);
                xput(tid + 3 * SPMM_NT, xr3);
            }
        }
        if (t + 1 < t1) {
            spmm_fetch<M, XT, KU>(a, tdn, units(tdn.len), su0, su1, su2, su3, su4, su5, su6, su7, xr0, xr1, xr2, xr3);
            tdc = tdn;
            if (t + 2 < t1) tdn = tile_at(t + 2);
        }
        __syncthreads();

        const Staged<T, IT> sp(stg, G * len);
        constexpr int CS = Staged<T, IT>::CS;
        const int rs = CS + cb;   // the local row sits rs bits up in a word
        static_assert(SPMM_STEP == 2, "the passes take two steps per batch");
        // row pass: U X
        {
            const A *xsrc = td.ext ? xs : xp + (size_t)(col0 - row0) * XS;
            for (int seg = grp; seg < G; seg += GK) {
                A ra[MW];
#pragma unroll
                for (int j = 0; j < MW; j++) ra[j] = (A)0;
                int cur = (int)(sp.word(2 * seg) >> rs);
                for (int e = 2 * seg, s0 = 0; s0 < len; s0 += 2, e += 2 * G) {
                    uint32_t w[2];
                    T v[2];
                    A av[2], xv[2][MW];
                    sp.entry2(e, w, v);
#pragma unroll
                    for (int u = 0; u < 2; u++) av[u] = (A)v[u];
#pragma unroll
                    for (int u = 0; u < 2; u++)
                        lds_get<MW, A>(xsrc + (size_t)((w[u] >> CS) & cm) * XS + q * MW, xv[u]);
#pragma unroll
                    for (int u = 0; u < 2; u++) {
                        const int r = (int)(w[u] >> rs);
                        if (r != cur) {
                            run_flush<MW, A>(acc + (size_t)cur * M + q * MW, ra);
                            cur = r;
                        }
#pragma unroll
                        for (int j = 0; j < MW; j++) ra[j] = fma(av[u], xv[u][j], ra[j]);
                    }
                }
                run_flush<MW, A>(acc + (size_t)cur * M + q * MW, ra);
            }
        }
        // column pass: U^T X, into the chunk accumulator (external tile) or
        // the panel accumulator (own tile)
        {
            double *tgt = td.ext ? ts : acc + (size_t)(col0 - row0) * M;
            for (int seg = grp; seg < G; seg += GK) {
                A ca[MW];
#pragma unroll
                for (int j = 0; j < MW; j++) ca[j] = (A)0;
                int cur;
                {
                    int p0[2];
                    sp.perm2(2 * seg, p0);
                    cur = (int)((sp.word(p0[0]) >> CS) & cm);
                }
                for (int k = 2 * seg, s0 = 0; s0 < len; s0 += 2, k += 2 * G) {
                    int pe[2];
                    uint32_t w[2];
                    A av[2], xv[2][MW];
                    sp.perm2(k, pe);
#pragma unroll
                    for (int u = 0; u < 2; u++) {
                        T v;
                        sp.entry(pe[u], w[u], v);
                        av[u] = (A)v;
                    }
#pragma unroll
                    for (int u = 0; u < 2; u++) lds_get<MW, A>(xp + (size_t)(w[u] >> rs) * XS + q * MW, xv[u]);
#pragma unroll
                    for (int u = 0; u < 2; u++) {
                        const int c = (int)((w[u] >> CS) & cm);
                        if (c != cur) {
                            run_flush<MW, A>(tgt + (size_t)cur * M + q * MW, ca);
                            cur = c;
                        }
#pragma unroll
                        for (int j = 0; j < MW; j++) ca[j] = fma(av[u], xv[u][j], ca[j]);
                    }
                }
                run_flush<MW, A>(tgt + (size_t)cur * M + q * MW, ca);
            }
        }
        __syncthreads();
        // an external tile's sums are complete: they go into Y at the start
        // of the next piece (or after the last), so that the atomics are in
        // flight while that piece runs
        if (td.ext && (td.flags & TILE_LAST)) flush_col0 = col0;
    }
    if (flush_col0 >= 0) flush_ts(flush_col0);
    const T *diag = reinterpret_cast<const T *>(a.diag);
    for (int i = tid; i < nrow * M; i += SPMM_NT) {
        const int r = i / M, k = i - r * M;
        if (k < m) {
            const int64_t row = row0 + r;
            y_add<YT>(Y + row * a.ldy + k, acc[i] + (double)diag[row] * (double)xp[r * XS + k]);
        }
    }
}

template <int M, typename T, typename A, typename XT, typename YT, typename IT, int KU>
__global__ __launch_bounds__(SPMM_NT) void k_spmm_panel(SpmmArgs a) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    spmm_panel_body<M, T, A, XT, YT, IT, KU>(a, blockIdx.x, smem_raw);
}

// batched over matrices (fp64 blocks): blockIdx.y selects the job
template <int M, typename T, typename A>
__global__ __launch_bounds__(SPMM_NT) void k_spmm_panel_b(const SpmmJob *__restrict__ jobs) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const SpmmJob J = jobs[blockIdx.y];
    if ((int64_t)blockIdx.x >= J.npanels) return;
    SpmmArgs a;
    a.ptp = J.ptp; a.porder = J.porder; a.tiles = J.tiles; a.blob = J.blob;
    a.diag = J.diag; a.X = J.X; a.ldx = J.ldx; a.Y = J.Y; a.ldy = J.ldy; a.n = J.n; a.npanels = J.npanels;
    a.g = J.g; a.m = J.m;
    // the code width is a property of each job's handle (uniform per workgroup)
    constexpr int KU = spmm_stage_units(M);
    if (J.g.idx_bytes == 2) spmm_panel_body<M, T, A, double, double, uint16_t, KU>(a, blockIdx.x, smem_raw);
    else spmm_panel_body<M, T, A, double, double, uint32_t, KU>(a, blockIdx.x, smem_raw);
}

// Y[r][0..m) = 0 for r < n (leading dimension ldy): the SpMM adds into Y (a
// kernel rather than a memset, so a graph may record it)
template <typename YT>
__global__ __launch_bounds__(256) void k_zero_rows(YT *__restrict__ Y, int64_t n, int m, int64_t ldy) {
    const int64_t cnt = n * m;
    for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < cnt; e += (int64_t)gridDim.x * 256) {
        const int64_t r = e / m;
        Y[r * ldy + (e - r * m)] = (YT)0;
    }
}

__global__ __launch_bounds__(256) void k_zero_rows_b(const SpmmJob *__restrict__ jobs) {
    const SpmmJob J = jobs[blockIdx.y];
    const int64_t cnt = J.n * J.m;
    for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < cnt; e += (int64_t)gridDim.x * 256) {
        const int64_t r = e / J.m;
        J.Y[r * J.ldy + (e - r * J.m)] = 0.0;
    }
}

template <typename YT>
static void zero_rows(YT *Y, int64_t n, int m, int64_t ldy, hipStream_t s) {
    const int64_t blocks = std::min<int64_t>((n * m + 255) / 256, 4096);
    hipLaunchKernelGGL(k_zero_rows<YT>, dim3((unsigned)std::max<int64_t>(blocks, 1)), dim3(256), 0, s, Y, n, m, ldy);
    HIPCHK(hipGetLastError());
}

// Checks that a call of width m fits the handle's geometry; returns the
// staging units per thread its pieces need (4 or 8).
static int check_fit(int storage, int m, const Geom &g) {
    const int M = round_m(m);
    if (spmm_lds_bytes(storage, m, g) > 160 * 1024)
        fail(HSYM_E_UNSUPPORTED, "block width too large for this handle's panel geometry");
    if ((size_t)g.C * M > (size_t)SPMM_XE * SPMM_NT)
        fail(HSYM_E_UNSUPPORTED, "chunk too wide for this block width");
    const int64_t e = g.maxe, sv = storage == HSYM_FP64 ? 8 : 4;
    const int64_t bytes = piece_parts(e, g.idx_bytes, (int)sv).bytes;
    const int64_t units = (bytes / 16 + SPMM_NT - 1) / SPMM_NT;
    if (units > 8) fail(HSYM_E_UNSUPPORTED, "pieces too large for the staging registers");
    return units > 4 ? 8 : 4;
}

template <int M, typename T, typename A, typename XT, typename YT, typename IT, int KU>
static void launch_typed(hsym_matrix *H, int m, const void *X, int64_t ldx, void *Y, int64_t ldy, hipStream_t s) {
    const DeviceTiles &dt = H->tiles;
    const size_t lds = spmm_lds_bytes(H->storage, m, dt.g);
    auto kp = k_spmm_panel<M, T, A, XT, YT, IT, KU>;
    static std::once_flag attr_once;   // the 160 KB LDS limit, set once (threads may launch concurrently)
    std::call_once(attr_once, [&] {
        HIPCHK(hipFuncSetAttribute((const void *)kp, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024));
    });
    SpmmArgs a;
    a.ptp = dt.panel_tile_ptr; a.porder = dt.panel_order; a.tiles = dt.tiles; a.blob = dt.blob;
    a.diag = H->storage == HSYM_FP64 ? (const void *)H->diag64 : (const void *)H->diag32;
    a.X = X; a.ldx = ldx; a.Y = Y; a.ldy = ldy; a.n = H->n; a.npanels = dt.npanels; a.g = dt.g; a.m = m;
    zero_rows<YT>((YT *)Y, H->n, m, ldy, s);
    hipLaunchKernelGGL(kp, dim3((unsigned)dt.npanels), dim3(SPMM_NT), lds, s, a);
    HIPCHK(hipGetLastError());
}

// pieces of a handle built for block width 1 or 2 need 8 staging units per
// thread; a wider call on such a handle takes the 8-unit kernel of its width
template <int M, typename T, typename A, typename XT, typename YT, typename IT>
static void launch_ku(hsym_matrix *H, int m, const void *X, int64_t ldx, void *Y, int64_t ldy, int ku,
                      hipStream_t s) {
    if (ku > 4) launch_typed<M, T, A, XT, YT, IT, 8>(H, m, X, ldx, Y, ldy, s);
    else launch_typed<M, T, A, XT, YT, IT, spmm_stage_units(M)>(H, m, X, ldx, Y, ldy, s);
}

template <typename T, typename A, typename XT, typename YT, typename IT>
static void launch_mi(hsym_matrix *H, int m, const void *X, int64_t ldx, void *Y, int64_t ldy, int ku,
                      hipStream_t s) {
    switch (round_m(m)) {
        case 1: launch_ku<1, T, A, XT, YT, IT>(H, m, X, ldx, Y, ldy, ku, s); break;
        case 2: launch_ku<2, T, A, XT, YT, IT>(H, m, X, ldx, Y, ldy, ku, s); break;
        case 4: launch_ku<4, T, A, XT, YT, IT>(H, m, X, ldx, Y, ldy, ku, s); break;
        case 8: launch_ku<8, T, A, XT, YT, IT>(H, m, X, ldx, Y, ldy, ku, s); break;
        default: launch_ku<16, T, A, XT, YT, IT>(H, m, X, ldx, Y, ldy, ku, s); break;
    }
}

template <typename T, typename A, typename XT, typename YT>
static void launch_m(hsym_matrix *H, int m, const void *X, int64_t ldx, void *Y, int64_t ldy, int ku,
                     hipStream_t s) {
    if (H->tiles.g.idx_bytes == 2) launch_mi<T, A, XT, YT, uint16_t>(H, m, X, ldx, Y, ldy, ku, s);
    else launch_mi<T, A, XT, YT, uint32_t>(H, m, X, ldx, Y, ldy, ku, s);
}

SpmmJob spmm_job(hsym_matrix *H, int m, const double *X, double *Y) {
    const DeviceTiles &dt = H->tiles;
    SpmmJob J{};
    J.ptp = dt.panel_tile_ptr; J.porder = dt.panel_order; J.tiles = dt.tiles; J.blob = dt.blob;
    J.diag = H->storage == HSYM_FP64 ? (const void *)H->diag64 : (const void *)H->diag32;
    J.X = X; J.ldx = m; J.Y = Y; J.ldy = m;
    J.n = H->n; J.npanels = dt.npanels; J.g = dt.g; J.m = m;
    return J;
}

template <int M, typename T, typename A>
static void batched_typed(const SpmmJob *jobs, const SpmmJob *host, int count, int storage, hipStream_t s) {
    size_t lds = 0;
    int64_t maxp = 0, maxn = 0;
    for (int i = 0; i < count; i++) {
        if (check_fit(storage, host[i].m, host[i].g) > spmm_stage_units(M))
            fail(HSYM_E_UNSUPPORTED, "batched SpMM: pieces too large for the staging registers of this width");
        lds = std::max(lds, spmm_lds_bytes(storage, host[i].m, host[i].g));
        maxp = std::max(maxp, host[i].npanels);
        maxn = std::max(maxn, host[i].n * host[i].m);
    }
    auto kp = k_spmm_panel_b<M, T, A>;
    static std::once_flag attr_once;   // the 160 KB LDS limit, set once (threads may launch concurrently)
    std::call_once(attr_once, [&] {
        HIPCHK(hipFuncSetAttribute((const void *)kp, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024));
    });
    hipLaunchKernelGGL(k_zero_rows_b, dim3((unsigned)std::min<int64_t>((maxn + 255) / 256, 4096), (unsigned)count),
                       dim3(256), 0, s, jobs);
    HIPCHK(hipGetLastError());
    hipLaunchKernelGGL(kp, dim3((unsigned)maxp, (unsigned)count), dim3(SPMM_NT), lds, s, jobs);
    HIPCHK(hipGetLastError());
}

void spmm_batched(const SpmmJob *jobs, const SpmmJob *host, int count, int m, int storage, hipStream_t s) {
    const bool f64 = storage == HSYM_FP64;
    switch (round_m(m)) {
        case 1: if (f64) batched_typed<1, double, double>(jobs, host, count, storage, s); else batched_typed<1, float, float>(jobs, host, count, storage, s); break;
        case 2: if (f64) batched_typed<2, double, double>(jobs, host, count, storage, s); else batched_typed<2, float, float>(jobs, host, count, storage, s); break;
        case 4: if (f64) batched_typed<4, double, double>(jobs, host, count, storage, s); else batched_typed<4, float, float>(jobs, host, count, storage, s); break;
        case 8: if (f64) batched_typed<8, double, double>(jobs, host, count, storage, s); else batched_typed<8, float, float>(jobs, host, count, storage, s); break;
        default: if (f64) batched_typed<16, double, double>(jobs, host, count, storage, s); else batched_typed<16, float, float>(jobs, host, count, storage, s); break;
    }
}

void spmm_launch(hsym_matrix *H, int m, const void *X, int xprec, int64_t ldx, void *Y, int yprec, int64_t ldy,
                 hipStream_t s) {
    const int ku = check_fit(H->storage, m, H->tiles.g);
    if (H->storage == HSYM_FP64) {
        if (xprec != T_F64 || yprec != T_F64) fail(HSYM_E_INVALID_ARG, "fp64 storage takes fp64 blocks");
        launch_m<double, double, double, double>(H, m, X, ldx, Y, ldy, ku, s);
    } else {
        if (xprec == T_F64 && yprec == T_F64) launch_m<float, float, double, double>(H, m, X, ldx, Y, ldy, ku, s);
        else if (xprec == T_F32 && yprec == T_F32) launch_m<float, float, float, float>(H, m, X, ldx, Y, ldy, ku, s);
        else if (xprec == T_F32 && yprec == T_F64) launch_m<float, float, float, double>(H, m, X, ldx, Y, ldy, ku, s);
        else launch_m<float, float, double, float>(H, m, X, ldx, Y, ldy, ku, s);
    }
}

}  // namespace hsym
