// Symmetric SpMM from one stored triangle: Y = D X + U X + U^T X.
//
// Each stored off-diagonal entry is used twice, once as itself (row half,
// U X) and once transposed (U^T X): the two local products per stored block of
// Section 4.1.  The diagonal D is applied separately so it is counted once.
//
// One 1024-thread workgroup owns one row panel of R rows and walks its tiles
// in column order, as the CSB traversal of Section 4.4 does.  In LDS it keeps
// the panel's accumulator and X rows, plus the X rows and the transposed
// accumulator of the current external chunk.  Entries carry tile-local index
// codes (local row << shift | local column), 32-bit, or 16-bit on request when
// R * C <= 2^16 (measured 4% slower at fp64, m = 16; 17% less handle memory).
// A tile's entries are split in
// equal segments, one per group of LPE lanes; each lane of a group handles
// MW = M/LPE adjacent columns (2 when M >= 2):
//   - row half: a register accumulator for the current row, added to the
//     panel accumulator with LDS atomics when the row changes;
//   - transposed half: LDS atomics into the panel accumulator (own tiles) or
//     into the chunk accumulator (external tiles, whose columns lie below the
//     panel);
//   - fp64 output: Y is zeroed first and every panel adds its rows and its
//     external chunks' sums into Y with device-scope fp64 atomic adds (this
//     was measured 8% faster than partial slots and a reduction, and needs
//     no slot memory);
//   - fp32 output: the chunk sums are written to per-tile partial slots and
//     a second kernel adds the slots of every output chunk in a fixed order
//     in fp64 before rounding once.
// LDS rows are stored in 16-byte chunks permuted by an XOR with the row index,
// so the lane groups of one wave, which touch different rows, spread their
// 16-byte reads and their atomics over the banks.
#include <mutex>

#include "hsym_internal.h"

namespace hsym {

static inline int round_m(int m) {
    if (m <= 1) return 1;
    if (m <= 2) return 2;
    if (m <= 4) return 4;
    if (m <= 8) return 8;
    return 16;
}

// Columns of X handled by one lane: up to 2 adjacent ones, one 16-byte LDS
// chunk of an fp64 row.
__host__ __device__ constexpr int mw_of(int M) { return M < 2 ? M : 2; }

int spmm_lanes_per_entry(int storage, int m) {
    (void)storage;
    const int M = round_m(m);
    return M / mw_of(M);
}

size_t spmm_lds_bytes(int storage, int m, int R, int C) {
    (void)storage;   // X is staged in fp64 for both storage precisions
    int M = round_m(m);
    return (size_t)(R + C) * M * (8 + 8);
}


__device__ __forceinline__ void lds_add(double *p, double v) {
    __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// LDS row layout: a row of M elements of type E is cut into 16-byte chunks
// and chunk j of row r is stored at position j ^ (r mod chunks-per-row).  A
// wave touches one row per lane group: the XOR spreads the groups' 16-byte
// reads over the banks.  In the fp64 accumulators (FLIP) the two slots of a
// chunk are also swapped on the next bit of r above those that place the
// row in the 64 banks, which gives the 8-byte atomics of one instruction 4
// or more distinct bank windows.  Rows shorter than 16 bytes are plain.
template <int M, typename E, bool FLIP>
struct RowLay {
    static constexpr int EPC = 16 / (int)sizeof(E);
    static constexpr int CPR = (M * (int)sizeof(E)) / 16;
    static constexpr int POS = CPR >= 1 ? 64 / (CPR * 4) : 1;   // row positions across 64 banks
    __device__ static __forceinline__ int slot_flip(int r) {
        if constexpr (FLIP && EPC == 2 && CPR >= 1) return (r / POS) & 1;
        else return 0;
    }
    __device__ static __forceinline__ int phys(int r, int k) {
        if constexpr (CPR < 1) return k;
        else return (((k / EPC) ^ (r & (CPR - 1))) * EPC) + ((k % EPC) ^ slot_flip(r));
    }
};

// A lane's MW = mw_of(M) elements k0 .. k0+MW-1 of row r (plain slots), as fp64.
template <int M, typename T>
__device__ __forceinline__ void read_row(const T *rowp, int r, int k0, double *o) {
    using RL = RowLay<M, T, false>;
    constexpr int MW = mw_of(M);
    if constexpr (sizeof(T) == 8 && MW == 2 && RL::CPR >= 1) {
        const double2 v = *reinterpret_cast<const double2 *>(rowp + RL::phys(r, k0));
        o[0] = v.x;
        o[1] = v.y;
    } else {
#pragma unroll
        for (int i = 0; i < MW; i++) o[i] = (double)rowp[RL::phys(r, k0 + i)];
    }
}

// T: stored values.  X is staged in LDS as fp64 and products and sums are
// fp64 for both storage precisions: an fp32 value is converted once per entry,
// the X rows once per staging (the LDS fp64 atomic add is also several times
// cheaper than the fp32 one on gfx950)
// IT: uint16_t or uint32_t index codes, local row << cs | local column
template <int M, typename T, typename XIN, typename YT, typename IT>
__device__ __forceinline__ void spmm_panel_body(
    const int64_t *__restrict__ ptp, const int32_t *__restrict__ porder, const TileDesc *__restrict__ tiles,
    const IT *__restrict__ idx, int cs,
    const T *__restrict__ vals, const T *__restrict__ diag, const XIN *__restrict__ X, int64_t ldx,
    YT *__restrict__ Y, int64_t ldy, double *__restrict__ partials, int64_t n, int R, int C, int G,
    int64_t npanels, int m, int64_t blk, unsigned char *smem_raw) {
    using XL = RowLay<M, double, false>;
    using AL = RowLay<M, double, true>;
    constexpr int NT = 1024, MW = mw_of(M), LPE = M / MW, GK = NT / LPE;
    double *acc = reinterpret_cast<double *>(smem_raw);
    double *ts = acc + (size_t)R * M;
    double *xp = ts + (size_t)C * M;
    double *xs = xp + (size_t)R * M;
    const int tid = threadIdx.x, g = tid / LPE, q = tid % LPE, k0 = q * MW;
    const uint32_t cmask = (1u << cs) - 1u;   // 16-bit codes: local row << cs | local column
    const int64_t p = porder[blk];
    const int64_t row0 = p * (int64_t)R;
    const int nrow = (int)((n - row0) < R ? (n - row0) : R);

    for (int i = tid; i < R * M; i += NT) {
        const int r = i / M, k = i - r * M;
        double v = 0.0;
        if (r < nrow && k < m) v = (double)X[(row0 + r) * ldx + k];
        xp[r * M + XL::phys(r, k)] = v;
        acc[i] = 0.0;
    }
    const int64_t t0 = ptp[p], t1 = ptp[p + 1];
    constexpr int B = 4;   // entries loaded ahead of use
    for (int64_t t = t0; t < t1; t++) {
        const TileDesc td = tiles[t];
        const int64_t col0 = (int64_t)td.chunk * C;
        const bool ext = td.slot >= 0;
        if (ext) {
            const int ncol = (int)((n - col0) < C ? (n - col0) : C);
            for (int i = tid; i < C * M; i += NT) {
                const int r = i / M, k = i - r * M;
                double v = 0.0;
                if (r < ncol && k < m) v = (double)X[(col0 + r) * ldx + k];
                xs[r * M + XL::phys(r, k)] = v;
                ts[i] = 0.0;
            }
        }
        __syncthreads();
        // own tiles read and update the panel's rows directly; col0 - row0 is a
        // multiple of C (itself a multiple of 8), so a chunk row has the
        // swizzle of its panel row
        const double *xsrc = ext ? xs : xp + (col0 - row0) * M;
        double *tgt = ext ? ts : acc + (col0 - row0) * M;
        const int len = td.len;
        for (int seg = g; seg < G; seg += GK) {
            const IT *ip = idx + td.base + seg;
            const T *vp = vals + td.base + seg;
            int cur = -1;
            double ra[MW], xr[MW];
#pragma unroll
            for (int j = 0; j < MW; j++) { ra[j] = 0.0; xr[j] = 0.0; }
            for (int e0 = 0; e0 < len; e0 += B) {
                uint32_t w[B];
                T a[B];
                const int cnt = (len - e0) < B ? (len - e0) : B;
#pragma unroll
                for (int u = 0; u < B; u++) {
                    const int off = (e0 + (u < cnt ? u : 0)) * G;
                    w[u] = ip[off];
                    a[u] = vp[off];
                }
#pragma unroll
                for (int u = 0; u < B; u++) {
                    if (u >= cnt) break;
                    int r, c;
                    if constexpr (sizeof(IT) == 2) {
                        r = (int)(w[u] >> cs);
                        c = (int)(w[u] & cmask);
                    } else {   // 32-bit codes: row << 16 | column
                        r = (int)(w[u] >> 16);
                        c = (int)(w[u] & 0xffffu);
                    }
                    if (r != cur) {
                        if (cur >= 0) {
#pragma unroll
                            for (int j = 0; j < MW; j++) {
                                lds_add(acc + cur * M + AL::phys(cur, k0 + j), ra[j]);
                                ra[j] = 0.0;
                            }
                        }
                        cur = r;
                        read_row<M, double>(xp + r * M, r, k0, xr);
                    }
                    double xc[MW];
                    read_row<M, double>(xsrc + c * M, c, k0, xc);
                    const double av = (double)a[u];
                    double *trow = tgt + c * M;
                    if constexpr (MW == 2 && AL::CPR >= 1) {
                        // both slots of the lane's chunk; the flip only swaps them
                        const int cb = AL::phys(c, k0) & ~1, f = AL::slot_flip(c);
                        ra[0] = fma(av, xc[0], ra[0]);
                        ra[1] = fma(av, xc[1], ra[1]);
                        lds_add(trow + cb + f, av * xr[0]);
                        lds_add(trow + cb + (f ^ 1), av * xr[1]);
                    } else {
#pragma unroll
                        for (int j = 0; j < MW; j++) {
                            ra[j] = fma(av, xc[j], ra[j]);
                            lds_add(trow + AL::phys(c, k0 + j), av * xr[j]);
                        }
                    }
                }
            }
            if (cur >= 0) {
#pragma unroll
                for (int j = 0; j < MW; j++) lds_add(acc + cur * M + AL::phys(cur, k0 + j), ra[j]);
            }
        }
        __syncthreads();
        if (ext) {
            if constexpr (sizeof(YT) == 8) {
                // fp64 output: the chunk's transposed sums go straight into Y
                // (zeroed before the launch) with device-scope atomic adds
                for (int i = tid; i < C * M; i += NT) {
                    const int r = i / M, k = i - r * M;
                    if (k < m && col0 + r < n) unsafeAtomicAdd(&Y[(col0 + r) * ldy + k], ts[r * M + AL::phys(r, k)]);
                }
            } else {
                double *dst = partials + (int64_t)td.slot * C * M;
                for (int i = tid; i < C * M; i += NT) {
                    const int r = i / M, k = i - r * M;
                    dst[i] = ts[r * M + AL::phys(r, k)];
                }
            }
            __syncthreads();
        }
    }
    for (int i = tid; i < nrow * M; i += NT) {
        const int r = i / M, k = i - r * M;
        if (k < m) {
            const int64_t row = row0 + r;
            const double v = acc[r * M + AL::phys(r, k)] + (double)diag[row] * xp[r * M + XL::phys(r, k)];
            if constexpr (sizeof(YT) == 8) unsafeAtomicAdd(&Y[row * ldy + k], v);
            else Y[row * ldy + k] = (YT)v;
        }
    }
}

template <int M, typename T, typename XIN, typename YT, typename IT>
__global__ __launch_bounds__(1024) void k_spmm_panel(
    const int64_t *__restrict__ ptp, const int32_t *__restrict__ porder, const TileDesc *__restrict__ tiles,
    const IT *__restrict__ idx, int cs,
    const T *__restrict__ vals, const T *__restrict__ diag, const XIN *__restrict__ X, int64_t ldx,
    YT *__restrict__ Y, int64_t ldy, double *__restrict__ partials, int64_t n, int R, int C, int G,
    int64_t npanels, int m) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    spmm_panel_body<M, T, XIN, YT, IT>(ptp, porder, tiles, idx, cs, vals, diag, X, ldx, Y, ldy, partials, n, R, C, G,
                                       npanels, m, blockIdx.x, smem_raw);
}

// batched over matrices (fp64 blocks): blockIdx.y selects the job
template <int M, typename T>
__global__ __launch_bounds__(1024) void k_spmm_panel_b(const SpmmJob *__restrict__ jobs) {
    extern __shared__ __align__(16) unsigned char smem_raw[];
    const SpmmJob J = jobs[blockIdx.y];
    if ((int64_t)blockIdx.x >= J.npanels) return;
    // the index width is a property of each job's handle (uniform per workgroup)
    if (J.idx_bytes == 2)
        spmm_panel_body<M, T, double, double, uint16_t>(J.ptp, J.porder, J.tiles, (const uint16_t *)J.idx, J.idx_shift,
                                                        (const T *)J.vals, (const T *)J.diag, J.X, J.ldx, J.Y, J.ldy,
                                                        J.partials, J.n, J.R, J.C, J.G, J.npanels, J.m, blockIdx.x,
                                                        smem_raw);
    else
        spmm_panel_body<M, T, double, double, uint32_t>(J.ptp, J.porder, J.tiles, (const uint32_t *)J.idx, J.idx_shift,
                                                        (const T *)J.vals, (const T *)J.diag, J.X, J.ldx, J.Y, J.ldy,
                                                        J.partials, J.n, J.R, J.C, J.G, J.npanels, J.m, blockIdx.x,
                                                        smem_raw);
}

// Y[chunk rows] += sum of the partial slots of that chunk, in slot order.
template <int M, typename YT, int NT>
__device__ __forceinline__ void spmm_reduce_body(const int32_t *__restrict__ red_chunks,
                                                 const int64_t *__restrict__ red_ptr,
                                                 const int32_t *__restrict__ red_slot,
                                                 const double *__restrict__ partials, YT *__restrict__ Y,
                                                 int64_t ldy, int64_t n, int C, int m, int64_t blk) {
    const int64_t g = red_chunks[blk];
    const int64_t col0 = g * C;
    const int ncol = (int)((n - col0) < C ? (n - col0) : C);
    const int64_t q0 = red_ptr[g], q1 = red_ptr[g + 1];
    for (int i = threadIdx.x; i < ncol * M; i += NT) {
        const int r = i / M, k = i - r * M;
        if (k >= m) continue;
        double s = 0.0;
        for (int64_t q = q0; q < q1; q++) s += partials[(int64_t)red_slot[q] * C * M + i];
        YT *y = Y + (col0 + r) * ldy + k;
        *y = (YT)((double)*y + s);
    }
}

template <int M, typename YT, int NT>
__global__ __launch_bounds__(NT) void k_spmm_reduce(const int32_t *__restrict__ red_chunks,
                                                    const int64_t *__restrict__ red_ptr,
                                                    const int32_t *__restrict__ red_slot,
                                                    const double *__restrict__ partials, YT *__restrict__ Y,
                                                    int64_t ldy, int64_t n, int C, int m) {
    spmm_reduce_body<M, YT, NT>(red_chunks, red_ptr, red_slot, partials, Y, ldy, n, C, m, blockIdx.x);
}

template <int M, int NT>
__global__ __launch_bounds__(NT) void k_spmm_reduce_b(const SpmmJob *__restrict__ jobs) {
    const SpmmJob J = jobs[blockIdx.y];
    if ((int64_t)blockIdx.x >= J.nred) return;
    spmm_reduce_body<M, double, NT>(J.red_chunks, J.red_ptr, J.red_slot, J.partials, J.Y, J.ldy, J.n, J.C, J.m,
                                    blockIdx.x);
}

// Y[r][0..m) = 0 for r < n (leading dimension ldy): the fp64 SpMM adds
// into Y (a kernel rather than a memset, so a graph may record it)
__global__ __launch_bounds__(256) void k_zero_rows(double *__restrict__ Y, int64_t n, int m, int64_t ldy) {
    const int64_t cnt = n * m;
    for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < cnt; e += (int64_t)gridDim.x * 256) {
        const int64_t r = e / m;
        Y[r * ldy + (e - r * m)] = 0.0;
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

static void zero_rows(double *Y, int64_t n, int m, int64_t ldy, hipStream_t s) {
    const int64_t blocks = std::min<int64_t>((n * m + 255) / 256, 4096);
    hipLaunchKernelGGL(k_zero_rows, dim3((unsigned)std::max<int64_t>(blocks, 1)), dim3(256), 0, s, Y, n, m, ldy);
    HIPCHK(hipGetLastError());
}

template <int M, typename T, typename XIN, typename YT, typename IT>
static void launch_typed(hsym_matrix *H, int m, const void *X, int64_t ldx, void *Y, int64_t ldy,
                         void *partials, hipStream_t s) {
    const DeviceTiles &dt = H->tiles;
    size_t lds = spmm_lds_bytes(H->storage, m, dt.R, dt.C);
    auto kp = k_spmm_panel<M, T, XIN, YT, IT>;
    static std::once_flag attr_once;   // the 160 KB LDS limit, set once (threads may launch concurrently)
    std::call_once(attr_once, [&] {
        HIPCHK(hipFuncSetAttribute((const void *)kp, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024));
    });
    const T *diag = (const T *)(H->storage == HSYM_FP64 ? (const void *)H->diag64 : (const void *)H->diag32);
    constexpr bool atomic_out = sizeof(YT) == 8;
    if (atomic_out) zero_rows((double *)Y, H->n, m, ldy, s);
    hipLaunchKernelGGL(kp, dim3((unsigned)dt.npanels), dim3(1024), lds, s, dt.panel_tile_ptr, dt.panel_order, dt.tiles,
                       (const IT *)dt.idx, dt.idx_shift, (const T *)dt.vals, diag, (const XIN *)X, ldx, (YT *)Y, ldy, (double *)partials, H->n, dt.R,
                       dt.C, dt.G, dt.npanels, m);
    HIPCHK(hipGetLastError());
    if (!atomic_out && dt.nred_chunks > 0) {
        hipLaunchKernelGGL((k_spmm_reduce<M, YT, 256>), dim3((unsigned)dt.nred_chunks), dim3(256), 0, s,
                           dt.red_chunks, dt.red_ptr, dt.red_slot, (const double *)partials, (YT *)Y, ldy, H->n, dt.C,
                           m);
        HIPCHK(hipGetLastError());
    }
}

template <typename T, typename XIN, typename YT, typename IT>
static void launch_mi(hsym_matrix *H, int m, const void *X, int64_t ldx, void *Y, int64_t ldy, void *part,
                      hipStream_t s) {
    switch (round_m(m)) {
        case 1: launch_typed<1, T, XIN, YT, IT>(H, m, X, ldx, Y, ldy, part, s); break;
        case 2: launch_typed<2, T, XIN, YT, IT>(H, m, X, ldx, Y, ldy, part, s); break;
        case 4: launch_typed<4, T, XIN, YT, IT>(H, m, X, ldx, Y, ldy, part, s); break;
        case 8: launch_typed<8, T, XIN, YT, IT>(H, m, X, ldx, Y, ldy, part, s); break;
        default: launch_typed<16, T, XIN, YT, IT>(H, m, X, ldx, Y, ldy, part, s); break;
    }
}

template <typename T, typename XIN, typename YT>
static void launch_m(hsym_matrix *H, int m, const void *X, int64_t ldx, void *Y, int64_t ldy, void *part,
                     hipStream_t s) {
    if (H->tiles.idx_bytes == 2) launch_mi<T, XIN, YT, uint16_t>(H, m, X, ldx, Y, ldy, part, s);
    else launch_mi<T, XIN, YT, uint32_t>(H, m, X, ldx, Y, ldy, part, s);
}

SpmmJob spmm_job(hsym_matrix *H, int m, const double *X, double *Y, double *partials) {
    const DeviceTiles &dt = H->tiles;
    SpmmJob J{};
    J.ptp = dt.panel_tile_ptr; J.porder = dt.panel_order; J.tiles = dt.tiles; J.idx = dt.idx; J.vals = dt.vals;
    J.idx_bytes = dt.idx_bytes; J.idx_shift = dt.idx_shift;
    J.diag = H->storage == HSYM_FP64 ? (const void *)H->diag64 : (const void *)H->diag32;
    J.X = X; J.ldx = m; J.Y = Y; J.ldy = m; J.partials = partials;
    J.n = H->n; J.R = dt.R; J.C = dt.C; J.G = dt.G; J.npanels = dt.npanels; J.m = m;
    J.red_chunks = dt.red_chunks; J.red_ptr = dt.red_ptr; J.red_slot = dt.red_slot; J.nred = dt.nred_chunks;
    return J;
}

template <int M, typename T>
static void batched_typed(const SpmmJob *jobs, const SpmmJob *host, int count, hipStream_t s) {
    size_t lds = 0;
    int64_t maxp = 0, maxr = 0;
    for (int i = 0; i < count; i++) {
        lds = std::max(lds, spmm_lds_bytes(HSYM_FP64, M, host[i].R, host[i].C));
        maxp = std::max(maxp, host[i].npanels);
        maxr = std::max(maxr, host[i].nred);
    }
    if (lds > 160 * 1024) fail(HSYM_E_UNSUPPORTED, "block width too large for a handle's panel geometry");
    auto kp = k_spmm_panel_b<M, T>;
    static std::once_flag attr_once;   // the 160 KB LDS limit, set once (threads may launch concurrently)
    std::call_once(attr_once, [&] {
        HIPCHK(hipFuncSetAttribute((const void *)kp, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024));
    });
    int64_t maxn = 0;
    for (int i = 0; i < count; i++) maxn = std::max(maxn, host[i].n * host[i].m);
    (void)maxr;
    hipLaunchKernelGGL(k_zero_rows_b, dim3((unsigned)std::min<int64_t>((maxn + 255) / 256, 4096), (unsigned)count),
                       dim3(256), 0, s, jobs);
    HIPCHK(hipGetLastError());
    hipLaunchKernelGGL(kp, dim3((unsigned)maxp, (unsigned)count), dim3(1024), lds, s, jobs);
    HIPCHK(hipGetLastError());
}

void spmm_batched(const SpmmJob *jobs, const SpmmJob *host, int count, int m, int storage, hipStream_t s) {
    const bool f64 = storage == HSYM_FP64;
    switch (round_m(m)) {
        case 1: if (f64) batched_typed<1, double>(jobs, host, count, s); else batched_typed<1, float>(jobs, host, count, s); break;
        case 2: if (f64) batched_typed<2, double>(jobs, host, count, s); else batched_typed<2, float>(jobs, host, count, s); break;
        case 4: if (f64) batched_typed<4, double>(jobs, host, count, s); else batched_typed<4, float>(jobs, host, count, s); break;
        case 8: if (f64) batched_typed<8, double>(jobs, host, count, s); else batched_typed<8, float>(jobs, host, count, s); break;
        default: if (f64) batched_typed<16, double>(jobs, host, count, s); else batched_typed<16, float>(jobs, host, count, s); break;
    }
}

size_t spmm_partial_bytes(hsym_matrix *H, int m, int yprec) {
    if (yprec == T_F64) return 256;   // fp64 outputs take the transposed sums by atomic adds
    return (size_t)std::max<int64_t>(H->tiles.nslots, 1) * H->tiles.C * round_m(m) * sizeof(double);
}

void spmm_launch(hsym_matrix *H, int m, const void *X, int xprec, int64_t ldx, void *Y, int yprec,
                 int64_t ldy, void *partials, hipStream_t s) {
    const DeviceTiles &dt = H->tiles;
    if (spmm_lds_bytes(H->storage, m, dt.R, dt.C) > 160 * 1024)
        fail(HSYM_E_UNSUPPORTED, "block width too large for this handle's panel geometry");
    if (H->storage == HSYM_FP64) {
        if (xprec != T_F64 || yprec != T_F64) fail(HSYM_E_INVALID_ARG, "fp64 storage takes fp64 blocks");
        launch_m<double, double, double>(H, m, X, ldx, Y, ldy, partials, s);
    } else {
        if (xprec == T_F64 && yprec == T_F64) launch_m<float, double, double>(H, m, X, ldx, Y, ldy, partials, s);
        else if (xprec == T_F32 && yprec == T_F32) launch_m<float, float, float>(H, m, X, ldx, Y, ldy, partials, s);
        else if (xprec == T_F32 && yprec == T_F64) launch_m<float, float, double>(H, m, X, ldx, Y, ldy, partials, s);
        else launch_m<float, double, float>(H, m, X, ldx, Y, ldy, partials, s);
    }
}

}  // namespace hsym
