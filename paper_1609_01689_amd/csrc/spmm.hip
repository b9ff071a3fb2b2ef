// Symmetric SpMM from one stored triangle: Y = D X + U X + U^T X.
//
// Each stored off-diagonal entry is used twice, once as itself (row half,
// U X) and once transposed (U^T X), the two local products per stored block
// of Section 4.1; the diagonal D is applied separately so it is counted once.
//
// One workgroup owns one row panel of R rows and walks its tiles (chunks of
// C columns) in column order, as the CSB traversal of Section 4.4 does:
//   - the X rows of the chunk are staged in LDS;
//   - lanes own slice rows: the row half is accumulated in registers and
//     added once per tile to the panel accumulator in LDS;
//   - the transposed half is accumulated with LDS atomics into the panel
//     accumulator (own tiles) or into a chunk accumulator that is written out
//     as a partial sum (external tiles, whose columns lie below the panel);
//   - a second kernel adds the partial sums of every output chunk in a fixed
//     order.  No global atomics are used.
#include "hsym_internal.h"

namespace hsym {

template <typename T, int M>
struct LdsStride {
    // one 16-byte pad per row spreads consecutive rows over the LDS banks
    static constexpr int MP = (M == 1) ? 1 : (M + 16 / (int)sizeof(T));
};

static inline int round_m(int m) {
    if (m <= 1) return 1;
    if (m <= 2) return 2;
    if (m <= 4) return 4;
    if (m <= 8) return 8;
    if (m <= 12) return 12;
    return 16;
}

template <typename T>
static int stride_of(int M) {
    return (M == 1) ? 1 : (M + 16 / (int)sizeof(T));
}

size_t spmm_lds_bytes(int storage, int m, int R, int C) {
    int M = round_m(m);
    if (storage == HSYM_FP64) return (size_t)(R + 2 * C) * stride_of<double>(M) * sizeof(double);
    return (size_t)(R + 2 * C) * stride_of<float>(M) * sizeof(float);
}

__device__ __forceinline__ int64_t xcd_panel(int64_t b, int64_t P) {
    // Workgroups are dealt round-robin to the 8 XCDs; give each XCD a run of
    // consecutive panels so the X chunks they share stay in that XCD's L2.
    const int64_t x = b & 7, i = b >> 3;
    const int64_t q = P >> 3, rem = P & 7;
    return x * q + (x < rem ? x : rem) + i;
}

__device__ __forceinline__ void lds_add(double *p, double v) {
    __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}
__device__ __forceinline__ void lds_add(float *p, float v) {
    __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// LPR lanes share one slice row, each handling MW = M/LPR columns.
template <int M, int LPR, typename T, typename XIN, typename YT, int NT>
__global__ __launch_bounds__(NT) void k_spmm_panel(
    const int64_t *__restrict__ ptp, const TileDesc *__restrict__ tiles,
    const SliceDesc *__restrict__ slices, const uint16_t *__restrict__ srows,
    const uint32_t *__restrict__ cols, const T *__restrict__ vals, const T *__restrict__ diag,
    const XIN *__restrict__ X, int64_t ldx, YT *__restrict__ Y, int64_t ldy,
    T *__restrict__ partials, int64_t n, int R, int C, int64_t npanels, int m) {
    constexpr int MP = LdsStride<T, M>::MP;
    constexpr int NW = NT / 64;
    constexpr int MW = M / LPR;
    extern __shared__ __align__(16) unsigned char smem_raw[];
    T *acc = reinterpret_cast<T *>(smem_raw);
    T *xs = acc + (size_t)R * MP;
    T *ts = xs + (size_t)C * MP;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int l = lane / LPR, h = lane % LPR;
    const int64_t p = xcd_panel(blockIdx.x, npanels);
    const int64_t row0 = p * (int64_t)R;
    const int nrow = (int)((n - row0) < R ? (n - row0) : R);

    for (int i = tid; i < R * MP; i += NT) acc[i] = T(0);
    const int64_t t0 = ptp[p], t1 = ptp[p + 1];
    for (int64_t t = t0; t < t1; t++) {
        const TileDesc td = tiles[t];
        const int64_t col0 = (int64_t)td.chunk * C;
        const int ncol = (int)((n - col0) < C ? (n - col0) : C);
        for (int i = tid; i < C * M; i += NT) {
            const int r = i / M, k = i - r * M;
            T v = T(0);
            if (r < ncol && k < m) v = (T)X[(col0 + r) * ldx + k];
            xs[r * MP + k] = v;
        }
        const bool ext = td.slot >= 0;
        if (ext)
            for (int i = tid; i < C * MP; i += NT) ts[i] = T(0);
        __syncthreads();
        T *tgt = ext ? ts : acc + (col0 - row0) * MP;
        for (int s = wave; s < td.nslices; s += NW) {
            const SliceDesc sd = slices[td.slice_begin + s];
            const int nr = sd.nrows;
            // a slice holds up to 64 rows; 64/LPR of them are processed per pass
            for (int lb = 0; lb < nr; lb += 64 / LPR) {
                const int lr = lb + l;
                if (lr >= nr) break;
                const int r = srows[(td.slice_begin + s) * 64 + lr];
                const XIN *xrow = X + (row0 + r) * ldx + h * MW;
                T xr[MW], ra[MW];
#pragma unroll
                for (int k = 0; k < MW; k++) {
                    xr[k] = (h * MW + k < m) ? (T)xrow[k] : T(0);
                    ra[k] = T(0);
                }
                const uint32_t *cp = cols + sd.base + lr;
                const T *vp = vals + sd.base + lr;
                const int len = sd.len;
                for (int e = 0; e < len; e++) {
                    const uint32_t c = cp[(int64_t)e * nr];
                    const T a = vp[(int64_t)e * nr];
                    const T *xc = xs + c * MP + h * MW;
                    T *tc = tgt + c * MP + h * MW;
#pragma unroll
                    for (int k = 0; k < MW; k++) ra[k] = fma(a, xc[k], ra[k]);
#pragma unroll
                    for (int k = 0; k < MW; k++) lds_add(tc + k, a * xr[k]);
                }
                T *ar = acc + r * MP + h * MW;
#pragma unroll
                for (int k = 0; k < MW; k++) lds_add(ar + k, ra[k]);
            }
        }
        __syncthreads();
        if (ext) {
            T *dst = partials + (int64_t)td.slot * C * M;
            for (int i = tid; i < C * M; i += NT) {
                const int r = i / M, k = i - r * M;
                dst[i] = ts[r * MP + k];
            }
            __syncthreads();
        }
    }
    for (int i = tid; i < nrow * M; i += NT) {
        const int r = i / M, k = i - r * M;
        if (k < m) {
            const int64_t row = row0 + r;
            const T x = (T)X[row * ldx + k];
            Y[row * ldy + k] = (YT)(acc[r * MP + k] + diag[row] * x);
        }
    }
}

// Y[chunk rows] += sum of the partial slots of that chunk, in slot order.
template <int M, typename T, typename YT, int NT>
__global__ __launch_bounds__(NT) void k_spmm_reduce(const int32_t *__restrict__ red_chunks,
                                                    const int64_t *__restrict__ red_ptr,
                                                    const int32_t *__restrict__ red_slot,
                                                    const T *__restrict__ partials, YT *__restrict__ Y,
                                                    int64_t ldy, int64_t n, int C, int m) {
    const int64_t g = red_chunks[blockIdx.x];
    const int64_t col0 = g * C;
    const int ncol = (int)((n - col0) < C ? (n - col0) : C);
    const int64_t q0 = red_ptr[g], q1 = red_ptr[g + 1];
    for (int i = threadIdx.x; i < ncol * M; i += NT) {
        const int r = i / M, k = i - r * M;
        if (k >= m) continue;
        T s = T(0);
        for (int64_t q = q0; q < q1; q++) s += partials[(int64_t)red_slot[q] * C * M + i];
        YT *y = Y + (col0 + r) * ldy + k;
        *y = *y + (YT)s;
    }
}

template <int M, int LPR, typename T, typename XIN, typename YT>
static void launch_typed(hsym_matrix *H, int m, const void *X, int64_t ldx, void *Y, int64_t ldy,
                         void *partials, hipStream_t s) {
    const DeviceTiles &dt = H->tiles;
    constexpr int NT = (M >= 8) ? 1024 : 512;
    size_t lds = (size_t)(dt.R + 2 * dt.C) * LdsStride<T, M>::MP * sizeof(T);
    auto kp = k_spmm_panel<M, LPR, T, XIN, YT, NT>;
    static bool attr_set = false;
    if (!attr_set) {
        HIPCHK(hipFuncSetAttribute((const void *)kp, hipFuncAttributeMaxDynamicSharedMemorySize, 160 * 1024));
        attr_set = true;
    }
    const T *diag = (const T *)(H->storage == HSYM_FP64 ? (const void *)H->diag64 : (const void *)H->diag32);
    hipLaunchKernelGGL(kp, dim3((unsigned)dt.npanels), dim3(NT), lds, s, dt.panel_tile_ptr, dt.tiles,
                       dt.slices, dt.slice_rows, dt.cols, (const T *)dt.vals, diag, (const XIN *)X, ldx,
                       (YT *)Y, ldy, (T *)partials, H->n, dt.R, dt.C, dt.npanels, m);
    HIPCHK(hipGetLastError());
    if (dt.nred_chunks > 0) {
        hipLaunchKernelGGL((k_spmm_reduce<M, T, YT, 256>), dim3((unsigned)dt.nred_chunks), dim3(256), 0, s,
                           dt.red_chunks, dt.red_ptr, dt.red_slot, (const T *)partials, (YT *)Y, ldy, H->n,
                           dt.C, m);
        HIPCHK(hipGetLastError());
    }
}

template <typename T, typename XIN, typename YT>
static void launch_m(hsym_matrix *H, int m, const void *X, int64_t ldx, void *Y, int64_t ldy, void *part,
                     hipStream_t s) {
    switch (round_m(m)) {
        case 1: launch_typed<1, 1, T, XIN, YT>(H, m, X, ldx, Y, ldy, part, s); break;
        case 2: launch_typed<2, 1, T, XIN, YT>(H, m, X, ldx, Y, ldy, part, s); break;
        case 4: launch_typed<4, 1, T, XIN, YT>(H, m, X, ldx, Y, ldy, part, s); break;
        case 8: launch_typed<8, 1, T, XIN, YT>(H, m, X, ldx, Y, ldy, part, s); break;
        case 12: launch_typed<12, 2, T, XIN, YT>(H, m, X, ldx, Y, ldy, part, s); break;
        default: launch_typed<16, 2, T, XIN, YT>(H, m, X, ldx, Y, ldy, part, s); break;
    }
}

size_t spmm_partial_bytes(hsym_matrix *H, int m) {
    size_t es = H->storage == HSYM_FP64 ? 8 : 4;
    return (size_t)std::max<int64_t>(H->tiles.nslots, 1) * H->tiles.C * round_m(m) * es;
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
