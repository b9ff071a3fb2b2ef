// Tall-skinny block-vector kernels of the LOBPCG iteration (fp64, row-major
// n x m blocks with leading dimension m, m <= 16):
//   - block inner products X^T Y (Section 4.4 "block inner product") on the
//     fp64 matrix cores, reduced in two deterministic stages;
//   - linear combinations Y = X G (Section 4.4 "linear combination"), fused
//     where the iteration allows (the Rayleigh-Ritz update of X, P, AX, AP
//     together with the next residual R = AX - X Theta and its column norms);
//   - the preconditioner applies of eq. 11 (diagonal and 64x64 blocks).
#include "hsym_internal.h"
#include "dense.h"
#include "wave.h"

namespace hsym {

typedef double double4_t __attribute__((ext_vector_type(4)));

// guarded shifted denominator: d, or +-delta where |d| < delta
__device__ __forceinline__ double guard_den(double d, double delta) {
    return fabs(d) >= delta ? d : (d >= 0.0 ? delta : -delta);
}

// ---------------------------------------------------------------------------
// Gram: G = [A_0 .. A_{na-1}]^T [B_0 .. B_{nb-1}], each block n x m (ld m).
// Stage 1: every workgroup reduces a contiguous row range into a K1 x K2
// partial with v_mfma_f64_16x16x4f64; stage 2 sums the partials in order.
// ---------------------------------------------------------------------------
// MFMA f64 16x16x4 operand layout: lane l holds A[i=l%16][k=l/16] and
// B[k=l/16][j=l%16]; accumulator register v of lane l holds D[l/16 + 4v][l%16].
template <int T1, int T2, bool SYM = false>
__device__ __forceinline__ void gram_partial_body(const GramArgs &g, double *__restrict__ part, int64_t rows_per_wg,
                                                  int64_t bx) {
    // the four waves' partial sums meet in LDS, at most 3 column tiles at a time
    constexpr int TC = T2 < 3 ? T2 : 3;
    __shared__ double red[4][T1 * 16][TC * 16 + 1];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int m = g.m;
    const int K1 = g.na * m, K2 = g.nb * m;
    const int li = lane & 15, lk = lane >> 4;
    // column this lane feeds for every 16-column tile
    const double *pa[T1];
    const double *pb[T2];
    int ca[T1], cb[T2];
#pragma unroll
    for (int t = 0; t < T1; t++) {
        int c = 16 * t + li;
        ca[t] = c < K1;
        int blk = c < K1 ? c / m : 0, col = c < K1 ? c % m : 0;
        pa[t] = g.a[blk] + col;
    }
#pragma unroll
    for (int t = 0; t < T2; t++) {
        int c = 16 * t + li;
        cb[t] = c < K2;
        int blk = c < K2 ? c / m : 0, col = c < K2 ? c % m : 0;
        pb[t] = g.b[blk] + col;
    }
    double4_t acc[T1][T2];
#pragma unroll
    for (int i = 0; i < T1; i++)
#pragma unroll
        for (int j = 0; j < T2; j++) acc[i][j] = (double4_t){0.0, 0.0, 0.0, 0.0};
    const int64_t r_begin = bx * rows_per_wg;
    int64_t r_end = r_begin + rows_per_wg;
    if (r_end > g.n) r_end = g.n;
    // GU row steps of 16 are loaded before their MFMAs (more loads in flight
    // per wave); each accumulator still takes the rows in ascending order
    constexpr int GU = 4;
    for (int64_t r0 = r_begin + 4 * wave; r0 < r_end; r0 += 16 * GU) {
        double av[GU][T1], bv[GU][T2];
#pragma unroll
        for (int u = 0; u < GU; u++) {
            const int64_t r = r0 + 16 * u + lk;
            const bool ok = r < r_end;
#pragma unroll
            for (int t = 0; t < T1; t++) av[u][t] = (ok && ca[t]) ? pa[t][r * m] : 0.0;
#pragma unroll
            for (int t = 0; t < T2; t++) bv[u][t] = (ok && cb[t]) ? pb[t][r * m] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < GU; u++)
#pragma unroll
            for (int i = 0; i < T1; i++)
#pragma unroll
                for (int j = 0; j < T2; j++) {
                    // SYM: tiles below the diagonal of either half are not formed
                    if (SYM && (j < T1 ? j < i : j - T1 < i)) continue;
                    acc[i][j] = __builtin_amdgcn_mfma_f64_16x16x4f64(av[u][i], bv[u][j], acc[i][j], 0, 0, 0);
                }
    }
    double *out = part + bx * K1 * K2;
#pragma unroll
    for (int j0 = 0; j0 < T2; j0 += TC) {
        if (j0) __syncthreads();
#pragma unroll
        for (int i = 0; i < T1; i++)
#pragma unroll
            for (int j = 0; j < TC; j++)
                if (j0 + j < T2)
#pragma unroll
                    for (int v = 0; v < 4; v++) red[wave][16 * i + lk + 4 * v][16 * j + li] = acc[i][j0 + j][v];
        __syncthreads();
        const int c0 = 16 * j0, cw = (K2 - c0) < 16 * TC ? (K2 - c0) : 16 * TC;
        for (int e = tid; e < K1 * cw; e += 256) {
            const int i = e / cw, j = e - (e / cw) * cw;
            out[i * K2 + c0 + j] = red[0][i][j] + red[1][i][j] + red[2][i][j] + red[3][i][j];
        }
    }
}

template <int T1, int T2, bool SYM = false>
__global__ __launch_bounds__(256) void k_gram_partial(GramArgs g, double *__restrict__ part, int64_t rows_per_wg) {
    gram_partial_body<T1, T2, SYM>(g, part, rows_per_wg, blockIdx.x);
}

// the Rayleigh-Ritz Gram [S^T S | S^T A S] without its lower tiles; its
// registers are capped so that two waves share a SIMD (measured 24% faster at
// T1 = 3 than one wave with more registers)
template <int T1>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) void k_gram_partial_sym(
    GramArgs g, double *__restrict__ part, int64_t rows_per_wg) {
    gram_partial_body<T1, 2 * T1, true>(g, part, rows_per_wg, blockIdx.x);
}

// batched over problems: blockIdx.y selects the job
template <int T1, int T2>
__global__ __launch_bounds__(256) void k_gram_partial_b(const GramJob *__restrict__ jobs) {
    const GramJob j = jobs[blockIdx.y];
    if ((int)blockIdx.x >= j.parts) return;
    gram_partial_body<T1, T2>(j.g, j.part, j.rpw, blockIdx.x);
}

// sum of the partial Gram matrices: 64 elements x 16 part-slices per
// 1024-thread workgroup, slices combined by a fixed tree (bitwise reproducible)
__device__ __forceinline__ void gram_final_body(const double *__restrict__ part, int nparts, int kk,
                                                double *__restrict__ out, int bx) {
    __shared__ double red[16][64];
    const int el = threadIdx.x & 63, sl = threadIdx.x >> 6;
    const int e = bx * 64 + el;
    // four independent chains per thread, so the loads of four part-slices
    // are in flight together; the order of the sums is fixed
    double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
    if (e < kk) {
        int p = sl;
        for (; p + 48 < nparts; p += 64) {
            const double a0 = part[(int64_t)p * kk + e], a1 = part[(int64_t)(p + 16) * kk + e];
            const double a2 = part[(int64_t)(p + 32) * kk + e], a3 = part[(int64_t)(p + 48) * kk + e];
            s0 += a0;
            s1 += a1;
            s2 += a2;
            s3 += a3;
        }
        for (; p < nparts; p += 16) s0 += part[(int64_t)p * kk + e];
    }
    red[sl][el] = (s0 + s1) + (s2 + s3);
    __syncthreads();
    for (int h = 8; h > 0; h >>= 1) {
        if (sl < h) red[sl][el] += red[sl + h][el];
        __syncthreads();
    }
    if (sl == 0 && e < kk) out[e] = red[0][el];
}

__global__ __launch_bounds__(1024) void k_gram_final(const double *__restrict__ part, int nparts, int kk,
                                                     double *__restrict__ out) {
    gram_final_body(part, nparts, kk, out, blockIdx.x);
}

__global__ __launch_bounds__(1024) void k_gram_final_b(const GramJob *__restrict__ jobs) {
    const GramJob j = jobs[blockIdx.y];
    if ((int)blockIdx.x * 64 >= j.kk) return;
    gram_final_body(j.part, j.parts, j.kk, j.out, blockIdx.x);
}

int gram_parts(int64_t n) {
    int64_t p = (n + 1023) / 1024;
    if (p > 1024) p = 1024;
    if (p < 1) p = 1;
    return (int)p;
}

size_t gram_scratch_bytes(int64_t n, int K1, int K2) { return (size_t)gram_parts(n) * K1 * K2 * sizeof(double); }

template <int T1, int T2>
static void gram_launch_t(const GramArgs &g, double *part, int parts, int64_t rpw, hipStream_t s) {
    hipLaunchKernelGGL((k_gram_partial<T1, T2>), dim3(parts), dim3(256), 0, s, g, part, rpw);
}

// rows per partial: a multiple of 64, shared by every kernel that writes
// Gram partials, so that all of them cut the rows alike
int64_t gram_rows(int64_t n, int parts) {
    int64_t rpw = (n + parts - 1) / parts;
    return (rpw + 63) / 64 * 64;
}

void gram(const GramArgs &g, double *out, double *scratch, hipStream_t s) {
    const int K1 = g.na * g.m, K2 = g.nb * g.m;
    const int T1 = (K1 + 15) / 16, T2 = (K2 + 15) / 16;
    const int parts = gram_parts(g.n);
    const int64_t rpw = gram_rows(g.n, parts);
    if (g.sym && K1 % 16 == 0 && g.nb == 2 * g.na) {
        // [S^T S | S^T A S]: the half-tile skipping needs the halves to start on a tile
#define GS(a) if (T1 == a) { hipLaunchKernelGGL((k_gram_partial_sym<a>), dim3(parts), dim3(256), 0, s, g, scratch, rpw); } else
        GS(1) GS(2) GS(3)
            fail(HSYM_E_UNSUPPORTED, "gram shape");
#undef GS
    } else {
#define GL(a, b) if (T1 == a && T2 == b) { gram_launch_t<a, b>(g, scratch, parts, rpw, s); } else
    GL(1, 1) GL(1, 2) GL(1, 3) GL(2, 1) GL(2, 2) GL(2, 3) GL(3, 1) GL(3, 2) GL(3, 3)
    GL(1, 4) GL(1, 6) GL(2, 4) GL(2, 5) GL(2, 6) GL(3, 4) GL(3, 5) GL(3, 6)
        fail(HSYM_E_UNSUPPORTED, "gram shape");
#undef GL
    }
    HIPCHK(hipGetLastError());
    const int kk = K1 * K2;
    hipLaunchKernelGGL(k_gram_final, dim3((kk + 63) / 64), dim3(1024), 0, s, scratch, parts, kk, out);
    HIPCHK(hipGetLastError());
}

// ---------------------------------------------------------------------------
// Linear combinations.  For every row r (one lane per row):
//   out_o[r, :] = sum_i in_i[r, :] C[i*m:(i+1)*m, o*m:(o+1)*m]
// for two sets sharing the coefficients (S = [X W P] and AS = [AX AW AP]).
// Rows of a set are read completely before they are written, so the outputs
// of a set may alias its inputs; an output of set 0 must not be an input of
// set 1 (set 1's rows are read while set 0's are written).  With theta !=
// NULL the kernel also forms the
// residual R = out_1_0 - out_0_0 diag(theta) of the new X (set 0, output 0)
// and its product AX (set 1, output 0), writes it to `res` and accumulates the
// squared column norms of R per workgroup.
// ---------------------------------------------------------------------------
// A workgroup (4 waves) walks lincomb_tiles_per_wg(n) consecutive tiles of 64
// rows, at most HSYM_LINCOMB_WGS workgroups in all; each wave computes 16 rows
// of a tile.  The MFMA A operands (lane: row li, four columns) are loaded
// straight from the input blocks and the B operands (coefficients, a few KB,
// cache resident) once per workgroup, so the kernel streams with no LDS
// staging and no barrier until the fixed-order reduction of the residual norms.
//
// Column of an input block that lane group lk feeds to the s4-th MFMA of a
// contraction over the block's m columns (any split of the columns into four
// groups of four serves, the same on both operands).  V16 (m = 16, 16-byte
// aligned blocks): columns 2lk, 2lk + 1, 8 + 2lk, 9 + 2lk, so that a lane
// loads its four values of a row with two 16-byte loads and the four lanes of
// a row read its first and its second 64 bytes in one instruction each.
template <bool V16>
__device__ __forceinline__ int lincomb_col(int s4, int lk) {
    return V16 ? 2 * lk + (s4 & 1) + 8 * (s4 >> 1) : 4 * s4 + lk;
}

template <bool V16>
__device__ __forceinline__ void lincomb_body(const LincombArgs &a, int64_t bx) {
    __shared__ double nred[4][4][16];
    if (a.skip && *a.skip) return;   // uniform: the flag was written by an earlier launch
    const int m = V16 ? 16 : a.m, nin = a.nin, nout = a.nout;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int li = lane & 15, lk = lane >> 4;
    // every coefficient this lane needs (MFMA B operands), loop-invariant
    double bv[2][3][4];
#pragma unroll
    for (int q = 0; q < 2; q++)
#pragma unroll
        for (int i = 0; i < 3; i++)
#pragma unroll
            for (int s4 = 0; s4 < 4; s4++) {
                const int kk = lincomb_col<V16>(s4, lk);
                bv[q][i][s4] = (q < nout && i < nin && kk < m && li < m)
                                   ? a.coef[(i * m + kk) * a.ldc + q * m + li] : 0.0;
            }
    double nrm = 0.0;
    const int64_t ntiles = (a.n + 63) / 64, tpw = lincomb_tiles_per_wg(a.n);
    const int64_t t_begin = bx * tpw;
    const int64_t t_end = (bx + 1) * tpw < ntiles ? (bx + 1) * tpw : ntiles;
    // The work is a sequence of steps (tile, set), set fastest.  A step loads
    // every input value of its set for this wave's 16 rows of the tile before
    // its first store (a wave reads and writes only its own rows, so the
    // outputs of a set may alias its inputs), and the next step's loads are in
    // flight while a step is combined and stored (the outputs of set 0 are not
    // inputs of set 1).
    auto load = [&](double (&av)[3][4], int64_t t, int set) {
        const int64_t ra = t * 64 + 16 * wave + li;
        const bool rok = ra < a.n;
#pragma unroll
        for (int i = 0; i < 3; i++) {
            if constexpr (V16) {
                double2 lo = make_double2(0.0, 0.0), hi = lo;
                if (i < nin && rok) {
                    const double *p = a.in[set * 3 + i] + ra * 16 + 2 * lk;
                    lo = *reinterpret_cast<const double2 *>(p);
                    hi = *reinterpret_cast<const double2 *>(p + 8);
                }
                av[i][0] = lo.x; av[i][1] = lo.y; av[i][2] = hi.x; av[i][3] = hi.y;
            } else {
#pragma unroll
                for (int s4 = 0; s4 < 4; s4++) {
                    const int kk = lincomb_col<V16>(s4, lk);
                    av[i][s4] = (i < nin && rok && kk < m) ? a.in[set * 3 + i][ra * m + kk] : 0.0;
                }
            }
        }
    };
    double4_t xkeep = (double4_t){0.0, 0.0, 0.0, 0.0};
    auto work = [&](const double (&av)[3][4], int64_t t, int set) {
        const int64_t w0 = t * 64 + 16 * wave;   // this wave's 16 rows
#pragma unroll
        for (int q = 0; q < 2; q++) {
            if (q >= nout) break;
            double4_t acc = (double4_t){0.0, 0.0, 0.0, 0.0};
#pragma unroll
            for (int i = 0; i < 3; i++) {
                if (i >= nin) break;
#pragma unroll
                for (int s4 = 0; s4 < 4; s4++) {
                    if (4 * s4 >= m) break;
                    acc = __builtin_amdgcn_mfma_f64_16x16x4f64(av[i][s4], bv[q][i][s4], acc, 0, 0, 0);
                }
            }
            // accumulator register v holds row lk + 4v, column li of this wave's 16 rows
            double *dst = a.out[set * 2 + q];
#pragma unroll
            for (int v = 0; v < 4; v++) {
                const int64_t r = w0 + lk + 4 * v;
                if (r < a.n && li < m) dst[r * m + li] = acc[v];
            }
            if (q == 0 && a.theta) {
                if (set == 0) {
                    xkeep = acc;
                } else {
                    const double th = li < m ? a.theta[li] : 0.0;
#pragma unroll
                    for (int v = 0; v < 4; v++) {
                        const int64_t r = w0 + lk + 4 * v;
                        if (r < a.n && li < m) {
                            const double rv = acc[v] - xkeep[v] * th;
                            a.res[r * m + li] = rv;
                            nrm += rv * rv;
                        }
                    }
                }
            }
        }
    };
    const int ns = a.nsets;
    const int64_t K = (t_end - t_begin) * ns;
    auto tile_of = [&](int64_t k) { return t_begin + (ns == 2 ? k >> 1 : k); };
    auto set_of = [&](int64_t k) { return ns == 2 ? (int)(k & 1) : 0; };
    double b0[3][4], b1[3][4];
    if (K > 0) load(b0, tile_of(0), set_of(0));
    for (int64_t k = 0; k < K; k += 2) {
        if (k + 1 < K) load(b1, tile_of(k + 1), set_of(k + 1));
        work(b0, tile_of(k), set_of(k));
        if (k + 1 >= K) break;
        if (k + 2 < K) load(b0, tile_of(k + 2), set_of(k + 2));
        work(b1, tile_of(k + 1), set_of(k + 1));
    }
    if (a.theta) {
        // squared column norms of R for this workgroup's rows, combined in a fixed order
        nred[wave][lk][li] = nrm;
        __syncthreads();
        if (tid < m) {
            double s = 0.0;
            for (int w = 0; w < 4; w++)
                for (int g = 0; g < 4; g++) s += nred[w][g][tid];
            a.norm_part[bx * m + tid] = s;
        }
    }
}

// three waves per SIMD (at most 168 registers; 1536 workgroups are two full
// rounds of the 256 CUs)
template <bool V16>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(3))) void k_lincomb(LincombArgs a) {
    lincomb_body<V16>(a, blockIdx.x);
}

__global__ __launch_bounds__(256) void k_lincomb_b(const LincombArgs *__restrict__ tab) {
    const LincombArgs a = tab[blockIdx.y];
    if ((int64_t)blockIdx.x >= lincomb_norm_parts(a.n)) return;
    lincomb_body<false>(a, blockIdx.x);
}

static bool aligned16(const void *p) { return ((uintptr_t)p & 15) == 0; }

void lincomb(const LincombArgs &a, hipStream_t s) {
    if (a.nin * a.m > 48 || a.nout * a.m > 32 || a.nout > 2 || a.nin > 3 || a.m > 16)
        fail(HSYM_E_UNSUPPORTED, "lincomb shape");
    bool v16 = a.m == 16;
    for (int set = 0; set < a.nsets; set++)
        for (int i = 0; i < a.nin; i++) v16 = v16 && aligned16(a.in[set * 3 + i]);
    const dim3 grid((unsigned)lincomb_norm_parts(a.n));
    if (v16) hipLaunchKernelGGL(k_lincomb<true>, grid, dim3(256), 0, s, a);
    else hipLaunchKernelGGL(k_lincomb<false>, grid, dim3(256), 0, s, a);
    HIPCHK(hipGetLastError());
}

// ---------------------------------------------------------------------------
// Linear combination with a Gram epilogue (m = 16): W' = [in] C (one set, one
// output) and the partial Gram matrices [A_0 .. A_{NA-2} W']^T W' of the rows
// the workgroup produced, so the Cholesky-QR pass that follows reads neither
// W' nor the A blocks again.  A workgroup walks rows_per_wg rows (a multiple
// of 64) in 64-row tiles, 16 rows per wave.  The accumulator of the linear
// combination holds W'[row lk + 4v][column li], which is exactly the operand
// layout of v_mfma_f64_16x16x4f64 for the Gram over the rows 4v .. 4v + 3;
// the A blocks are read again in that layout (rows the wave has just loaded,
// from cache).  Partials are laid out as those of k_gram_partial.
// ---------------------------------------------------------------------------
template <int NA>
__device__ __forceinline__ void lincomb_gram_body(const LincombArgs &l, const GramArgs &g, double *__restrict__ part,
                                                  int64_t rows_per_wg, int64_t bx) {
    __shared__ double red[4][NA * 16][17];
    if (l.skip && *l.skip) return;   // uniform: the flag was written by an earlier launch
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int li = lane & 15, lk = lane >> 4;
    const int nin = l.nin;
    // coefficients: loop-invariant MFMA B operands, the columns of the input
    // blocks split as in the linear combination (lincomb_col<true>)
    double bv[3][4];
#pragma unroll
    for (int i = 0; i < 3; i++)
#pragma unroll
        for (int s4 = 0; s4 < 4; s4++)
            bv[i][s4] = i < nin ? l.coef[(i * 16 + lincomb_col<true>(s4, lk)) * l.ldc + li] : 0.0;
    double4_t G[NA];
#pragma unroll
    for (int t = 0; t < NA; t++) G[t] = (double4_t){0.0, 0.0, 0.0, 0.0};
    const int64_t r_begin = bx * rows_per_wg;
    const int64_t r_end = (r_begin + rows_per_wg < l.n) ? r_begin + rows_per_wg : l.n;
    for (int64_t w0 = r_begin + 16 * wave; w0 < r_end; w0 += 64) {
        const int64_t ra = w0 + li;
        const bool rok = ra < r_end;
        double av[3][4];
#pragma unroll
        for (int i = 0; i < 3; i++) {
            double2 lo = make_double2(0.0, 0.0), hi = lo;
            if (i < nin && rok) {
                const double *p = l.in[i] + ra * 16 + 2 * lk;
                lo = *reinterpret_cast<const double2 *>(p);
                hi = *reinterpret_cast<const double2 *>(p + 8);
            }
            av[i][0] = lo.x; av[i][1] = lo.y; av[i][2] = hi.x; av[i][3] = hi.y;
        }
        // the A blocks in the Gram layout (row w0 + lk + 4v, column li)
        double ax[NA > 1 ? NA - 1 : 1][4];
#pragma unroll
        for (int t = 0; t < NA - 1; t++)
#pragma unroll
            for (int v = 0; v < 4; v++) {
                const int64_t r = w0 + lk + 4 * v;
                ax[t][v] = r < r_end ? g.a[t][r * 16 + li] : 0.0;
            }
        double4_t acc = (double4_t){0.0, 0.0, 0.0, 0.0};
#pragma unroll
        for (int i = 0; i < 3; i++) {
            if (i >= nin) break;
#pragma unroll
            for (int s4 = 0; s4 < 4; s4++) acc = __builtin_amdgcn_mfma_f64_16x16x4f64(av[i][s4], bv[i][s4], acc, 0, 0, 0);
        }
        double *dst = l.out[0];
#pragma unroll
        for (int v = 0; v < 4; v++) {
            const int64_t r = w0 + lk + 4 * v;
            if (r < r_end) dst[r * 16 + li] = acc[v];
        }
        // rows past r_end carry zero inputs, hence zero acc: they add nothing
#pragma unroll
        for (int v = 0; v < 4; v++) {
#pragma unroll
            for (int t = 0; t < NA - 1; t++) G[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(ax[t][v], acc[v], G[t], 0, 0, 0);
            G[NA - 1] = __builtin_amdgcn_mfma_f64_16x16x4f64(acc[v], acc[v], G[NA - 1], 0, 0, 0);
        }
    }
#pragma unroll
    for (int t = 0; t < NA; t++)
#pragma unroll
        for (int v = 0; v < 4; v++) red[wave][16 * t + lk + 4 * v][li] = G[t][v];
    __syncthreads();
    double *out = part + bx * (NA * 16) * 16;
    for (int e = tid; e < NA * 16 * 16; e += 256) {
        const int i = e >> 4, j = e & 15;
        out[e] = red[0][i][j] + red[1][i][j] + red[2][i][j] + red[3][i][j];
    }
}

template <int NA>
__global__ __launch_bounds__(256) void k_lincomb_gram(LincombArgs l, GramArgs g, double *__restrict__ part,
                                                      int64_t rows_per_wg) {
    lincomb_gram_body<NA>(l, g, part, rows_per_wg, blockIdx.x);
}

template <int NA>
__global__ __launch_bounds__(256) void k_lincomb_gram_b(const LincombArgs *__restrict__ lt,
                                                        const GramJob *__restrict__ gt) {
    const GramJob j = gt[blockIdx.y];
    if ((int)blockIdx.x >= j.parts) return;
    const LincombArgs l = lt[blockIdx.y];
    lincomb_gram_body<NA>(l, j.g, j.part, j.rpw, blockIdx.x);
}

bool lincomb_gram_fusable(const LincombArgs &l, const GramArgs &g) {
    bool al = true;
    for (int i = 0; i < l.nin; i++) al = al && aligned16(l.in[i]);
    return l.m == 16 && g.m == 16 && l.nsets == 1 && l.nout == 1 && !l.theta && l.nin >= 1 && l.nin <= 3 &&
           l.ldc == 16 && g.nb == 1 && g.na >= 1 && g.na <= 3 && g.b[0] == l.out[0] && g.a[g.na - 1] == l.out[0] &&
           l.n == g.n && al;
}

void lincomb_gram(const LincombArgs &l, const GramArgs &g, double *out, double *scratch, hipStream_t s) {
    if (!lincomb_gram_fusable(l, g)) {
        lincomb(l, s);
        gram(g, out, scratch, s);
        return;
    }
    const int parts = gram_parts(g.n);
    const int64_t rpw = gram_rows(g.n, parts);
    switch (g.na) {
        case 1: hipLaunchKernelGGL(k_lincomb_gram<1>, dim3(parts), dim3(256), 0, s, l, g, scratch, rpw); break;
        case 2: hipLaunchKernelGGL(k_lincomb_gram<2>, dim3(parts), dim3(256), 0, s, l, g, scratch, rpw); break;
        default: hipLaunchKernelGGL(k_lincomb_gram<3>, dim3(parts), dim3(256), 0, s, l, g, scratch, rpw); break;
    }
    HIPCHK(hipGetLastError());
    const int kk = g.na * 16 * 16;
    hipLaunchKernelGGL(k_gram_final, dim3((kk + 63) / 64), dim3(1024), 0, s, scratch, parts, kk, out);
    HIPCHK(hipGetLastError());
}

void lincomb_gram_batched(const LincombArgs *lt, const GramJob *gt, int count, int na, int max_parts,
                          hipStream_t s) {
    const dim3 grid((unsigned)max_parts, (unsigned)count);
    switch (na) {
        case 1: hipLaunchKernelGGL(k_lincomb_gram_b<1>, grid, dim3(256), 0, s, lt, gt); break;
        case 2: hipLaunchKernelGGL(k_lincomb_gram_b<2>, grid, dim3(256), 0, s, lt, gt); break;
        default: hipLaunchKernelGGL(k_lincomb_gram_b<3>, grid, dim3(256), 0, s, lt, gt); break;
    }
    HIPCHK(hipGetLastError());
    const int kk = na * 16 * 16;
    hipLaunchKernelGGL(k_gram_final_b, dim3((unsigned)((kk + 63) / 64), (unsigned)count), dim3(1024), 0, s, gt);
    HIPCHK(hipGetLastError());
}

// The Jacobi apply with a Gram epilogue (m = 16): W[r][c] /= g(d_r - mu_c)
// in place, and the partial Gram matrices [A_0 .. A_{NA-2} W]^T W of the
// workgroup's rows.  Rows and accumulation order are those of
// k_gram_partial, so the partials are the ones the two separate passes give.
template <int NA>
__global__ __launch_bounds__(256) void k_jacobi_gram(GramArgs g, const double *__restrict__ diag,
                                                     const double *__restrict__ mu, double delta,
                                                     double *__restrict__ part, int64_t rows_per_wg) {
    __shared__ double red[4][NA * 16][17];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const int li = lane & 15, lk = lane >> 4;
    double *W = const_cast<double *>(g.b[0]);
    const double muc = mu[li];
    double4_t G[NA];
#pragma unroll
    for (int t = 0; t < NA; t++) G[t] = (double4_t){0.0, 0.0, 0.0, 0.0};
    const int64_t r_begin = (int64_t)blockIdx.x * rows_per_wg;
    const int64_t r_end = (r_begin + rows_per_wg < g.n) ? r_begin + rows_per_wg : g.n;
    constexpr int GU = 4;
    for (int64_t r0 = r_begin + 4 * wave; r0 < r_end; r0 += 16 * GU) {
        double ax[GU][NA > 1 ? NA - 1 : 1], wv[GU], dg[GU];
#pragma unroll
        for (int u = 0; u < GU; u++) {
            const int64_t r = r0 + 16 * u + lk;
            const bool ok = r < r_end;
#pragma unroll
            for (int t = 0; t < NA - 1; t++) ax[u][t] = ok ? g.a[t][r * 16 + li] : 0.0;
            wv[u] = ok ? W[r * 16 + li] : 0.0;
            dg[u] = ok ? diag[r] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < GU; u++) {
            const int64_t r = r0 + 16 * u + lk;
            if (r < r_end) {
                wv[u] = wv[u] / guard_den(dg[u] - muc, delta);
                W[r * 16 + li] = wv[u];
            }
        }
#pragma unroll
        for (int u = 0; u < GU; u++) {
#pragma unroll
            for (int t = 0; t < NA - 1; t++) G[t] = __builtin_amdgcn_mfma_f64_16x16x4f64(ax[u][t], wv[u], G[t], 0, 0, 0);
            G[NA - 1] = __builtin_amdgcn_mfma_f64_16x16x4f64(wv[u], wv[u], G[NA - 1], 0, 0, 0);
        }
    }
#pragma unroll
    for (int t = 0; t < NA; t++)
#pragma unroll
        for (int v = 0; v < 4; v++) red[wave][16 * t + lk + 4 * v][li] = G[t][v];
    __syncthreads();
    double *out = part + (int64_t)blockIdx.x * (NA * 16) * 16;
    for (int e = tid; e < NA * 16 * 16; e += 256) {
        const int i = e >> 4, j = e & 15;
        out[e] = red[0][i][j] + red[1][i][j] + red[2][i][j] + red[3][i][j];
    }
}

bool jacobi_gram_fusable(const GramArgs &g) {
    return g.m == 16 && g.nb == 1 && g.na >= 1 && g.na <= 3 && g.b[0] == g.a[g.na - 1];
}

void jacobi_gram(const GramArgs &g, const double *diag, const double *mu, double delta, double *out,
                 double *scratch, hipStream_t s) {
    if (!jacobi_gram_fusable(g)) fail(HSYM_E_UNSUPPORTED, "jacobi_gram shape");
    const int parts = gram_parts(g.n);
    const int64_t rpw = gram_rows(g.n, parts);
    switch (g.na) {
        case 1: hipLaunchKernelGGL(k_jacobi_gram<1>, dim3(parts), dim3(256), 0, s, g, diag, mu, delta, scratch, rpw); break;
        case 2: hipLaunchKernelGGL(k_jacobi_gram<2>, dim3(parts), dim3(256), 0, s, g, diag, mu, delta, scratch, rpw); break;
        default: hipLaunchKernelGGL(k_jacobi_gram<3>, dim3(parts), dim3(256), 0, s, g, diag, mu, delta, scratch, rpw); break;
    }
    HIPCHK(hipGetLastError());
    const int kk = g.na * 16 * 16;
    hipLaunchKernelGGL(k_gram_final, dim3((kk + 63) / 64), dim3(1024), 0, s, scratch, parts, kk, out);
    HIPCHK(hipGetLastError());
}

// sum of per-workgroup partial column sums: one 1024-thread workgroup per
// column, strided partial sums combined by a fixed tree (bitwise reproducible)
__device__ __forceinline__ void colsum_body(const double *__restrict__ part, int64_t nparts, int m,
                                            double *__restrict__ out, int j) {
    __shared__ double red[1024];
    double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
    int64_t p = threadIdx.x;
    for (; p + 3072 < nparts; p += 4096) {
        const double a0 = part[p * m + j], a1 = part[(p + 1024) * m + j];
        const double a2 = part[(p + 2048) * m + j], a3 = part[(p + 3072) * m + j];
        s0 += a0;
        s1 += a1;
        s2 += a2;
        s3 += a3;
    }
    for (; p < nparts; p += 1024) s0 += part[p * m + j];
    red[threadIdx.x] = (s0 + s1) + (s2 + s3);
    __syncthreads();
    for (int off = 512; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[j] = red[0];
}

__global__ __launch_bounds__(1024) void k_colsum_final(const double *__restrict__ part, int64_t nparts, int m,
                                                       double *__restrict__ out) {
    colsum_body(part, nparts, m, out, blockIdx.x);
}

__global__ __launch_bounds__(1024) void k_colsum_final_b(const ColsumJob *__restrict__ jobs) {
    const ColsumJob j = jobs[blockIdx.y];
    colsum_body(j.part, j.nparts, j.m, j.out, blockIdx.x);
}

// *p = v as a kernel (a memset cannot be recorded in a captured graph)
__global__ void k_set_int(int *p, int v) { *p = v; }

void set_int(int *p, int v, hipStream_t s) {
    hipLaunchKernelGGL(k_set_int, dim3(1), dim3(1), 0, s, p, v);
    HIPCHK(hipGetLastError());
}

void colsum_final(const double *part, int64_t nparts, int m, double *out, hipStream_t s) {
    hipLaunchKernelGGL(k_colsum_final, dim3(m), dim3(1024), 0, s, part, nparts, m, out);
    HIPCHK(hipGetLastError());
}


// ---------------------------------------------------------------------------
// Preconditioners (eq. 11): T_j = Htilde - mu_j I, solved directly.
// The shifted denominators are kept at least delta away from zero.
// ---------------------------------------------------------------------------

// Elementwise over the row-major n x M block (coalesced): W[r][j] /= g(d_r - mu_j).
template <int M>
__global__ __launch_bounds__(256) void k_precond_jacobi(double *__restrict__ W, const double *__restrict__ diag,
                                                        const double *__restrict__ mu, double delta, int64_t n) {
    const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (e >= n * M) return;
    const int64_t r = e / M;
    const int j = (int)(e - r * M);
    W[e] = W[e] / guard_den(diag[r] - mu[j], delta);
}

template <int M>
__global__ __launch_bounds__(256) void k_precond_jacobi_b(const JacobiJob *__restrict__ jobs) {
    const JacobiJob jb = jobs[blockIdx.y];
    const int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (e >= jb.n * M) return;
    const int64_t r = e / M;
    const int j = (int)(e - r * M);
    jb.W[e] = jb.W[e] / guard_den(jb.diag[r] - jb.mu[j], jb.delta);
}

// One wave per 64-row chunk: W_b = Q diag(1/g(lambda - mu_j)) Q^T R_b.
// QT: the storage of the factors Q (fp64, or fp32 for fp32-storage handles; the
// products are fp64 either way)
template <typename QT>
__global__ __launch_bounds__(256) void k_precond_block64(double *__restrict__ W, const QT *__restrict__ Q,
                                                         const double *__restrict__ lam,
                                                         const double *__restrict__ mu, double delta, int64_t n,
                                                         int m) {
    // One wave per 64-row block, both products on the matrix cores
    // (v_mfma_f64_16x16x4f64; lane l: li = l & 15, lk = l >> 4; A operand
    // A[li][lk], B operand B[lk][li], accumulator v = row lk + 4v, column li):
    //   T = Q^T R as four 16-row tiles over 16 k-steps, the rows of tile tt
    //   taken in the order pi (A row li is T row 16 tt + pi(li)), so that
    //   accumulator v of tile tt in lane (li, lk) holds T row
    //   16 tt + 2 lk + (v & 1) + 8 (v >> 1); scaled row-wise by
    //   1/g(lambda_i - mu_j);
    //   then W = Q T over the k-steps (tt, v) with B operand = that
    //   accumulator, whose A operands Q[row][16 tt + 2 lk + {0, 1, 8, 9}] a
    //   lane loads with two 16-byte loads per row.
    const int lane = threadIdx.x & 63, li = lane & 15, lk = lane >> 4;
    const int64_t b = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    const int64_t r0 = b * 64;
    if (r0 >= n) return;   // whole wave
    const int rows = (int)((n - r0) < 64 ? (n - r0) : 64);
    const QT *Qb = Q + b * 64 * 64;
    const bool col = li < m;
    // R rows 4s + lk of column li, s = 0..15
    double rv[16];
#pragma unroll
    for (int s = 0; s < 16; s++) {
        const int k = 4 * s + lk;
        rv[s] = (col && k < rows) ? W[(r0 + k) * m + li] : 0.0;
    }
    // pi(x) = 2 (x & 3) + ((x >> 2) & 1) + 8 (x >> 3): a permutation of 0..15
    auto pi = [](int x) { return 2 * (x & 3) + ((x >> 2) & 1) + 8 * (x >> 3); };
    const int pli = pi(li);
    double4_t t[4];
#pragma unroll
    for (int tt = 0; tt < 4; tt++) {
        t[tt] = (double4_t){0.0, 0.0, 0.0, 0.0};
        double qa[16];
#pragma unroll
        for (int s = 0; s < 16; s++) qa[s] = (double)Qb[(4 * s + lk) * 64 + 16 * tt + pli];   // Q^T[16tt + pi(li)][4s + lk]
#pragma unroll
        for (int s = 0; s < 16; s++) t[tt] = __builtin_amdgcn_mfma_f64_16x16x4f64(qa[s], rv[s], t[tt], 0, 0, 0);
    }
    const double muj = col ? mu[li] : 0.0;
#pragma unroll
    for (int tt = 0; tt < 4; tt++)
#pragma unroll
        for (int v = 0; v < 4; v++) {
            const int i = 16 * tt + 2 * lk + (v & 1) + 8 * (v >> 1);   // = 16 tt + pi(lk + 4v)
            t[tt][v] = col ? t[tt][v] / guard_den(lam[b * 64 + i] - muj, delta) : 0.0;
        }
#pragma unroll
    for (int tt = 0; tt < 4; tt++) {
        double qa[16];
        const QT *qrow = Qb + (16 * tt + li) * 64 + 2 * lk;
#pragma unroll
        for (int q = 0; q < 4; q++) {
            if constexpr (sizeof(QT) == 8) {
                const double2 lo = *reinterpret_cast<const double2 *>(qrow + 16 * q);
                const double2 hi = *reinterpret_cast<const double2 *>(qrow + 16 * q + 8);
                qa[4 * q] = lo.x; qa[4 * q + 1] = lo.y; qa[4 * q + 2] = hi.x; qa[4 * q + 3] = hi.y;
            } else {
                const float2 lo = *reinterpret_cast<const float2 *>(qrow + 16 * q);
                const float2 hi = *reinterpret_cast<const float2 *>(qrow + 16 * q + 8);
                qa[4 * q] = lo.x; qa[4 * q + 1] = lo.y; qa[4 * q + 2] = hi.x; qa[4 * q + 3] = hi.y;
            }
        }
        double4_t w = (double4_t){0.0, 0.0, 0.0, 0.0};
        // k-step (q, v): Q[16tt + li][16q + 2lk + (v & 1) + 8 (v >> 1)] times T of that row
#pragma unroll
        for (int s = 0; s < 16; s++) w = __builtin_amdgcn_mfma_f64_16x16x4f64(qa[s], t[s >> 2][s & 3], w, 0, 0, 0);
#pragma unroll
        for (int v = 0; v < 4; v++) {
            const int i = 16 * tt + lk + 4 * v;
            if (col && i < rows) W[(r0 + i) * m + li] = w[v];
        }
    }
}

// ---------------------------------------------------------------------------
// Tile-diagonal preconditioner (end of Section 3.2, Section 4.3): for every
// diagonal group tile (rows [a, a+s), s <= 64, dense in LDS) and every column
// j, `iters` steps of the full orthogonalization method (Saad, Algorithm 6.4)
// on (Ht - mu_j I) w = r_j, started from w = 0: Arnoldi with modified
// Gram-Schmidt from v_1 = r_j / ||r_j||, stopped early when the next basis
// vector vanishes, then w = V y with H y = ||r_j|| e_1 solved by Gaussian
// elimination with partial pivoting, pivots kept delta away from zero.
// One wave per column (lane = tile row); the inner products are butterfly
// sums, identical in every lane.
// ---------------------------------------------------------------------------
constexpr int FOM_KMAX = 4;

__global__ __launch_bounds__(1024) void k_precond_fom(double *__restrict__ W, const int64_t *__restrict__ gstart,
                                                      const int64_t *__restrict__ goff,
                                                      const double *__restrict__ gdense,
                                                      const double *__restrict__ mu, double delta, int iters,
                                                      int m) {
    __shared__ double Ht[64][65];
    __shared__ double vs[16][64];
    const int64_t t = blockIdx.x;
    const int64_t a = gstart[t];
    const int s = (int)(gstart[t + 1] - a);
    const double *D = gdense + goff[t];
    // the tile, zero-padded to 64 x 64: four loads per thread in flight at once
    for (int e0 = threadIdx.x; e0 < 64 * 64; e0 += 4 * blockDim.x) {
        double v[4];
#pragma unroll
        for (int u = 0; u < 4; u++) {
            const int e = e0 + u * blockDim.x, r = e >> 6, c = e & 63;
            v[u] = (e < 64 * 64 && r < s && c < s) ? D[r * s + c] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < 4; u++) {
            const int e = e0 + u * blockDim.x;
            if (e < 64 * 64) Ht[e >> 6][e & 63] = v[u];
        }
    }
    __syncthreads();
    // from here on the waves (columns) are independent: no further barrier
    const int lane = threadIdx.x & 63, j = threadIdx.x >> 6;
    if (j >= m) return;
    const bool in = lane < s;
    const double shift = mu[j];
    const double b = in ? W[(a + lane) * m + j] : 0.0;
    const double beta = sqrt(wave_sum(b * b));
    if (beta == 0.0) {
        if (in) W[(a + lane) * m + j] = 0.0;
        return;
    }
    double V[FOM_KMAX + 1];
    double Hh[FOM_KMAX + 1][FOM_KMAX];
#pragma unroll
    for (int i = 0; i <= FOM_KMAX; i++) {
        V[i] = 0.0;
#pragma unroll
        for (int k = 0; k < FOM_KMAX; k++) Hh[i][k] = 0.0;
    }
    V[0] = b / beta;
    int kk = iters;
#pragma unroll
    for (int i = 0; i < FOM_KMAX; i++) {
        if (i >= iters) break;
        vs[j][lane] = V[i];
        __builtin_amdgcn_wave_barrier();
        // (T v)_lane over the s columns of the tile (zero past s), four chains
        double w0 = 0.0, w1 = 0.0, w2 = 0.0, w3 = 0.0;
        for (int c = 0; c < s; c += 4) {
            w0 = fma(Ht[lane][c], vs[j][c], w0);
            w1 = fma(Ht[lane][c + 1], vs[j][c + 1], w1);
            w2 = fma(Ht[lane][c + 2], vs[j][c + 2], w2);
            w3 = fma(Ht[lane][c + 3], vs[j][c + 3], w3);
        }
        double w = (w0 + w1) + (w2 + w3);
        __builtin_amdgcn_wave_barrier();
        w = in ? w - shift * V[i] : 0.0;
#pragma unroll
        for (int l = 0; l <= i; l++) {
            const double h = wave_sum(w * V[l]);
            Hh[l][i] = h;
            w -= h * V[l];
        }
        const double hn = sqrt(wave_sum(w * w));
        Hh[i + 1][i] = hn;
        const bool live = hn > 1e-14 * beta;
        if (live) V[i + 1] = w / hn;
        if (!live || i + 1 == iters) {
            kk = i + 1;
            break;
        }
    }
    // H y = beta e_1 (kk x kk upper Hessenberg), the same in every lane
    double T[FOM_KMAX][FOM_KMAX], rhs[FOM_KMAX], y[FOM_KMAX];
#pragma unroll
    for (int r = 0; r < FOM_KMAX; r++) {
        rhs[r] = r == 0 ? beta : 0.0;
        y[r] = 0.0;
#pragma unroll
        for (int c = 0; c < FOM_KMAX; c++) T[r][c] = Hh[r][c];
    }
#pragma unroll
    for (int c = 0; c < FOM_KMAX; c++) {
        if (c >= kk) break;
        int p = c;
#pragma unroll
        for (int r = c + 1; r < FOM_KMAX; r++)
            if (r < kk && fabs(T[r][c]) > fabs(T[p][c])) p = r;
        if (p != c) {
#pragma unroll
            for (int q = 0; q < FOM_KMAX; q++) {
                const double x = T[c][q];
                T[c][q] = T[p][q];
                T[p][q] = x;
            }
            const double x = rhs[c];
            rhs[c] = rhs[p];
            rhs[p] = x;
        }
        T[c][c] = guard_den(T[c][c], delta);
#pragma unroll
        for (int r = c + 1; r < FOM_KMAX; r++) {
            if (r >= kk) break;
            const double f = T[r][c] / T[c][c];
#pragma unroll
            for (int q = 0; q < FOM_KMAX; q++)
                if (q >= c) T[r][q] -= f * T[c][q];
            rhs[r] -= f * rhs[c];
        }
    }
#pragma unroll
    for (int c = FOM_KMAX - 1; c >= 0; c--) {
        if (c >= kk) continue;
        double acc = rhs[c];
#pragma unroll
        for (int q = 0; q < FOM_KMAX; q++)
            if (q > c && q < kk) acc -= T[c][q] * y[q];
        y[c] = acc / T[c][c];
    }
    double x = 0.0;
#pragma unroll
    for (int i = 0; i < FOM_KMAX; i++)
        if (i < kk) x = fma(V[i], y[i], x);
    if (in) W[(a + lane) * m + j] = x;
}

// ---------------------------------------------------------------------------
// Batched launches: one launch runs the same step for `count` problems whose
// arguments sit in a device table; blockIdx.y selects the problem and the
// blocks a smaller problem does not need return at once.
// ---------------------------------------------------------------------------
void gram_batched(const GramJob *jobs, int count, int K1, int K2, int max_parts, hipStream_t s) {
    const int T1 = (K1 + 15) / 16, T2 = (K2 + 15) / 16;
    const dim3 grid((unsigned)max_parts, (unsigned)count);
#define GB(a, b) if (T1 == a && T2 == b) { hipLaunchKernelGGL((k_gram_partial_b<a, b>), grid, dim3(256), 0, s, jobs); } else
    GB(1, 1) GB(1, 2) GB(1, 3) GB(2, 1) GB(2, 2) GB(2, 3) GB(3, 1) GB(3, 2) GB(3, 3)
    GB(1, 4) GB(1, 6) GB(2, 4) GB(2, 5) GB(2, 6) GB(3, 4) GB(3, 5) GB(3, 6)
        fail(HSYM_E_UNSUPPORTED, "gram shape");
#undef GB
    HIPCHK(hipGetLastError());
    hipLaunchKernelGGL(k_gram_final_b, dim3((unsigned)((K1 * K2 + 63) / 64), (unsigned)count), dim3(1024), 0, s, jobs);
    HIPCHK(hipGetLastError());
}

void lincomb_batched(const LincombArgs *tab, int count, int64_t max_n, hipStream_t s) {
    // every job's workgroup count (lincomb_norm_parts) is at most
    // min(HSYM_LINCOMB_WGS, its tiles of 64 rows)
    const int64_t gx = std::min<int64_t>(HSYM_LINCOMB_WGS, (max_n + 63) / 64);
    hipLaunchKernelGGL(k_lincomb_b, dim3((unsigned)std::max<int64_t>(gx, 1), (unsigned)count), dim3(256), 0, s, tab);
    HIPCHK(hipGetLastError());
}

void colsum_batched(const ColsumJob *jobs, int count, int m, hipStream_t s) {
    hipLaunchKernelGGL(k_colsum_final_b, dim3((unsigned)m, (unsigned)count), dim3(1024), 0, s, jobs);
    HIPCHK(hipGetLastError());
}

void jacobi_batched(const JacobiJob *jobs, int count, int m, int64_t max_n, hipStream_t s) {
    const dim3 grid((unsigned)((max_n * m + 255) / 256), (unsigned)count);
    switch (m) {
#define HSYM_JB(MM) case MM: hipLaunchKernelGGL(k_precond_jacobi_b<MM>, grid, dim3(256), 0, s, jobs); break;
        HSYM_JB(1) HSYM_JB(2) HSYM_JB(3) HSYM_JB(4) HSYM_JB(5) HSYM_JB(6) HSYM_JB(7) HSYM_JB(8)
        HSYM_JB(9) HSYM_JB(10) HSYM_JB(11) HSYM_JB(12) HSYM_JB(13) HSYM_JB(14) HSYM_JB(15) HSYM_JB(16)
#undef HSYM_JB
        default: fail(HSYM_E_INVALID_ARG, "block width must be 1..16");
    }
    HIPCHK(hipGetLastError());
}

__global__ void k_set_ints(int *const *__restrict__ p, int count, int v) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i < count) *p[i] = v;
}

void set_ints(int *const *p, int count, int v, hipStream_t s) {
    hipLaunchKernelGGL(k_set_ints, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, s, p, count, v);
    HIPCHK(hipGetLastError());
}

// dst[i*words .. (i+1)*words) = src[i][0 .. words), 32-bit words, one workgroup per item
__global__ __launch_bounds__(64) void k_gather_words(const int *const *__restrict__ src, int *__restrict__ dst,
                                                     int words) {
    const int *a = src[blockIdx.x];
    for (int w = threadIdx.x; w < words; w += 64) dst[(int64_t)blockIdx.x * words + w] = a[w];
}

void gather_words(const int *const *src, int *dst, int words, int count, hipStream_t s) {
    hipLaunchKernelGGL(k_gather_words, dim3((unsigned)count), dim3(64), 0, s, src, dst, words);
    HIPCHK(hipGetLastError());
}

void precond_apply(hsym_matrix *H, int kind, double *W, const double *mu, double delta, int m, hipStream_t s,
                   int fom_iters) {
    const int64_t n = H->n;
    if (kind == HSYM_PRECOND_FOM) {
        if (!H->tg_dense) fail(HSYM_E_INVALID_ARG, "FOM preconditioner needs hsym_attach_group_tiles");
        if (fom_iters < 1 || fom_iters > FOM_KMAX) fail(HSYM_E_INVALID_ARG, "fom_iters must be in [1, 4]");
        if (m < 1 || m > 16) fail(HSYM_E_INVALID_ARG, "block width must be 1..16");
        hipLaunchKernelGGL(k_precond_fom, dim3((unsigned)H->ntg), dim3((unsigned)(64 * m)), 0, s, W, H->tg_start,
                           H->tg_off, H->tg_dense, mu, delta, fom_iters, m);
        HIPCHK(hipGetLastError());
        return;
    }
    if (kind == HSYM_PRECOND_JACOBI) {
        const unsigned grid = (unsigned)((n * m + 255) / 256);
        switch (m) {
#define HSYM_JAC(MM) case MM: hipLaunchKernelGGL(k_precond_jacobi<MM>, dim3(grid), dim3(256), 0, s, W, H->diag64, mu, delta, n); break;
            HSYM_JAC(1) HSYM_JAC(2) HSYM_JAC(3) HSYM_JAC(4) HSYM_JAC(5) HSYM_JAC(6) HSYM_JAC(7) HSYM_JAC(8)
            HSYM_JAC(9) HSYM_JAC(10) HSYM_JAC(11) HSYM_JAC(12) HSYM_JAC(13) HSYM_JAC(14) HSYM_JAC(15) HSYM_JAC(16)
#undef HSYM_JAC
            default: fail(HSYM_E_INVALID_ARG, "block width must be 1..16");
        }
    } else if (kind == HSYM_PRECOND_BLOCK64) {
        const dim3 grid((unsigned)((n + 255) / 256));
        if (H->pre_q32)
            hipLaunchKernelGGL(k_precond_block64<float>, grid, dim3(256), 0, s, W, (const float *)H->pre_q,
                               H->pre_lam, mu, delta, n, m);
        else
            hipLaunchKernelGGL(k_precond_block64<double>, grid, dim3(256), 0, s, W, (const double *)H->pre_q,
                               H->pre_lam, mu, delta, n, m);
    }
    HIPCHK(hipGetLastError());
}

// fp64 -> fp32 copy of a block (mixed-precision SpMM input)
__global__ void k_to_f32(const double *__restrict__ x, float *__restrict__ y, int64_t cnt) {
    int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (e < cnt) y[e] = (float)x[e];
}

// --- counter-based Gaussian generator (same definition as the input generator) ---
__device__ __forceinline__ uint64_t mix64(uint64_t z) {
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}
__device__ __forceinline__ double unif(uint64_t key, uint64_t a, uint64_t b) {
    const uint64_t G = 0x9E3779B97F4A7C15ULL;
    uint64_t ctr = (a << 32) | (b & 0xffffffffULL);
    return (double)(mix64(key + (ctr + 1ULL) * G) >> 11) * (1.0 / 9007199254740992.0);
}

__global__ void k_gauss(double *__restrict__ V, int64_t n, int m, int64_t ld, uint64_t key, int mask) {
    int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (e >= n * m) return;
    int64_t i = e / m;
    int j = (int)(e - i * m);
    if (!((mask >> j) & 1)) return;
    double u1 = unif(key, (uint64_t)i, 2 * (uint64_t)j), u2 = unif(key, (uint64_t)i, 2 * (uint64_t)j + 1);
    V[i * ld + j] = sqrt(-2.0 * log(1.0 - u1)) * cos(6.283185307179586476925286766559 * u2);
}

void gauss_fill(double *V, int64_t n, int m, int64_t ld, uint64_t seed, uint64_t purpose, int mask,
                hipStream_t s) {
    const uint64_t G = 0x9E3779B97F4A7C15ULL;
    auto hmix = [](uint64_t z) {
        z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
        z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
        return z ^ (z >> 31);
    };
    uint64_t key = hmix(hmix(seed + G) ^ (purpose * G));
    hipLaunchKernelGGL(k_gauss, dim3((unsigned)((n * m + 255) / 256)), dim3(256), 0, s, V, n, m, ld, key, mask);
    HIPCHK(hipGetLastError());
}

// --- sign convention of returned eigenvectors ---
struct AbsMax { double a; double v; int64_t r; };

__global__ __launch_bounds__(256) void k_absmax_part(const double *__restrict__ X, int m, int nev, int64_t n,
                                                     int64_t rows_per, AbsMax *__restrict__ part) {
    __shared__ AbsMax red[256];
    for (int j = 0; j < nev; j++) {
        AbsMax best = {-1.0, 0.0, 0};
        int64_t r0 = (int64_t)blockIdx.x * rows_per, r1 = r0 + rows_per < n ? r0 + rows_per : n;
        for (int64_t r = r0 + threadIdx.x; r < r1; r += 256) {
            double v = X[r * m + j], a = fabs(v);
            if (a > best.a) { best.a = a; best.v = v; best.r = r; }
        }
        red[threadIdx.x] = best;
        __syncthreads();
        for (int off = 128; off > 0; off >>= 1) {
            if ((int)threadIdx.x < off) {
                AbsMax o = red[threadIdx.x + off], c = red[threadIdx.x];
                if (o.a > c.a || (o.a == c.a && o.r < c.r)) red[threadIdx.x] = o;
            }
            __syncthreads();
        }
        if (threadIdx.x == 0) part[(int64_t)blockIdx.x * nev + j] = red[0];
        __syncthreads();
    }
}

__global__ __launch_bounds__(256) void k_sign_copy(const double *__restrict__ X, int m, int nev, int64_t n,
                                                   const AbsMax *__restrict__ part, int nparts,
                                                   double *__restrict__ out) {
    __shared__ double sg[16];
    if ((int)threadIdx.x < nev) {
        AbsMax b = {-1.0, 0.0, 0};
        for (int p = 0; p < nparts; p++) {
            AbsMax o = part[(int64_t)p * nev + threadIdx.x];
            if (o.a > b.a || (o.a == b.a && o.r < b.r)) b = o;
        }
        sg[threadIdx.x] = b.v < 0 ? -1.0 : 1.0;
    }
    __syncthreads();
    int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (e >= n * nev) return;
    int64_t r = e / nev;
    int j = (int)(e - r * nev);
    out[e] = sg[j] * X[r * m + j];
}

static int absmax_parts(int64_t n) {
    int64_t p = (n + 4095) / 4096;
    return (int)(p > 1024 ? 1024 : (p < 1 ? 1 : p));
}

size_t sign_fix_scratch_bytes(int64_t n, int m) { return (size_t)absmax_parts(n) * m * sizeof(AbsMax); }

void sign_fix_copy(const double *X, int m, int nev, int64_t n, double *evecs, double *scratch, hipStream_t s) {
    int parts = absmax_parts(n);
    int64_t rows_per = (n + parts - 1) / parts;
    hipLaunchKernelGGL(k_absmax_part, dim3(parts), dim3(256), 0, s, X, m, nev, n, rows_per, (AbsMax *)scratch);
    HIPCHK(hipGetLastError());
    hipLaunchKernelGGL(k_sign_copy, dim3((unsigned)((n * nev + 255) / 256)), dim3(256), 0, s, X, m, nev, n,
                       (const AbsMax *)scratch, parts, evecs);
    HIPCHK(hipGetLastError());
}

void to_f32(const double *x, float *y, int64_t cnt, hipStream_t s) {
    hipLaunchKernelGGL(k_to_f32, dim3((unsigned)((cnt + 255) / 256)), dim3(256), 0, s, x, y, cnt);
    HIPCHK(hipGetLastError());
}

// ---------------------------------------------------------------------------
// Lanczos helpers: V is k x n (one basis vector per row, contiguous).
// h = V^T w (one workgroup per basis vector), then w -= V^T h.
// ---------------------------------------------------------------------------
// h[j] = V_j . w for the k vectors V_j (each n long, ld ldv): every
// workgroup takes DOT_ROWS rows of all k vectors (w staged once in LDS, one
// wave per vector at a time), then one workgroup per vector sums the
// per-chunk partials in a fixed order.
constexpr int DOT_ROWS = 2048;

int dots_parts(int64_t n) { return (int)((n + DOT_ROWS - 1) / DOT_ROWS); }

size_t dots_scratch_bytes(int64_t n, int k) { return (size_t)dots_parts(n) * (size_t)k * sizeof(double); }

__global__ __launch_bounds__(256) void k_dots_part(const double *__restrict__ V, int64_t ldv,
                                                   const double *__restrict__ w, int64_t n, int k,
                                                   double *__restrict__ part) {
    __shared__ double ws[DOT_ROWS];
    const int64_t r0 = (int64_t)blockIdx.x * DOT_ROWS;
    const int rows = (int)((n - r0) < DOT_ROWS ? (n - r0) : DOT_ROWS);
    for (int i = threadIdx.x; i < DOT_ROWS; i += 256) ws[i] = i < rows ? w[r0 + i] : 0.0;
    __syncthreads();
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int j = wave; j < k; j += 4) {
        const double *v = V + (int64_t)j * ldv + r0;
        double s0 = 0.0, s1 = 0.0;
        int i = lane;
        for (; i + 64 < rows; i += 128) {
            s0 = fma(v[i], ws[i], s0);
            s1 = fma(v[i + 64], ws[i + 64], s1);
        }
        if (i < rows) s0 = fma(v[i], ws[i], s0);
        double t = s0 + s1;
        for (int off = 32; off > 0; off >>= 1) t += __shfl_down(t, off, 64);
        if (lane == 0) part[(int64_t)blockIdx.x * k + j] = t;
    }
}

__global__ __launch_bounds__(256) void k_dots_final(const double *__restrict__ part, int nparts, int k,
                                                    double *__restrict__ h) {
    __shared__ double red[256];
    const int j = blockIdx.x;
    double s = 0.0;
    for (int c = threadIdx.x; c < nparts; c += 256) s += part[(int64_t)c * k + j];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x == 0) h[j] = red[0];
}

__global__ __launch_bounds__(256) void k_sub_vh(const double *__restrict__ V, int64_t ldv, const double *__restrict__ h,
                                                int k, double *__restrict__ w, int64_t n) {
    __shared__ double hs[1024];
    for (int i = threadIdx.x; i < k && i < 1024; i += 256) hs[i] = h[i];
    __syncthreads();
    const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    double s = 0.0;
    for (int j = 0; j < k; j++) s = fma(hs[j], V[(int64_t)j * ldv + i], s);
    w[i] -= s;
}

void dots(const double *V, int64_t ldv, int k, const double *w, int64_t n, double *h, double *scratch,
          hipStream_t s) {
    const int parts = dots_parts(n);
    hipLaunchKernelGGL(k_dots_part, dim3((unsigned)parts), dim3(256), 0, s, V, ldv, w, n, k, scratch);
    HIPCHK(hipGetLastError());
    hipLaunchKernelGGL(k_dots_final, dim3((unsigned)k), dim3(256), 0, s, scratch, parts, k, h);
    HIPCHK(hipGetLastError());
}

void sub_vh(const double *V, int64_t ldv, const double *h, int k, double *w, int64_t n, hipStream_t s) {
    for (int j0 = 0; j0 < k; j0 += 1024) {
        int kk = k - j0 < 1024 ? k - j0 : 1024;
        hipLaunchKernelGGL(k_sub_vh, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, V + (int64_t)j0 * ldv, ldv,
                           h + j0, kk, w, n);
        HIPCHK(hipGetLastError());
    }
}

// w = (w - a*v1 - b*v0) ; used by the three-term recurrence
__global__ void k_axpby2(double *__restrict__ w, const double *__restrict__ v1, const double *__restrict__ ab,
                         const double *__restrict__ v0, int64_t n) {
    int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    double r = w[i] - ab[0] * v1[i];
    if (v0) r -= ab[1] * v0[i];
    w[i] = r;
}

void axpby2(double *w, const double *v1, const double *ab, const double *v0, int64_t n, hipStream_t s) {
    hipLaunchKernelGGL(k_axpby2, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, w, v1, ab, v0, n);
    HIPCHK(hipGetLastError());
}

__global__ void k_scale_to(const double *__restrict__ w, const double *__restrict__ nrm2, double *__restrict__ v,
                           int64_t n) {
    int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    v[i] = w[i] / sqrt(nrm2[0]);
}

void scale_to(const double *w, const double *nrm2, double *v, int64_t n, hipStream_t s) {
    hipLaunchKernelGGL(k_scale_to, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, w, nrm2, v, n);
    HIPCHK(hipGetLastError());
}

}  // namespace hsym
