// Internal declarations shared by the host code and the HIP kernels of libhsym.
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>
#include <functional>
#include <string>
#include <vector>

#include "../../include/hsym.h"

namespace hsym {

// Elements of an X row that one lane of the SpMM handles: 2 (one 16-byte LDS
// read at fp64, 8 bytes at fp32), so that a run's flush issues two fp64 LDS
// atomics per lane, the count measured fastest on gfx950 (four per lane, as
// 32-byte fp64 or 16-byte fp32 lanes need, run at half the rate; with the
// record format of the pieces, four elements per lane measured 18-37% slower).
// HSYM_LANE_ELEMS overrides it at build time, for such measurements.
#ifndef HSYM_LANE_ELEMS
#define HSYM_LANE_ELEMS 2
#endif
__host__ __device__ constexpr int spmm_lane_elems(int M) { return M < HSYM_LANE_ELEMS ? M : HSYM_LANE_ELEMS; }
// 16-byte units of a staged piece per thread of the 1024-thread SpMM
// workgroup: 8 at block widths 1 and 2 (the X rows and accumulators then leave
// room for larger pieces and the kernel for the registers), else 4.
__host__ __device__ constexpr int spmm_stage_units(int M) { return M <= 2 ? 8 : 4; }
// Elements of padding after each X row the SpMM stages in LDS (block widths of
// 4 and more), so that the rows gathered by one wave start on more banks.
#ifndef HSYM_XPAD
#define HSYM_XPAD 0
#endif
__host__ __device__ constexpr int spmm_xpad(int M) { return M >= 4 ? HSYM_XPAD : 0; }


// block widths are rounded up to the next of 1, 2, 4, 8, 16 for the kernels
inline int round_m(int m) { return m <= 1 ? 1 : m <= 2 ? 2 : m <= 4 ? 4 : m <= 8 ? 8 : 16; }

// ---------------------------------------------------------------------------
// Errors: every entry point converts failures into a status and a message.
// ---------------------------------------------------------------------------
struct Error {
    int status;
    std::string msg;
};
void set_error(const std::string &msg);
[[noreturn]] void fail(int status, const std::string &msg);
void check_hip(hipError_t e, const char *what);
#define HIPCHK(x) ::hsym::check_hip((x), #x)

// ---------------------------------------------------------------------------
// Tile format of the stored upper triangle (compressed sparse blocks,
// Section 4.2: independently addressable blocks whose entries carry indices
// local to the block).  Rows are cut into panels of R rows and columns into
// chunks of C columns (C a power of two dividing R).  The strictly-upper
// entries of one panel that fall into one chunk form a tile; a tile with more
// than MAXE entries is cut into pieces of consecutive entries.  A piece of cnt
// entries is padded to E = G * len positions (len even) and stored as one
// contiguous run of bytes (16-byte aligned).  Its entries are known in two
// orders, each cut into G segments of len steps, the two steps 2t and 2t + 1
// of segment g sitting next to each other at positions 2tG + 2g and
// 2tG + 2g + 1 (piece_pos):
//   - the row-major order (rows ascending, columns ascending within a row),
//     which holds the entries themselves: their code, local row << cb | local
//     column (cb = log2 C), and their value (T);
//   - the column-major order, as a perm: at each position the position of the
//     entry in the row-major order.
// With 16-bit codes (R * C <= 2^16) code and perm share one 32-bit word,
// code << 16 | perm (the perm at the same position, not of the same entry):
// fp32 values sit next to their word in 8-byte records; fp64 values follow
// the words (a part of their own).  With 32-bit codes the codes, the perm
// (16-bit) and the values are three parts.  Every part starts on 16 bytes
// (piece_parts).  Padding positions repeat the code of the piece's last entry
// with value 0.
// A tile is "own" when its chunk lies inside the panel (its transposed half
// lands in the panel's rows) and "external" otherwise.
// ---------------------------------------------------------------------------
// steps per segment are a multiple of this (the SpMM takes two per batch)
constexpr int SPMM_STEP = 2;
// position of step s of segment g in a piece of G segments (steps paired)
static_assert(SPMM_STEP == 2, "piece_pos pairs the steps of a batch");
__host__ __device__ inline int64_t piece_pos(int64_t s, int64_t g, int64_t G) {
    return (s >> 1) * 2 * G + 2 * g + (s & 1);
}
struct PieceParts {
    int64_t perm;    // byte offset of the perm part (32-bit codes), else 0
    int64_t val;     // byte offset of the first value
    int64_t bytes;   // bytes of the piece (a multiple of 16)
};
__host__ __device__ inline PieceParts piece_parts(int64_t E, int idx_bytes, int val_bytes) {
    PieceParts p;
    const int64_t w16 = (4 * E + 15) & ~(int64_t)15;
    if (idx_bytes == 2 && val_bytes == 4) {
        p.perm = 0; p.val = 4; p.bytes = 8 * E;
    } else if (idx_bytes == 2) {
        p.perm = 0; p.val = w16; p.bytes = w16 + 8 * E;
    } else {
        p.perm = w16;
        p.val = w16 + ((2 * E + 15) & ~(int64_t)15);
        p.bytes = p.val + ((E * val_bytes + 15) & ~(int64_t)15);
    }
    return p;
}

struct TileDesc {
    int64_t base;          // first byte of the piece (a multiple of 16)
    int32_t len;           // steps per segment
    int32_t chunk;         // global chunk index g: columns [g*C, g*C+C)
    int32_t ext;           // 1 for an external tile, 0 for an own tile
    int32_t flags;         // TILE_FIRST: first piece of its tile; TILE_LAST: last piece
};
enum { TILE_FIRST = 1, TILE_LAST = 2 };

// panel geometry of a handle
struct Geom {
    int R = 0, C = 0;      // panel rows, chunk columns
    int cb = 0;            // log2 C
    int G = 0;             // segments per piece
    int maxe = 0;          // entries per piece at most (a multiple of 8)
    int idx_bytes = 2;     // code width
};

struct DeviceTiles {
    Geom g;
    int64_t npanels = 0, nchunks = 0, ntiles = 0, npieces = 0, nentries = 0, next = 0;
    int64_t *panel_tile_ptr = nullptr;   // pieces of panel p: [ptp[p], ptp[p+1])
    int32_t *panel_order = nullptr;      // panel of workgroup b (see build.cpp: per-XCD runs)
    TileDesc *tiles = nullptr;
    unsigned char *blob = nullptr;       // the pieces
    int64_t nbytes = 0;
    int64_t bytes = 0;
};

}  // namespace hsym

struct hsym_matrix {
    int64_t n = 0;
    int64_t nnz = 0;              // stored entries incl. diagonal
    int storage = HSYM_FP64;
    double norm1 = 0.0;
    int device = 0;
    // diagonal in both precisions
    double *diag64 = nullptr;
    float *diag32 = nullptr;
    // tile format of the strictly-upper part (one panel geometry per handle)
    hsym::DeviceTiles tiles;
    int geom_m = 16;              // block width the geometry is sized for
    int geom_r64 = 0, geom_lc = 0; // explicit panel rows / 64 and log2 chunk columns (0: automatic)
    std::vector<double> d_host;   // diagonal, fp64, host copy
    std::vector<double> colsum;   // absolute column sums (streaming create)
    // block-64 preconditioner: per 64-row chunk Q (64x64, row-major) and lambda;
    // Q is fp32 for fp32 storage (pre_q32), else fp64
    void *pre_q = nullptr;
    bool pre_q32 = false;
    double *pre_lam = nullptr;
    int64_t pre_nchunks = 0;
    // diagonal group tiles (FOM preconditioner): tile t covers rows
    // [tg_start[t], tg_start[t+1]) (at most 64), dense fp64 at tg_dense + tg_off[t]
    int64_t ntg = 0;
    int64_t *tg_start = nullptr;
    int64_t *tg_off = nullptr;
    double *tg_dense = nullptr;
    int64_t tg_bytes = 0;
    int64_t bytes = 0;
    // streaming create
    int64_t stream_rows = 0;
    int flags = 0;
    bool ready = false;
    hipStream_t stream = nullptr;
};

namespace hsym {

// geometry for a storage precision and block width (explicit rows/64 and log2 C
// when r64 > 0)
Geom geometry_for(int storage, int m, int64_t n, int r64, int lc);
// LDS bytes the SpMM needs at block width m on geometry g (160 KB available)
size_t spmm_lds_bytes(int storage, int m, const Geom &g);
void free_tiles(DeviceTiles *dt);

// device scratch (per call)
struct Scratch {
    void *p = nullptr;
    size_t bytes = 0;
    ~Scratch();
    void *get(size_t b);
};

// SpMM launch: X (n x m, ld ldx) -> Y; XIN/YOUT precision flags.  Y is
// cleared and receives every contribution by device-scope atomic adds.
enum { T_F64 = 0, T_F32 = 1 };
void spmm_launch(hsym_matrix *H, int m, const void *X, int xprec, int64_t ldx, void *Y, int yprec,
                 int64_t ldy, hipStream_t s);

// one matrix of a batched SpMM (fp64 blocks with leading dimension m)
struct SpmmJob {
    const int64_t *ptp;
    const int32_t *porder;
    const TileDesc *tiles;
    const unsigned char *blob;
    const void *diag;
    const double *X;
    int64_t ldx;
    double *Y;
    int64_t ldy;
    int64_t n;
    int64_t npanels;
    Geom g;
    int m;
};
SpmmJob spmm_job(hsym_matrix *H, int m, const double *X, double *Y);
// jobs: device table; host: the same table on the host (for the launch shape).
// Every matrix has the given storage; m is the same for all.
void spmm_batched(const SpmmJob *jobs, const SpmmJob *host, int count, int m, int storage, hipStream_t s);

// small parallel-for on host threads
void parallel_for(int64_t n, int64_t grain, const std::function<void(int64_t, int64_t)> &fn);
int host_threads();

}  // namespace hsym
