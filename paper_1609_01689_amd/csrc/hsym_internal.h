// Internal declarations shared by the host code and the HIP kernels of libhsym.
#pragma once

#include <hip/hip_runtime.h>
#include <cstdint>
#include <functional>
#include <string>
#include <vector>

#include "../../include/hsym.h"

namespace hsym {

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
// Section 4.2: independently addressable blocks, each holding its entries in
// coordinate form with 16-bit local row and column offsets).  Rows are cut
// into panels of R rows and columns into chunks of C columns (R a multiple of
// C).  The strictly-upper entries of one panel that fall into one chunk form a
// tile, stored row-major as index codes (local row << shift | local column)
// plus values: 32-bit codes with shift = 16, or, on request (HSYM_INDEX16),
// 16-bit codes with shift = log2 C when C is a power of two and R * C <= 2^16
// (Section 4.2: indices local to a block need only 16 bits).  A tile's entries are cut into G equal segments (the last one padded
// with zero values) stored interleaved: entry e of segment s sits at
// base + e*G + s, so G lane groups stream a tile with coalesced loads and equal
// work.  A tile is "own" when its chunk lies inside the panel (its transposed
// half lands in the panel's rows) and "external" otherwise; every external tile
// owns one partial-sum slot of C rows (used when the output is fp32).
// ---------------------------------------------------------------------------
struct TileDesc {
    int64_t base;          // first stored entry
    int32_t len;           // entries per segment (after padding)
    int32_t chunk;         // global chunk index g: columns [g*C, g*C+C)
    int32_t slot;          // partial slot, -1 for an own tile
    int32_t pad;
};

struct DeviceTiles {
    int R = 0, C = 0, G = 0;
    int64_t npanels = 0, nchunks = 0, ntiles = 0, nentries = 0, nslots = 0;
    int64_t nred_chunks = 0;
    int64_t *panel_tile_ptr = nullptr;
    int32_t *panel_order = nullptr;   // panel of workgroup b (see build.cpp: per-XCD, heaviest first)
    TileDesc *tiles = nullptr;
    void *idx = nullptr;          // uint16_t codes when idx_bytes == 2, else uint32_t
    int idx_bytes = 4;
    int idx_shift = 16;           // local row << idx_shift | local column
    void *vals = nullptr;
    int64_t *red_ptr = nullptr;
    int32_t *red_slot = nullptr;
    int32_t *red_chunks = nullptr;
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
    int geom_lr = 0, geom_lc = 0; // explicit log2 panel rows / chunk columns (0: automatic)
    std::vector<double> d_host;   // diagonal, fp64, host copy
    std::vector<double> colsum;   // absolute column sums (streaming create)
    // block-64 preconditioner: per 64-row chunk Q (64x64, row-major) and lambda
    double *pre_q = nullptr;
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

// geometry: (R, C) for a block width and storage precision
void geometry_for(int storage, int m, int64_t n, int lr, int lc, int *R, int *C, int *G);
int spmm_lanes_per_entry(int storage, int m);
size_t spmm_lds_bytes(int storage, int m, int R, int C);
void free_tiles(DeviceTiles *dt);

// device scratch (per call)
struct Scratch {
    void *p = nullptr;
    size_t bytes = 0;
    ~Scratch();
    void *get(size_t b);
};

// SpMM launch: X (n x m, ld ldx) -> Y; XIN/YOUT precision flags
enum { T_F64 = 0, T_F32 = 1 };
void spmm_launch(hsym_matrix *H, int m, const void *X, int xprec, int64_t ldx, void *Y, int yprec,
                 int64_t ldy, void *partials, hipStream_t s);
// partial-slot scratch of one SpMM call: fp32 outputs sum the transposed half
// of external tiles through slots and a reduction; fp64 outputs add it into Y
size_t spmm_partial_bytes(hsym_matrix *H, int m, int yprec = T_F64);

// one matrix of a batched SpMM (fp64 blocks with leading dimension m)
struct SpmmJob {
    const int64_t *ptp;
    const int32_t *porder;
    const TileDesc *tiles;
    const void *idx;
    int idx_bytes, idx_shift;
    const void *vals;
    const void *diag;
    const double *X;
    int64_t ldx;
    double *Y;
    int64_t ldy;
    double *partials;
    int64_t n;
    int R, C, G;
    int64_t npanels;
    int m;
    const int32_t *red_chunks;
    const int64_t *red_ptr;
    const int32_t *red_slot;
    int64_t nred;
};
SpmmJob spmm_job(hsym_matrix *H, int m, const double *X, double *Y, double *partials);
// jobs: device table; host: the same table on the host (for the launch shape).
// Every matrix has the given storage; m is the same for all.
void spmm_batched(const SpmmJob *jobs, const SpmmJob *host, int count, int m, int storage, hipStream_t s);

// small parallel-for on host threads
void parallel_for(int64_t n, int64_t grain, const std::function<void(int64_t, int64_t)> &fn);
int host_threads();

}  // namespace hsym
