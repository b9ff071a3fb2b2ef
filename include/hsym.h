/*
 * hsym.h - C ABI of the MI355X (gfx950) LOBPCG hot path.
 *
 * Problem (Section 3.1, eq. 6 and Algorithm 1 of Shao et al., "Accelerating
 * nuclear configuration interaction calculations through a preconditioned
 * block iterative eigensolver"): given a sparse symmetric H and a start block
 * X0 (n x k), find the k smallest eigenpairs H X = X Theta.  H is handed over
 * as one stored triangle (Section 4.1), block vectors are row-major
 * (Section 4.2), the block width exceeds the number of wanted pairs
 * (Section 3.1, end; Section 5.2 uses 50% extra vectors), and the solver takes
 * a preconditioner choice (Section 3.2) and a start block (Section 3.3).
 *
 * Conventions for every call:
 *   - every function returns an int status (enum hsym_status); no exception or
 *     abort crosses the ABI; hsym_last_error() gives a message for the
 *     calling thread;
 *   - "device" pointers are HIP device allocations on the current device,
 *     "host" pointers are ordinary host memory;
 *   - a stream argument is a hipStream_t passed as void* (NULL = the null
 *     stream).  Calls marked "async" only enqueue work on that stream;
 *   - n x m blocks are row-major with a leading dimension (elements between
 *     consecutive rows) >= m;
 *   - eigenvalues are ascending; each returned eigenvector is scaled to unit
 *     2-norm with its largest-magnitude entry positive.
 *
 * The library allocates device memory with hipMalloc (matrix, per-call
 * scratch, solver work blocks) and frees it before returning, except what a
 * handle owns until it is destroyed.
 */
#ifndef HSYM_H
#define HSYM_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

enum hsym_status {
    HSYM_OK = 0,
    HSYM_NOT_CONVERGED = 1,      /* results written, tolerance not met at maxit        */
    HSYM_E_INVALID_ARG = -1,     /* bad sizes, malformed CSR, NaN/Inf values, NULL ptr */
    HSYM_E_OUT_OF_MEMORY = -2,   /* device or host allocation failed                   */
    HSYM_E_DEVICE = -3,          /* a HIP runtime call failed                          */
    HSYM_E_BREAKDOWN = -4,       /* block lost rank and could not be repaired          */
    HSYM_E_NUMERIC = -5,         /* NaN/Inf appeared during a solve                    */
    HSYM_E_UNSUPPORTED = -6      /* block width / option combination not built         */
};

enum hsym_prec { HSYM_FP64 = 0, HSYM_FP32 = 1 };

/* Preconditioners of Section 3.2 (eq. 11): none, the diagonal of H
 * ("the extreme case" of a block-diagonal approximation), the dense 64x64
 * diagonal blocks of H solved directly (eigenvector factors stored in the
 * handle's storage precision, applied with fp64 products), or the paper's own
 * choice (end of Section 3.2, Section 4.3): the diagonal tiles of the
 * many-body groups (hsym_attach_group_tiles), each shifted system solved by
 * lobpcg_opts.fom_iters steps of the full orthogonalization method per
 * right-hand side. */
enum hsym_precond { HSYM_PRECOND_NONE = 0, HSYM_PRECOND_JACOBI = 1, HSYM_PRECOND_BLOCK64 = 2,
                     HSYM_PRECOND_FOM = 3 };

/* hsym_create flags */
#define HSYM_HOST_PTRS     0x0   /* rowptr/colind/values are host memory (default)   */
#define HSYM_DEVICE_PTRS   0x1   /* hsym_create only: rowptr/colind/values are device
                                    memory (copied to the host, where the tiles are
                                    built; the copy is synchronous)                 */
#define HSYM_BUILD_BLOCK64 0x2   /* also build the 64x64 block preconditioner factors */
/* Accepted for compatibility: tile-local index codes (local row and column
 * packed together, Section 4.2: indices local to a block need only 16 bits)
 * are 16-bit whenever R * C <= 2^16, which the default geometries satisfy at
 * block widths of 4 and more; hsym_info reports the width in use. */
#define HSYM_INDEX16       0x4
/* Tile geometry hint: the block width (1..16) the panel sizes are chosen for,
 * in bits 8..15 (0 = 16).  The tile streams are laid out for the lane groups
 * of that width; other widths whose LDS footprint fits the geometry can be
 * used with the handle, at lower efficiency. */
#define HSYM_GEOM_M(m) (((m) & 0xff) << 8)
/* Explicit panel geometry: R = 64 * r64 panel rows (1 <= r64 <= 255) and
 * C = 2^lc chunk columns (3 <= lc <= 12, C dividing R), in bits 16..27
 * (0 = chosen from the block width hint, n and the first rows given: the
 * tallest panels whose pieces fit the LDS with room to spare, or shorter ones
 * whose larger pieces keep the tiles of those rows whole, whichever the
 * library's cost model of the SpMM prefers).  hsym_create fails with
 * HSYM_E_INVALID_ARG when C does not divide R or the geometry does not fit
 * the LDS at the hinted block width; spmm_sym fails with HSYM_E_UNSUPPORTED
 * when it does not fit at the requested width.  hsym_autotune_geometry
 * returns such flags. */
#define HSYM_GEOM_PANEL(r64, lc) ((((r64) & 0xff) << 16) | (((lc) & 0xf) << 24))

typedef struct hsym_matrix *hsym_t;
typedef struct lobpcg_ctx *lobpcg_ctx_t;

typedef struct {
    int64_t n;
    int64_t nnz_stored;         /* stored entries incl. the diagonal                  */
    double norm1;               /* ||H||_1 = max absolute row sum of the full matrix  */
    int storage;                /* enum hsym_prec of the stored values                */
    int panel_rows;             /* rows per panel of the tile format                  */
    int chunk_cols;             /* columns per tile chunk                             */
    int64_t npanels;
    int64_t ntiles;
    int64_t nslots;             /* tiles whose transposed half leaves the panel       */
    int64_t padded_entries;     /* stored off-diagonal entries after segment padding  */
    int64_t device_bytes;       /* device memory held by the handle                   */
    int has_block64;
    int index_bytes;            /* bytes of one tile-local index code: 2 or 4         */
    int64_t npieces;            /* tiles after cutting them into pieces               */
    int piece_entries;          /* entries per piece at most                          */
} hsym_info_t;

/*
 * Build a device-resident handle from the upper triangle of H in CSR form
 * (Section 4.1 stores one triangle; this ABI takes the upper one, which is
 * the transpose of the paper's lower triangle).
 *   rowptr  host (or device, see flags) int64[n+1], rowptr[0]=0,
 *           non-decreasing, rowptr[n]=nnz;
 *   colind  int32[nnz], row i holds columns >= i, strictly increasing;
 *           a missing diagonal entry means H_ii = 0;
 *   values  fp64 (values_prec=HSYM_FP64) or fp32 (HSYM_FP32), finite;
 *   storage precision of the device copy: HSYM_FP64 (plain form) or HSYM_FP32
 *           (mixed form, Section 4.4 footnote 5: H stored and multiplied in
 *           single precision); fp64 input is rounded to nearest once;
 *   flags   HSYM_HOST_PTRS or HSYM_DEVICE_PTRS, optional HSYM_BUILD_BLOCK64,
 *           HSYM_INDEX16, HSYM_GEOM_M, HSYM_GEOM_PANEL.
 * The call copies: the caller may free its arrays on return.  Synchronous.
 * Errors: HSYM_E_INVALID_ARG for any CSR violation listed above or n < 1 or
 * n >= 2^31; HSYM_E_OUT_OF_MEMORY; HSYM_E_DEVICE.  *H is NULL on error.
 */
int hsym_create(hsym_t *H, int64_t n, const int64_t *rowptr, const int32_t *colind,
                const void *values, int values_prec, int storage, int flags, void *stream);

/*
 * Streaming form of hsym_create for inputs too large to hold whole on the
 * host: begin, then append consecutive row slabs starting at row 0 (each slab
 * in the same CSR convention, rowptr_local relative to the slab, int64[nrows+1]),
 * then finish.  Slabs need not align with anything.  The handle is usable only
 * after finish returns HSYM_OK; on any error the handle is destroyed and *H
 * (begin) or the passed handle (append/finish) must not be used again.
 */
int hsym_create_begin(hsym_t *H, int64_t n, int storage, int flags, void *stream);
int hsym_create_append(hsym_t H, int64_t nrows, const int64_t *rowptr_local,
                       const int32_t *colind, const void *values, int values_prec);
int hsym_create_finish(hsym_t H);

/*
 * Diagonal group tiles for HSYM_PRECOND_FOM (Section 4.3: a separate matrix
 * of the diagonal tiles, set up next to H).  group_start (host
 * int64[ngroups+1]) holds ascending group boundaries, group_start[0] = 0 and
 * group_start[ngroups] = n; groups longer than 64 rows are cut into 64-row
 * pieces.  rowptr/colind/values are the same upper CSR as hsym_create's (the
 * entries inside each group's diagonal tile are kept, densely, in fp64).
 * Replaces tiles attached before.  Synchronous.  Errors: HSYM_E_INVALID_ARG
 * (NULL pointers, bad boundaries, malformed CSR), HSYM_E_OUT_OF_MEMORY,
 * HSYM_E_DEVICE.
 */
int hsym_attach_group_tiles(hsym_t H, int64_t ngroups, const int64_t *group_start, const int64_t *rowptr,
                            const int32_t *colind, const void *values, int values_prec);

int hsym_destroy(hsym_t H);
int hsym_info(hsym_t H, hsym_info_t *out);

/*
 * Y = H X (async).  X, Y device fp64 n x m with leading dimensions ldx, ldy;
 * m in {1..16}.  H is applied from its stored triangle as D X + U X + U^T X
 * (U strictly upper, D the diagonal; Section 4.1: each stored block is used
 * once as itself and once transposed).  With fp32 storage the values are
 * held in fp32 and X is taken as it is (staged in fp64); every product is
 * formed and summed in fp64 and Y is returned in fp64.  The transposed half is summed with workgroup-local
 * atomics and added into Y with device-scope atomics, so repeated calls agree
 * to rounding, not bitwise.
 * X and Y must not overlap.  Errors: HSYM_E_INVALID_ARG, HSYM_E_DEVICE.
 */
int spmm_sym(hsym_t H, int m, const double *X, int64_t ldx, double *Y, int64_t ldy,
             void *stream);

/* Same product on fp32 blocks (fp32 storage only; m in {1..16}). */
int spmm_sym_f32(hsym_t H, int m, const float *X, int64_t ldx, float *Y, int64_t ldy,
                 void *stream);

/*
 * Tile-shape autotuner (request loop, "autotuned tile shape").  Takes the
 * same host CSR as hsym_create and a block width m.  It builds a row sample of
 * H (sample_rows rows around the middle, <= 0 for min(n, 262144); entries whose
 * column leaves the sample are dropped) once per candidate panel geometry
 * (R = 256..448 rows in steps of 64, 512..960 in steps of 128, 1024..2048 in
 * steps of 256; C = 64 or 128 columns dividing R; those whose LDS footprint at
 * width m fits 160 KB), times spmm_sym on it (3 warm-up calls, then 5 calls
 * between HIP events on a private stream) and returns in *out_flags the
 * HSYM_GEOM_M(m) | HSYM_GEOM_PANEL(..) flags of the fastest, to be or-ed into
 * hsym_create's flags.  table (host, cap entries, may be NULL) receives every
 * candidate tried (ms < 0 when it could not be built or run); *ntried (may be
 * NULL) their number.  Synchronous; allocates and frees device memory.
 * Errors: HSYM_E_INVALID_ARG (NULL pointers, m outside [1, 16], malformed
 * rowptr or lower entries), HSYM_E_UNSUPPORTED (no candidate ran),
 * HSYM_E_OUT_OF_MEMORY, HSYM_E_DEVICE.
 */
typedef struct {
    int panel_rows;
    int chunk_cols;
    double ms;                  /* mean spmm_sym time on the sample, < 0: failed */
} hsym_tune_entry;

int hsym_autotune_geometry(int64_t n, const int64_t *rowptr, const int32_t *colind, const void *values,
                           int values_prec, int storage, int m, int64_t sample_rows, int *out_flags,
                           hsym_tune_entry *table, int cap, int *ntried);

typedef struct {
    int maxit;              /* default 1000                                          */
    uint64_t seed;          /* Gaussian start block / rank-repair columns            */
    int check_every;        /* host convergence check every k iterations (>=1)       */
    int no_precond_iters;   /* Section 4.3 rule 1, default 3                         */
    double near;            /* Section 4.3 rules 2-4 threshold, default 0.1          */
    double guard;           /* shifted denominators kept >= guard*||H||_1, 1e-4       */
    int keep_history;       /* record per-iteration residual norms                   */
    int graph;              /* 1: record the launches of each steady-state iteration
                               phase once in a HIP graph and replay it (fewer launch
                               calls for small n; the SpMM is then not timed in
                               lobpcg_report.phase_ms); default 0. While a context
                               records (its first steady-state iterations) the HIP
                               runtime refuses stream synchronisation in other
                               threads of the process: use it where one thread
                               creates and steps the contexts (hsym_serve, whose
                               loader thread builds requests meanwhile, leaves it
                               off).  Needs a non-null stream: on the null stream
                               the solve runs without graphs                    */
    int fom_iters;          /* FOM steps of HSYM_PRECOND_FOM, 1..4; default 3 (the
                               paper performs up to three)                       */
    int timers;             /* 1: time every phase of the iteration with events on
                               the solve stream (lobpcg_report.phase_ms[1..7], the
                               split of Section 5.2, Fig. 7); default 0.  Phases
                               replayed from a graph are not timed              */
} lobpcg_opts;

#define HSYM_MAX_BLOCK 16
#define HSYM_MAX_HISTORY 4096

typedef struct {
    int iters;                        /* LOBPCG iterations performed                 */
    int converged;
    int spmm_calls;                   /* block SpMMs, start block included           */
    int p_dropped;                    /* iterations where P lost rank and was dropped */
    int w_replaced;                   /* W columns replaced by random columns         */
    double theta[HSYM_MAX_BLOCK];     /* all m Ritz values at exit                    */
    double resnorm[HSYM_MAX_BLOCK];   /* ||r_j|| / ||H||_1 at exit, all m columns     */
    double seconds;                   /* wall time of the solve                      */
    double phase_ms[8];               /* [0]: device time of the block SpMMs launched on
                                         the context's own stream (events; SpMMs of
                                         batched rounds are not timed).  With
                                         opts.timers, device time of [1] the
                                         preconditioner (with the Jacobi apply, the
                                         first Gram of the orthogonalisation, fused
                                         into it), [2] the Cholesky-QR of W, [3] the
                                         Gram products of Rayleigh-Ritz, [4] the
                                         Rayleigh-Ritz eigensolve, [5] the update of
                                         X, P, AX, AP with the next residuals and
                                         norms, [7] the start block, repairs and
                                         status copies; [6] is host wall time spent
                                         waiting for the stream.  Otherwise 0      */
    int history_len;
    double history[HSYM_MAX_HISTORY]; /* max_{j<=nev} rho_j per iteration           */
    int rr_rounds_max;                /* most multisection rounds any Rayleigh-Ritz eigenvalue search took */
    int batched_iters;                /* iterations run in batched rounds (lobpcg_ctx_step) */
} lobpcg_report;

void lobpcg_opts_default(lobpcg_opts *o);

/*
 * LOBPCG (Algorithm 1) for the nev smallest eigenpairs with block width
 * block_width (nev <= block_width <= 16, 3*block_width <= n).  tol > 0 is the
 * relative residual ||H x_j - theta_j x_j|| / (||H||_1 ||x_j||) that each of
 * the first nev pairs must reach.  X0: device n x block_width fp64 (ld =
 * block_width) or NULL for a seeded Gaussian block.  evals: host[nev].
 * evecs: device n x nev fp64 (ld = nev) or NULL.  rep, opts may be NULL.
 * Block vectors, Gram products, Cholesky-QR, the Rayleigh-Ritz eigensolve and
 * the convergence test are fp64 for both storage precisions.
 * Host-synchronous: returns after convergence or maxit (HSYM_NOT_CONVERGED,
 * results written).
 */
int lobpcg_solve(hsym_t H, int nev, int block_width, double tol, const double *X0,
                 int precond, const lobpcg_opts *opts, double *evals, double *evecs,
                 lobpcg_report *rep, void *stream);

/*
 * Multi-level start block (Section 3.3.1, eq. 12, applied recursively as the
 * section's closing remark describes).  Takes the host CSR of hsym_create and
 * level (host int32[n]): the level of every row, for CI matrices the
 * excitation quanta of its configuration.  caps (host int32[ncaps], strictly
 * ascending, 1 <= ncaps <= 16) lists the smaller configuration spaces.  For
 * each cap in turn, the library:
 *   1. takes the principal submatrix H11 on the rows with level <= cap
 *      (order kept);
 *   2. solves for its m lowest eigenpairs with lobpcg_solve (block width m,
 *      tol, precond, opts, all m columns gating convergence);
 *   3. starts that solve from a seeded Gaussian block for the first cap, and
 *      from the previous cap's eigenvectors padded with zeros (eq. 12) for
 *      the others.
 * X0 (device n x m, row-major ld m, caller-owned) receives the last cap's
 * eigenvectors padded with zeros: the start block of the full solve.
 * iters (host int[ncaps], may be NULL) receives each sub-solve's iteration
 * count; a sub-solve that stops at maxit is not an error.  Synchronous.
 * Errors: HSYM_E_INVALID_ARG (NULL pointers, malformed CSR, caps not
 * ascending, a cap keeping fewer than 3m rows), and those of hsym_create and
 * lobpcg_solve.
 */
int lobpcg_guess_multilevel(int64_t n, const int64_t *rowptr, const int32_t *colind, const void *values,
                            int values_prec, const int32_t *level, int ncaps, const int32_t *caps,
                            int storage, int m, double tol, int precond, const lobpcg_opts *opts,
                            double *X0, int *iters, void *stream);

typedef struct {
    int maxit;        /* default 2000 (also capped by n)                             */
    uint64_t seed;    /* Gaussian start vector when v0 is NULL                       */
} lanczos_opts;

typedef struct {
    int iters;
    int converged;
    double resnorm[HSYM_MAX_BLOCK];  /* Ritz residual / ||H||_1 of the nev pairs     */
    double seconds;
    double spmv_ms;
    double orth_ms;
} lanczos_report;

/*
 * Single-vector Lanczos with full re-orthogonalisation (the baseline the paper
 * replaces; Section 3, opening) with convergence checks on the schedule of
 * Section 5.2 footnote 7.  nev <= 16.  v0: device fp64[n] or NULL.  evals host[nev];
 * evecs device n x nev or NULL.  Host-synchronous.
 */
int lanczos_solve(hsym_t H, int nev, double tol, const double *v0, const lanczos_opts *opts,
                  double *evals, double *evecs, lanczos_report *rep, void *stream);

/*
 * Context/step form of lobpcg_solve for request loops: a context owns its
 * block vectors on the device and runs on its own stream (created when
 * stream is NULL); lobpcg_ctx_step advances `count` contexts by up to
 * `iters` iterations each, issuing each phase for all of them before waiting
 * on any, so that their kernels overlap on the device.  A context's
 * arithmetic does not depend on which other contexts are stepped with it.
 */
int lobpcg_ctx_create(lobpcg_ctx_t *ctx, hsym_t H, int nev, int block_width, double tol,
                      const double *X0, int precond, const lobpcg_opts *opts, void *stream);
int lobpcg_ctx_step(lobpcg_ctx_t *ctxs, int count, int iters);
int lobpcg_ctx_status(lobpcg_ctx_t ctx, int *done, double *evals, lobpcg_report *rep);
int lobpcg_ctx_evecs(lobpcg_ctx_t ctx, double *evecs);
int64_t lobpcg_ctx_device_bytes(lobpcg_ctx_t ctx);
int lobpcg_ctx_destroy(lobpcg_ctx_t ctx);

/*
 * Request loop (serving layer around the solver; the paper runs one solve per
 * job).  Continuous batching at iteration granularity: requests are admitted
 * in arrival order while their estimated device memory fits budget_bytes and
 * fewer than max_active are in flight; a loader thread builds each request's
 * handle and context; every scheduling round advances all active requests by
 * iters_per_round iterations (lobpcg_ctx_step), so short requests finish
 * while long ones run.  A request whose estimate exceeds the budget finishes
 * at admission with HSYM_E_OUT_OF_MEMORY.
 *
 * hsym_request inputs: host upper CSR as for hsym_create (must stay valid
 * until hsym_serve returns), storage precision, nev <= block_width <= 16,
 * tol, precond, seed of the Gaussian start block, arrival_s >= 0 (seconds
 * from the start of the call).  Outputs: status (HSYM_OK, HSYM_NOT_CONVERGED
 * or an error), iters, evals[0..nev), admit_s and finish_s (same clock),
 * device_bytes held while active, error (message when status < 0).
 * Latency = finish_s - arrival_s.
 */
typedef struct {
    int64_t n;
    const int64_t *rowptr;
    const int32_t *colind;
    const void *values;
    int values_prec;
    int storage;
    int nev;
    int block_width;
    int precond;
    double tol;
    uint64_t seed;
    double arrival_s;
    /* outputs */
    int status;
    int iters;
    double evals[HSYM_MAX_BLOCK];
    double admit_s;
    double finish_s;
    int64_t device_bytes;
    char error[128];        /* message of a failed request, "" otherwise */
} hsym_request;

typedef struct {
    int64_t budget_bytes;   /* device memory for requests in flight; default 200 GiB */
    int max_active;         /* requests in flight at most; default 64                */
    int iters_per_round;    /* iterations per active request per round; default 1   */
    int maxit;              /* per-request iteration cap; default 1000               */
    int autotune;           /* 1: the first request of each size class (power of two
                               of n, block width, storage) runs
                               hsym_autotune_geometry on its matrix, and the class
                               keeps that panel geometry; default 0                 */
    int loaders;            /* threads that build admitted requests (tile build and
                               context set-up) in parallel; 1..16, default 2      */
} hsym_serve_opts;

typedef struct {
    double wall_s;                  /* first arrival to last finish              */
    int rounds;                     /* scheduling rounds that stepped requests   */
    int tuned_classes;              /* size classes the autotuner ran for        */
    int max_active_seen;
    int64_t peak_reserved_bytes;    /* largest sum of admitted estimates         */
} hsym_serve_report;

void hsym_serve_opts_default(hsym_serve_opts *o);
/* Runs the whole trace on the current device; returns when every request has
 * finished.  Errors of single requests are reported in their status. */
int hsym_serve(hsym_request *reqs, int count, const hsym_serve_opts *opts, hsym_serve_report *rep);
/* The same scheduler on a virtual clock, without a device: request r takes
 * iters[r] iterations of iter_s[r] seconds, holds bytes[r], and loads take
 * load_s each on one loader; a round costs the longest iteration among the
 * requests it steps.  For checking admission and accounting on the host. */
int hsym_serve_sim(hsym_request *reqs, int count, const hsym_serve_opts *opts, const int *iters,
                   const double *iter_s, const int64_t *bytes, double load_s, hsym_serve_report *rep);

/* Message of the last error on the calling thread ("" if none). */
const char *hsym_last_error(void);

#ifdef __cplusplus
}
#endif
#endif
