// LOBPCG driver (Algorithm 1 with the preconditioning of Section 3.2 and the
// rules of Section 4.3).  Host code enqueues the kernels on one stream and
// reads back one small status block per iteration (residual norms, Ritz
// values) to run the convergence test and the shift rules.
//
// Basis handling (Algorithm 1, step 7): W is orthonormalised against [X P]
// and itself by Cholesky-QR passes driven by Gram matrices.  The Rayleigh-
// Ritz step then measures the basis: one pass over S = [X W P] and AS forms
// both S^T S and S^T A S, and the small kernel orthonormalises S in
// coefficient space (Cholesky of S^T S in the order X, W, P: Gram-Schmidt of
// P against X and W, and of W against X), dropping P for the iteration when
// one of its pivots is small.  After Rayleigh-Ritz the new P is built in
// coefficient space from the W,P-components of the new X made orthogonal to
// it, so span{X_new, P_new} equals span{X_new, (I - X X^T) X_new} of step 10
// and no full-size pass is needed to orthogonalise P.  The rounding of X and
// P away from orthonormality does not accumulate: every iteration's
// Rayleigh-Ritz takes the basis as measured.
#include <atomic>
#include <memory>
#include <chrono>
#include <cmath>
#include <cstring>

#include <rocprofiler-sdk-roctx/roctx.h>

#include "dense.h"

namespace hsym {

struct Status {
    double norms[HSYM_MAX_BLOCK];     // squared column norms of R
    double theta[HSYM_MAX_BLOCK];
    int flags[8];                     // 0: orth deficiency mask, 1: rr bisection rounds
};

// Orthonormalise V (n x m) against the kb orthonormal blocks B and itself
// (Cholesky-QR with column scaling, then a second Cholesky-QR pass).  Columns
// that turn out numerically inside span(B, V) are replaced with seeded
// Gaussian columns and the procedure is repeated.  Returns the number of
// replaced columns.  Synchronises the stream once per attempt.
int orthonormalize_block(int64_t n, int m, double *V, const double *const *B, int kb, uint64_t seed,
                         OrthWork &w, hipStream_t s) {
    int replaced = 0;
    for (int attempt = 0;; attempt++) {
        HIPCHK(hipMemsetAsync(w.flag_d, 0, sizeof(int), s));
        GramArgs g{};
        for (int i = 0; i < kb; i++) g.a[i] = B[i];
        g.a[kb] = V; g.b[0] = V; g.na = kb + 1; g.nb = 1; g.m = m; g.n = n;
        gram(g, w.gbuf, w.gram_scr, s);
        OrthArgs oa{w.gbuf, w.coef, w.flag_d, kb, m, 0};
        small_orth(&oa, 1, s);
        LincombArgs l{};
        for (int i = 0; i < kb; i++) l.in[i] = B[i];
        l.in[kb] = V; l.out[0] = V; l.coef = w.coef; l.ldc = m; l.nin = kb + 1; l.nout = 1; l.nsets = 1;
        l.m = m; l.n = n;
        lincomb(l, s);
        gram(g, w.gbuf, w.gram_scr, s);
        oa.stage = 1;
        small_orth(&oa, 1, s);
        HIPCHK(hipMemcpyAsync(w.flag_h, w.flag_d, sizeof(int), hipMemcpyDeviceToHost, s));
        HIPCHK(hipStreamSynchronize(s));
        int flag = *w.flag_h;
        if (flag) {
            if (attempt >= 3) fail(HSYM_E_BREAKDOWN, "block stays rank deficient after 3 random repairs");
            int mask = flag & ((1 << m) - 1);
            replaced += __builtin_popcount((unsigned)mask);
            gauss_fill(V, n, m, m, seed + (uint64_t)attempt, 10, mask, s);
            continue;
        }
        lincomb(l, s);
        GramArgs g2{};
        g2.a[0] = V; g2.b[0] = V; g2.na = g2.nb = 1; g2.m = m; g2.n = n;
        gram(g2, w.gbuf, w.gram_scr, s);
        OrthArgs o2{w.gbuf, w.coef, w.flag_d, 0, m, 2};
        small_orth(&o2, 1, s);
        LincombArgs l2{};
        l2.in[0] = V; l2.out[0] = V; l2.coef = w.coef; l2.ldc = m; l2.nin = 1; l2.nout = 1; l2.nsets = 1;
        l2.m = m; l2.n = n;
        lincomb(l2, s);
        return replaced;
    }
}

struct Lobpcg {
    hsym_matrix *H = nullptr;
    hipStream_t s = nullptr;
    int64_t n = 0;
    int m = 0, nev = 0, precond = HSYM_PRECOND_NONE;
    double tol = 0.0;
    lobpcg_opts o{};
    // device blocks
    double *X = nullptr, *AX = nullptr, *W = nullptr, *AW = nullptr, *P = nullptr, *AP = nullptr;
    double *gram_scr = nullptr, *gbuf = nullptr, *coef = nullptr, *rrcoef = nullptr;
    double *mu = nullptr, *norm_part = nullptr;
    Status *st_d = nullptr;
    Status *st_h = nullptr;      // pinned
    double *mu_h = nullptr;      // pinned
    int64_t bytes = 0;
    // iteration state
    int it = 0;
    bool have_p = false;
    bool done = false;
    int status = HSYM_NOT_CONVERGED;
    lobpcg_report rep{};
    std::chrono::steady_clock::time_point t0;
    std::vector<void *> allocs;
    hipEvent_t ev_spmm[2] = {nullptr, nullptr};   // brackets the latest SpMM on s
    bool spmm_pending = false;
    // opts.timers: an event opens each phase's stretch of the stream; the
    // stretches are added to phase_ms[] at the next synchronisation
    static constexpr int NMARK = 24;
    hipEvent_t ev_mark[NMARK] = {};
    int mark_phase[NMARK] = {};
    int nmark = 0;
    bool range_open = false;
    // graphs of the steady-state iteration (opts.graph): phase A without and
    // with the preconditioner, phase B
    hipGraphExec_t graph_a[2] = {nullptr, nullptr}, graph_b = nullptr;
    bool capturing = false;
    uint64_t serial = 0;          // unique per context (batch tables are keyed by it)

    template <class T>
    T *dalloc(size_t count) {
        void *p = nullptr;
        size_t b = std::max<size_t>(count * sizeof(T), 256);
        if (hipMalloc(&p, b) != hipSuccess) {
            (void)hipGetLastError();
            fail(HSYM_E_OUT_OF_MEMORY, "solver allocation of " + std::to_string(b) + " bytes");
        }
        allocs.push_back(p);
        bytes += (int64_t)b;
        return (T *)p;
    }

    ~Lobpcg() {
        for (hipGraphExec_t ge : {graph_a[0], graph_a[1], graph_b})
            if (ge) (void)hipGraphExecDestroy(ge);
        for (hipEvent_t e : ev_spmm)
            if (e) (void)hipEventDestroy(e);
        for (hipEvent_t e : ev_mark)
            if (e) (void)hipEventDestroy(e);
        if (range_open) roctxRangePop();
        for (void *p : allocs) (void)hipFree(p);
        if (st_h) (void)hipHostFree(st_h);
        if (mu_h) (void)hipHostFree(mu_h);
    }

    void setup(hsym_matrix *H_, int nev_, int m_, double tol_, const double *X0, int pc, const lobpcg_opts *opts,
               hipStream_t s_) {
        static std::atomic<uint64_t> next_serial{1};
        serial = next_serial++;
        H = H_; s = s_; n = H->n; m = m_; nev = nev_; tol = tol_; precond = pc;
        lobpcg_opts_default(&o);
        if (opts) o = *opts;
        if (o.maxit < 1) o.maxit = 1000;
        if (o.check_every < 1) o.check_every = 1;
        if (pc == HSYM_PRECOND_FOM && !H->tg_dense)
            fail(HSYM_E_INVALID_ARG, "FOM preconditioner needs hsym_attach_group_tiles on the handle");
        if (o.fom_iters < 1 || o.fom_iters > 4) fail(HSYM_E_INVALID_ARG, "fom_iters must be in [1, 4]");
        if (pc == HSYM_PRECOND_BLOCK64 && !H->pre_q)
            fail(HSYM_E_INVALID_ARG, "block64 preconditioner needs a handle created with HSYM_BUILD_BLOCK64");
        size_t nm = (size_t)n * m;
        X = dalloc<double>(nm); AX = dalloc<double>(nm); W = dalloc<double>(nm);
        AW = dalloc<double>(nm); P = dalloc<double>(nm); AP = dalloc<double>(nm);
        gram_scr = (double *)dalloc<char>(std::max(gram_scratch_bytes(n, 3 * m, 6 * m),
                                                   sign_fix_scratch_bytes(n, m)));
        gbuf = dalloc<double>(48 * 96);
        coef = dalloc<double>(48 * 32);
        rrcoef = dalloc<double>(48 * 32);
        mu = dalloc<double>(HSYM_MAX_BLOCK);
        norm_part = dalloc<double>((size_t)lincomb_norm_parts(n) * m);
        st_d = dalloc<Status>(1);
        HIPCHK(hipHostMalloc((void **)&st_h, sizeof(Status), hipHostMallocDefault));
        HIPCHK(hipHostMalloc((void **)&mu_h, sizeof(double) * HSYM_MAX_BLOCK, hipHostMallocDefault));
        memset(&rep, 0, sizeof(rep));
        for (hipEvent_t &e : ev_spmm) HIPCHK(hipEventCreate(&e));
        if (o.timers)
            for (hipEvent_t &e : ev_mark) HIPCHK(hipEventCreate(&e));
        t0 = std::chrono::steady_clock::now();
        mark(7);
        // start block: X0 or a seeded Gaussian block
        if (X0) HIPCHK(hipMemcpyAsync(X, X0, sizeof(double) * nm, hipMemcpyDeviceToDevice, s));
        else gauss_fill(X, n, m, m, o.seed, 8, -1, s);
        // step 1: orthonormalise X0, Rayleigh quotient, Ritz vectors of span(X0)
        OrthWork ow{gbuf, coef, gram_scr, &st_d->flags[0], &st_h->flags[0]};
        rep.w_replaced += orthonormalize_block(n, m, X, nullptr, 0, o.seed * 1000003ULL + 5ULL, ow, s);
        mark(0);
        spmm(X, AX);
        rep.spmm_calls++;
        GramArgs g{};
        g.a[0] = X; g.b[0] = X; g.b[1] = AX; g.na = 1; g.nb = 2; g.m = m; g.n = n; g.sym = 1;
        mark(3);
        gram(g, gbuf, gram_scr, s);
        mark(4);
        rayleigh_ritz(1);
        mark(5);
        LincombArgs u{};
        u.in[0] = X; u.in[3] = AX; u.out[0] = X; u.out[2] = AX;
        u.coef = rrcoef; u.ldc = 2 * m; u.nin = 1; u.nout = 1; u.nsets = 2; u.m = m; u.n = n;
        u.theta = st_d->theta; u.res = W; u.norm_part = norm_part;
        lincomb(u, s);
        colsum_final(norm_part, lincomb_norm_parts(n), m, st_d->norms, s);
        have_p = false;
        it = 0;
    }

    // the block SpMM, bracketed by events whose elapsed time is added to
    // phase_ms[0] at the next synchronisation
    void spmm(const double *V, double *AV) {
        if (!capturing) HIPCHK(hipEventRecord(ev_spmm[0], s));
        spmm_launch(H, m, V, T_F64, m, AV, T_F64, m, s);
        if (!capturing) {
            HIPCHK(hipEventRecord(ev_spmm[1], s));
            spmm_pending = true;
        }
    }

    // graphs need a stream that can be captured: the null stream cannot, so
    // a solve on it runs eagerly
    bool use_graph() const { return o.graph && have_p && s != nullptr; }

    // Run f's launches on s; with opts.graph, record them once into ge (a
    // graph of the stream's work) and replay ge from then on.  The launches
    // of a steady-state phase take the same arguments every iteration: the
    // block pointers are fixed and the values that change (shifts, flags,
    // Ritz values) travel through device or pinned memory.
    template <class F>
    void graphed(hipGraphExec_t &ge, F &&f) {
        if (!ge) {
            // The recorded phase makes no allocating or synchronising call.
            // While a capture is open the runtime also refuses stream
            // synchronisation in other threads of the process.
            HIPCHK(hipStreamBeginCapture(s, hipStreamCaptureModeRelaxed));
            capturing = true;
            hipGraph_t gr = nullptr;
            try {
                f();
            } catch (...) {
                capturing = false;
                (void)hipStreamEndCapture(s, &gr);
                if (gr) (void)hipGraphDestroy(gr);
                throw;
            }
            capturing = false;
            HIPCHK(hipStreamEndCapture(s, &gr));
            const hipError_t e = hipGraphInstantiate(&ge, gr, nullptr, nullptr, 0);
            (void)hipGraphDestroy(gr);
            HIPCHK(e);
        }
        HIPCHK(hipGraphLaunch(ge, s));
    }

    // gbuf holds [S^T S | S^T A S] for the nblk blocks of S
    void rayleigh_ritz(int nblk) {
        RRArgs r{};
        r.gram = gbuf; r.coef = rrcoef; r.theta = st_d->theta; r.evals_all = nullptr;   // only the m lowest are needed
        r.flag = &st_d->flags[1]; r.nblk = nblk; r.m = m;
        small_rr(&r, 1, s);
    }

    // ---- phases of one iteration (A: up to the rank flag; B: the rest) ----
    // post_status: enqueue the copy of the status block (norms, Ritz values)
    void post_status() { HIPCHK(hipMemcpyAsync(st_h, st_d, sizeof(Status), hipMemcpyDeviceToHost, s)); }

    // Section 4.3 rules 1-4 on the host; returns false when W = R
    bool shifts(const double *rho, const double *rnorm, const double *theta) {
        if (precond == HSYM_PRECOND_NONE || it <= o.no_precond_iters || rho[0] > o.near) return false;
        bool far = false;
        for (int j = 0; j < m; j++) {
            if (!far && rho[j] > o.near) far = true;
            mu_h[j] = far ? mu_h[j - 1] : theta[j] - 2.0 * rnorm[j];
        }
        return true;
    }

    // evaluate (status copy complete): convergence test of step 5; true when done
    double rho_[HSYM_MAX_BLOCK], rnorm_[HSYM_MAX_BLOCK];
    int evaluated = -1;
    bool evaluate() {
        if (done) return true;
        if (evaluated == it) return false;
        evaluated = it;
        const double normH = H->norm1;
        double mx = 0.0;
        for (int j = 0; j < m; j++) {
            double v = st_h->norms[j];
            if (!std::isfinite(v) || !std::isfinite(st_h->theta[j])) fail(HSYM_E_NUMERIC, "NaN/Inf in residual");
            rnorm_[j] = std::sqrt(v);
            rho_[j] = rnorm_[j] / normH;
            if (j < nev) mx = std::max(mx, rho_[j]);
        }
        if (st_h->flags[1] < 0) fail(HSYM_E_NUMERIC, "Rayleigh-Ritz eigensolver broke down (non-finite inverse iterate)");
        rep.rr_rounds_max = std::max(rep.rr_rounds_max, st_h->flags[1] - 1);
        rep.p_dropped += st_h->flags[2];
        if (o.keep_history && rep.history_len < HSYM_MAX_HISTORY) rep.history[rep.history_len++] = mx;
        for (int j = 0; j < m; j++) { rep.theta[j] = st_h->theta[j]; rep.resnorm[j] = rho_[j]; }
        rep.iters = it;
        if (mx <= tol) { status = HSYM_OK; rep.converged = 1; done = true; }
        else if (it >= o.maxit) { status = HSYM_NOT_CONVERGED; done = true; }
        return done;
    }

    // advance_a: step 6 (W = T^-1 R) and the first Cholesky-QR stage of step 7,
    // ending with the copy of the rank-deficiency flag
    GramArgs orth_gram() const {
        const double *B[2] = {X, P};
        const int kb = have_p ? 2 : 1;
        GramArgs g{};
        for (int i = 0; i < kb; i++) g.a[i] = B[i];
        g.a[kb] = W; g.b[0] = W; g.na = kb + 1; g.nb = 1; g.m = m; g.n = n;
        return g;
    }
    // gram_done: gbuf already holds [X P W]^T W (computed with the preconditioner)
    void orth_part1(bool gram_done = false) {
        const double *B[2] = {X, P};
        const int kb = have_p ? 2 : 1;
        mark(2);
        set_int(&st_d->flags[0], 0, s);
        const GramArgs g = orth_gram();
        if (!gram_done) gram(g, gbuf, gram_scr, s);
        OrthArgs oa{gbuf, coef, &st_d->flags[0], kb, m, 0};
        small_orth(&oa, 1, s);
        orth_lc = LincombArgs{};
        for (int i = 0; i < kb; i++) orth_lc.in[i] = B[i];
        orth_lc.in[kb] = W; orth_lc.out[0] = W; orth_lc.coef = coef; orth_lc.ldc = m; orth_lc.nin = kb + 1;
        orth_lc.nout = 1; orth_lc.nsets = 1; orth_lc.m = m; orth_lc.n = n;
        lincomb_gram(orth_lc, g, gbuf, gram_scr, s);   // the update and the next pass's Gram
        oa.stage = 1;
        small_orth(&oa, 1, s);
        HIPCHK(hipMemcpyAsync(&st_h->flags[0], &st_d->flags[0], sizeof(int), hipMemcpyDeviceToHost, s));
    }
    LincombArgs orth_lc{};
    int orth_attempt = 0;

    void advance_a() {
        it++;
        const bool pre = shifts(rho_, rnorm_, st_h->theta);
        orth_attempt = 0;
        auto body = [&] {
            bool gram_done = false;
            if (pre) {
                mark(1);
                HIPCHK(hipMemcpyAsync(mu, mu_h, sizeof(double) * m, hipMemcpyHostToDevice, s));
                const GramArgs g = orth_gram();
                if (precond == HSYM_PRECOND_JACOBI && jacobi_gram_fusable(g)) {
                    // the Jacobi apply and the first Gram in one pass over the rows
                    jacobi_gram(g, H->diag64, mu, o.guard * H->norm1, gbuf, gram_scr, s);
                    gram_done = true;
                } else {
                    precond_apply(H, precond, W, mu, o.guard * H->norm1, m, s, o.fom_iters);
                }
            }
            orth_part1(gram_done);
        };
        if (use_graph()) graphed(graph_a[pre ? 1 : 0], body);
        else body();
    }

    // a deficient W (flag copy complete): replace the flagged columns and redo
    // the first Cholesky-QR stage, ending with a new flag copy
    void repair_once() {
        const int flag = st_h->flags[0];
        if (orth_attempt >= 3) {
            // W stays dependent on [X P] after three random repairs (a basis
            // that nearly fills the space): restart the recurrence without P
            // for this iteration, which leaves W the room P took, as the
            // oracle drops P at a small pivot; without P the failure stands
            if (!have_p) fail(HSYM_E_BREAKDOWN, "block stays rank deficient after 3 random repairs");
            have_p = false;
            rep.p_dropped++;
            orth_attempt = 0;
        }
        int mask = flag & ((1 << m) - 1);
        rep.w_replaced += __builtin_popcount((unsigned)mask);
        mark(7);
        gauss_fill(W, n, m, m,
                   o.seed * 1000003ULL + (uint64_t)it * 101ULL + 7ULL + (uint64_t)orth_attempt + (have_p ? 0 : 50),
                   10, mask, s);
        orth_attempt++;
        orth_part1();
    }

    // Phase B: the second Cholesky-QR pass, the SpMM, Rayleigh-Ritz (steps
    // 7-9) and the update of X, P, AX, AP (step 10) fused with the next
    // residual, then the status copy.  It is enqueued right behind phase A,
    // before the rank flag is known: the two launches that overwrite the
    // basis (the second update of W and the update of X, P, AX, AP) write
    // nothing when the flag is set, so that a repair can start from them.
    void phase_b() {
        auto body = [&] {
            // second Cholesky-QR stage of W (projection and normalisation);
            // the Rayleigh-Ritz step measures what is left of W's deviation
            // from orthonormality
            LincombArgs lc2 = orth_lc;
            lc2.skip = &st_d->flags[0];
            lincomb(lc2, s);
            mark(0);
            spmm(W, AW);
            const int nblk = have_p ? 3 : 2;
            GramArgs g{};
            g.a[0] = X; g.a[1] = W; g.a[2] = P;
            g.b[0] = X; g.b[1] = W; g.b[2] = P;
            g.b[nblk] = AX; g.b[nblk + 1] = AW; if (nblk == 3) g.b[5] = AP;
            g.na = nblk; g.nb = 2 * nblk; g.m = m; g.n = n; g.sym = 1;
            mark(3);
            gram(g, gbuf, gram_scr, s);
            mark(4);
            rayleigh_ritz(nblk);
            mark(5);
            LincombArgs u{};
            u.in[0] = X; u.in[1] = W; u.in[2] = P; u.in[3] = AX; u.in[4] = AW; u.in[5] = AP;
            u.out[0] = X; u.out[1] = P; u.out[2] = AX; u.out[3] = AP;
            u.coef = rrcoef; u.ldc = 2 * m; u.nin = nblk; u.nout = 2; u.nsets = 2; u.m = m; u.n = n;
            u.theta = st_d->theta; u.res = W; u.norm_part = norm_part; u.skip = &st_d->flags[0];
            lincomb(u, s);
            colsum_final(norm_part, lincomb_norm_parts(n), m, st_d->norms, s);
            mark(7);
            post_status();
        };
        if (use_graph()) graphed(graph_b, body);
        else body();
        rep.spmm_calls++;
        have_p = true;
    }

    // One iteration with one host wait: phases A and B and the status copy
    // are enqueued together (begin), then the status is checked (complete).
    Status prev_st{};
    bool prev_have_p = false;
    void begin_iteration() {
        prev_st = *st_h;
        prev_have_p = have_p;
        advance_a();
        phase_b();
    }
    // A set rank flag (from Cholesky-QR stage 0, 1 or 2) means phase B left
    // X, P, AX, AP and W as they were: restore the status and P of before the
    // iteration, repair the flagged columns of W until the first stage is
    // clean, and run phase B again.
    void complete_iteration() {
        for (;;) {
            sync();
            const int flag = st_h->flags[0];
            if (!flag) return;
            *st_h = prev_st;
            st_h->flags[0] = flag;
            have_p = prev_have_p;
            do {
                repair_once();
                sync();
            } while (st_h->flags[0]);
            phase_b();
        }
    }

    // The launches enqueued from here on belong to phase ph (phase_ms[ph];
    // 0 is the SpMM, timed by its own events).  A roctx range names the phase
    // on the host timeline of a trace.
    static constexpr const char *PHASE_NAMES[8] = {"lobpcg: spmm", "lobpcg: preconditioner", "lobpcg: cholesky-qr",
                                                   "lobpcg: rr gram", "lobpcg: rr eigensolve", "lobpcg: update",
                                                   "lobpcg: wait", "lobpcg: other"};
    void mark(int ph) {
        if (!o.timers || capturing) return;
        if (range_open) roctxRangePop();
        roctxRangePush(PHASE_NAMES[ph]);
        range_open = true;
        record_mark(ph);
    }
    void record_mark(int ph) {
        if (nmark == NMARK) settle_marks(true);   // not reached in one iteration
        HIPCHK(hipEventRecord(ev_mark[nmark], s));
        mark_phase[nmark++] = ph;
    }
    // add the stretches between recorded marks to their phases (the last
    // mark ends a stretch and opens none, unless keep_last: then it stays
    // open as the first mark of the next window)
    void settle_marks(bool keep_last) {
        if (nmark == 0) return;
        HIPCHK(hipEventSynchronize(ev_mark[nmark - 1]));
        for (int i = 0; i + 1 < nmark; i++) {
            float ms = 0.0f;
            HIPCHK(hipEventElapsedTime(&ms, ev_mark[i], ev_mark[i + 1]));
            if (mark_phase[i] > 0) rep.phase_ms[mark_phase[i]] += ms;
        }
        if (keep_last) {
            std::swap(ev_mark[0], ev_mark[nmark - 1]);
            mark_phase[0] = mark_phase[nmark - 1];
            nmark = 1;
        } else {
            nmark = 0;
        }
    }

    void sync() {
        const bool timed = o.timers && !capturing;
        if (timed) {
            if (nmark > 0) record_mark(-1);   // closes the stretch in flight
            if (range_open) roctxRangePop();
            roctxRangePush(PHASE_NAMES[6]);
            range_open = true;
        }
        const auto w0 = std::chrono::steady_clock::now();
        HIPCHK(hipStreamSynchronize(s));
        if (timed) {
            rep.phase_ms[6] += std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - w0).count();
            settle_marks(false);
            roctxRangePop();
            range_open = false;
        }
        if (spmm_pending) {
            float ms = 0.0f;
            HIPCHK(hipEventElapsedTime(&ms, ev_spmm[0], ev_spmm[1]));
            rep.phase_ms[0] += ms;
            spmm_pending = false;
        }
    }

    // whole solve on one stream
    void run() {
        post_status();
        for (;;) {
            sync();
            if (evaluate()) return;
            begin_iteration();
            complete_iteration();
        }
    }

    void finish(double *evals, double *evecs) {
        for (int j = 0; j < nev; j++) evals[j] = st_h->theta[j];
        if (evecs) sign_fix_copy(X, m, nev, n, evecs, gram_scr, s);
        HIPCHK(hipStreamSynchronize(s));
        rep.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    }
};

// ---------------------------------------------------------------------------
// Batched steady-state iterations.  Contexts that are small, in the steady
// state (P present), use the Jacobi or no preconditioner and record no
// graphs are stepped together: every step of the iteration is one launch
// for all of them (argument tables in device memory, one problem per
// blockIdx.y), on one stream, with the iteration's host synchronisation
// shared.  The arithmetic of each problem is that of
// Lobpcg::advance_a / phase_b; only the launches are merged.
// ---------------------------------------------------------------------------
constexpr int64_t BATCH_MAX_N = (int64_t)1 << 18;   // larger problems fill the GPU alone
constexpr int BATCH_CAP = 256;

static bool batchable(const Lobpcg &L) {
    return L.have_p && !L.o.graph && L.n <= BATCH_MAX_N &&
           (L.precond == HSYM_PRECOND_NONE || L.precond == HSYM_PRECOND_JACOBI);
}

struct BatchPlan {
    hipStream_t bs = nullptr;
    std::vector<std::pair<const Lobpcg *, uint64_t>> key;   // contexts the tables describe
    // device tables (one allocation) and their pinned staging
    char *dev = nullptr, *pin = nullptr;
    size_t bytes = 0;
    GramJob *gA = nullptr, *gS = nullptr;
    LincombArgs *lcO = nullptr, *lcO2 = nullptr, *lcU = nullptr;   // lcO2: phase B's copy of lcO
    ColsumJob *cs = nullptr;
    SpmmJob *sp = nullptr;
    int **flag_ptr = nullptr;
    const int **stat_src = nullptr;
    int *stat_dst = nullptr;       // count x Status, device
    JacobiJob *jac = nullptr;      // per round
    double *mu = nullptr;          // per round: count x 16
    // host-side copies needed for launch shapes and the small kernels
    std::vector<SpmmJob> sp_h;
    std::vector<OrthArgs> o0, o1;
    std::vector<RRArgs> rr;
    int m = 0, storage = 0, count = 0;
    int64_t max_n = 0;
    int maxpA = 0, maxpS = 0;

    ~BatchPlan() {
        if (dev) (void)hipFree(dev);
        if (pin) (void)hipHostFree(pin);
        if (bs) (void)hipStreamDestroy(bs);
    }

    // (re)build the tables for the contexts in cs
    void build(const std::vector<Lobpcg *> &ctxs) {
        count = (int)ctxs.size();
        m = ctxs[0]->m;
        storage = ctxs[0]->H->storage;
        if (!bs) HIPCHK(hipStreamCreateWithFlags(&bs, hipStreamNonBlocking));
        if (!dev) {
            // layout for BATCH_CAP problems: offsets first, then one allocation
            size_t off = 0;
            auto at = [&](size_t each) {
                off = (off + 255) & ~(size_t)255;
                const size_t o = off;
                off += each * BATCH_CAP;
                return o;
            };
            const size_t oA = at(sizeof(GramJob)), oS = at(sizeof(GramJob));
            const size_t oO = at(sizeof(LincombArgs)), oO2 = at(sizeof(LincombArgs)), oU = at(sizeof(LincombArgs));
            const size_t oC = at(sizeof(ColsumJob)), oP = at(sizeof(SpmmJob)), oF = at(sizeof(int *));
            const size_t oR = at(sizeof(int *)), oT = at(sizeof(Status)), oJ = at(sizeof(JacobiJob));
            const size_t oM = at(sizeof(double) * HSYM_MAX_BLOCK);
            bytes = off;
            HIPCHK(hipMalloc((void **)&dev, bytes));
            HIPCHK(hipHostMalloc((void **)&pin, bytes, hipHostMallocDefault));
            gA = (GramJob *)(dev + oA); gS = (GramJob *)(dev + oS);
            lcO = (LincombArgs *)(dev + oO); lcO2 = (LincombArgs *)(dev + oO2); lcU = (LincombArgs *)(dev + oU);
            cs = (ColsumJob *)(dev + oC); sp = (SpmmJob *)(dev + oP); flag_ptr = (int **)(dev + oF);
            stat_src = (const int **)(dev + oR); stat_dst = (int *)(dev + oT); jac = (JacobiJob *)(dev + oJ);
            mu = (double *)(dev + oM);
        }
        auto host = [&](const void *d) { return pin + ((const char *)d - dev); };
        GramJob *hgA = (GramJob *)host(gA), *hgS = (GramJob *)host(gS);
        LincombArgs *hlO = (LincombArgs *)host(lcO), *hlO2 = (LincombArgs *)host(lcO2), *hlU = (LincombArgs *)host(lcU);
        ColsumJob *hcs = (ColsumJob *)host(cs);
        SpmmJob *hsp = (SpmmJob *)host(sp);
        int **hfl = (int **)host(flag_ptr);
        const int **hss = (const int **)host(stat_src);
        sp_h.assign((size_t)count, SpmmJob{});
        o0.clear(); o1.clear(); rr.clear();
        key.clear();
        max_n = 0; maxpA = maxpS = 0;
        auto gjob = [&](Lobpcg &L, const double *a0, const double *a1, const double *a2, const double *b0,
                        const double *b1, const double *b2, int na, int nb, int &maxp) {
            GramJob j{};
            j.g.a[0] = a0; j.g.a[1] = a1; j.g.a[2] = a2; j.g.b[0] = b0; j.g.b[1] = b1; j.g.b[2] = b2;
            j.g.na = na; j.g.nb = nb; j.g.m = L.m; j.g.n = L.n;
            j.parts = gram_parts(L.n);
            j.rpw = gram_rows(L.n, j.parts);
            j.part = L.gram_scr;
            j.kk = na * L.m * nb * L.m;
            j.out = L.gbuf;
            maxp = std::max(maxp, j.parts);
            return j;
        };
        for (int i = 0; i < count; i++) {
            Lobpcg &L = *ctxs[(size_t)i];
            key.emplace_back(&L, L.serial);
            max_n = std::max(max_n, L.n);
            hgA[i] = gjob(L, L.X, L.P, L.W, L.W, nullptr, nullptr, 3, 1, maxpA);
            hgS[i] = gjob(L, L.X, L.W, L.P, L.X, L.W, L.P, 3, 6, maxpS);
            hgS[i].g.b[3] = L.AX; hgS[i].g.b[4] = L.AW; hgS[i].g.b[5] = L.AP;
            LincombArgs lo{};
            lo.in[0] = L.X; lo.in[1] = L.P; lo.in[2] = L.W; lo.out[0] = L.W; lo.coef = L.coef; lo.ldc = L.m;
            lo.nin = 3; lo.nout = 1; lo.nsets = 1; lo.m = L.m; lo.n = L.n;
            hlO[i] = lo;
            lo.skip = &L.st_d->flags[0];   // phase B runs before the rank flag is read
            hlO2[i] = lo;
            LincombArgs u{};
            u.in[0] = L.X; u.in[1] = L.W; u.in[2] = L.P; u.in[3] = L.AX; u.in[4] = L.AW; u.in[5] = L.AP;
            u.out[0] = L.X; u.out[1] = L.P; u.out[2] = L.AX; u.out[3] = L.AP;
            u.coef = L.rrcoef; u.ldc = 2 * L.m; u.nin = 3; u.nout = 2; u.nsets = 2; u.m = L.m; u.n = L.n;
            u.theta = L.st_d->theta; u.res = L.W; u.norm_part = L.norm_part; u.skip = &L.st_d->flags[0];
            hlU[i] = u;
            hcs[i] = ColsumJob{L.norm_part, lincomb_norm_parts(L.n), L.m, L.st_d->norms};
            hsp[i] = spmm_job(L.H, L.m, L.W, L.AW);
            sp_h[(size_t)i] = hsp[i];
            hfl[i] = &L.st_d->flags[0];
            hss[i] = (const int *)L.st_d;
            o0.push_back(OrthArgs{L.gbuf, L.coef, &L.st_d->flags[0], 2, L.m, 0});
            o1.push_back(OrthArgs{L.gbuf, L.coef, &L.st_d->flags[0], 2, L.m, 1});
            RRArgs r{};
            r.gram = L.gbuf; r.coef = L.rrcoef; r.theta = L.st_d->theta; r.evals_all = nullptr;
            r.flag = &L.st_d->flags[1]; r.nblk = 3; r.m = L.m;
            rr.push_back(r);
        }
        // the static tables: everything before the per-round Jacobi jobs
        const size_t static_bytes = (size_t)((char *)jac - dev);
        HIPCHK(hipMemcpyAsync(dev, pin, static_bytes, hipMemcpyHostToDevice, bs));
    }

    bool matches(const std::vector<Lobpcg *> &ctxs) const {
        if (!dev || ctxs.size() != key.size()) return false;
        for (size_t i = 0; i < ctxs.size(); i++)
            if (key[i].first != ctxs[i] || key[i].second != ctxs[i]->serial) return false;
        return true;
    }

    // one iteration of every context (all evaluated, none done)
    void round(const std::vector<Lobpcg *> &ctxs) {
        std::vector<hipStream_t> own;
        for (Lobpcg *L : ctxs) {
            own.push_back(L->s);
            L->s = bs;
        }
        auto restore = [&] {
            for (size_t i = 0; i < ctxs.size(); i++) ctxs[i]->s = own[i];
        };
        try {
            // ---- phase A: shifts, preconditioner, first Cholesky-QR stage ----
            JacobiJob *hj = (JacobiJob *)(pin + ((char *)jac - dev));
            double *hmu = (double *)(pin + ((char *)mu - dev));
            int npre = 0;
            for (int i = 0; i < count; i++) {
                Lobpcg &L = *ctxs[(size_t)i];
                L.it++;
                L.orth_attempt = 0;
                L.orth_lc = LincombArgs{};
                L.orth_lc.in[0] = L.X; L.orth_lc.in[1] = L.P; L.orth_lc.in[2] = L.W; L.orth_lc.out[0] = L.W;
                L.orth_lc.coef = L.coef; L.orth_lc.ldc = L.m; L.orth_lc.nin = 3; L.orth_lc.nout = 1;
                L.orth_lc.nsets = 1; L.orth_lc.m = L.m; L.orth_lc.n = L.n;
                if (L.shifts(L.rho_, L.rnorm_, L.st_h->theta)) {
                    double *row = hmu + (size_t)npre * HSYM_MAX_BLOCK;
                    for (int j = 0; j < L.m; j++) row[j] = L.mu_h[j];
                    hj[npre] = JacobiJob{L.W, L.H->diag64, mu + (size_t)npre * HSYM_MAX_BLOCK,
                                         L.o.guard * L.H->norm1, L.n};
                    npre++;
                }
            }
            if (npre) {
                HIPCHK(hipMemcpyAsync(jac, hj, sizeof(JacobiJob) * (size_t)npre, hipMemcpyHostToDevice, bs));
                HIPCHK(hipMemcpyAsync(mu, hmu, sizeof(double) * HSYM_MAX_BLOCK * (size_t)npre,
                                      hipMemcpyHostToDevice, bs));
                jacobi_batched(jac, npre, m, max_n, bs);
            }
            set_ints(flag_ptr, count, 0, bs);
            gram_batched(gA, count, 3 * m, m, maxpA, bs);
            small_orth(o0.data(), count, bs);
            if (m == 16) {
                lincomb_gram_batched(lcO, gA, count, 3, maxpA, bs);
            } else {
                lincomb_batched(lcO, count, max_n, bs);
                gram_batched(gA, count, 3 * m, m, maxpA, bs);
            }
            small_orth(o1.data(), count, bs);
            // ---- phase B, enqueued at once: its launches that overwrite the
            // basis skip a problem whose rank flag is set (see Lobpcg::phase_b) ----
            lincomb_batched(lcO2, count, max_n, bs);
            spmm_batched(sp, sp_h.data(), count, m, storage, bs);
            gram_batched(gS, count, 3 * m, 6 * m, maxpS, bs);
            small_rr(rr.data(), count, bs);
            lincomb_batched(lcU, count, max_n, bs);
            colsum_batched(cs, count, m, bs);
            gather_words(stat_src, stat_dst, (int)(sizeof(Status) / 4), count, bs);
            Status *hst = (Status *)(pin + ((char *)stat_dst - dev));
            HIPCHK(hipMemcpyAsync(hst, stat_dst, sizeof(Status) * (size_t)count, hipMemcpyDeviceToHost, bs));
            HIPCHK(hipStreamSynchronize(bs));
            for (int i = 0; i < count; i++) {
                Lobpcg &L = *ctxs[(size_t)i];
                L.rep.spmm_calls++;
                if (!hst[i].flags[0]) {
                    memcpy(L.st_h, &hst[i], sizeof(Status));
                    L.rep.batched_iters++;
                    continue;
                }
                // rare: a deficient W; this problem's phase B wrote nothing to
                // its basis.  Repair it alone (same stream) and rerun phase B.
                const Status keep = *L.st_h;
                int flag = hst[i].flags[0];
                for (;;) {
                    L.st_h->flags[0] = flag;
                    do {
                        L.repair_once();
                        L.sync();
                    } while (L.st_h->flags[0]);
                    L.phase_b();
                    L.sync();
                    flag = L.st_h->flags[0];
                    if (!flag) break;
                    *L.st_h = keep;
                }
            }
        } catch (...) {
            (void)hipStreamSynchronize(bs);
            restore();
            throw;
        }
        restore();
    }
};

// per stepping thread: the plans of the batches stepped last (one per
// block width and storage precision)
struct BatchPlans {
    std::vector<std::pair<int, std::unique_ptr<BatchPlan>>> plans;
    BatchPlan &get(int key) {
        for (auto &p : plans)
            if (p.first == key) return *p.second;
        plans.emplace_back(key, std::make_unique<BatchPlan>());
        return *plans.back().second;
    }
};

static void step_batched(std::vector<Lobpcg *> &group) {
    static thread_local BatchPlans tp;
    const int key = group[0]->m * 2 + group[0]->H->storage;
    // groups larger than a plan's capacity run in slices, each with its plan
    for (size_t b0 = 0, slice = 0; b0 < group.size(); b0 += BATCH_CAP, slice++) {
        std::vector<Lobpcg *> part(group.begin() + (long)b0,
                                   group.begin() + (long)std::min(group.size(), b0 + BATCH_CAP));
        BatchPlan &P = tp.get(key + (int)slice * 64);
        if (!P.matches(part)) P.build(part);
        P.round(part);
    }
}

}  // namespace hsym

using namespace hsym;

extern "C" {

void lobpcg_opts_default(lobpcg_opts *o) {
    if (!o) return;
    memset(o, 0, sizeof(*o));
    o->maxit = 1000;
    o->seed = 0;
    o->check_every = 1;
    o->no_precond_iters = 3;
    o->near = 0.1;
    o->guard = 1e-4;
    o->keep_history = 1;
    o->fom_iters = 3;
}

static void check_solve_args(hsym_t H, int nev, int m, double tol) {
    if (!H || !H->ready) fail(HSYM_E_INVALID_ARG, "invalid handle");
    if (nev < 1 || m < nev || m > HSYM_MAX_BLOCK) fail(HSYM_E_INVALID_ARG, "need 1 <= nev <= block_width <= 16");
    if (3 * (int64_t)m > H->n) fail(HSYM_E_INVALID_ARG, "need 3*block_width <= n");
    if (!(tol > 0.0)) fail(HSYM_E_INVALID_ARG, "tol must be > 0");
}

int lobpcg_solve(hsym_t H, int nev, int block_width, double tol, const double *X0, int precond,
                 const lobpcg_opts *opts, double *evals, double *evecs, lobpcg_report *rep, void *stream) {
    try {
        check_solve_args(H, nev, block_width, tol);
        if (!evals) fail(HSYM_E_INVALID_ARG, "NULL evals");
        if (precond < HSYM_PRECOND_NONE || precond > HSYM_PRECOND_FOM) fail(HSYM_E_INVALID_ARG, "bad precond");
        Lobpcg L;
        L.setup(H, nev, block_width, tol, X0, precond, opts, (hipStream_t)stream);
        L.run();
        L.finish(evals, evecs);
        if (rep) *rep = L.rep;
        set_error("");
        return L.status;
    } catch (Error &e) {
        set_error(e.msg);
        return e.status;
    } catch (std::bad_alloc &) {
        set_error("host allocation failed");
        return HSYM_E_OUT_OF_MEMORY;
    }
}

}  // extern "C"

// ---------------------------------------------------------------------------
// context/step API
// ---------------------------------------------------------------------------
struct lobpcg_ctx {
    hsym::Lobpcg L;
    hipStream_t own = nullptr;
};

template <class F>
static int ctx_guard(F &&f) {
    try {
        int st = f();
        set_error("");
        return st;
    } catch (Error &e) {
        set_error(e.msg);
        return e.status;
    } catch (std::bad_alloc &) {
        set_error("host allocation failed");
        return HSYM_E_OUT_OF_MEMORY;
    }
}

extern "C" {

int lobpcg_ctx_create(lobpcg_ctx_t *out, hsym_t H, int nev, int block_width, double tol, const double *X0,
                      int precond, const lobpcg_opts *opts, void *stream) {
    if (out) *out = nullptr;
    return ctx_guard([&] {
        if (!out) fail(HSYM_E_INVALID_ARG, "NULL context pointer");
        check_solve_args(H, nev, block_width, tol);
        if (precond < HSYM_PRECOND_NONE || precond > HSYM_PRECOND_FOM) fail(HSYM_E_INVALID_ARG, "bad precond");
        lobpcg_ctx *c = new lobpcg_ctx();
        try {
            hipStream_t s = (hipStream_t)stream;
            if (!s) {
                HIPCHK(hipStreamCreateWithFlags(&c->own, hipStreamNonBlocking));
                s = c->own;
            }
            c->L.setup(H, nev, block_width, tol, X0, precond, opts, s);
            c->L.post_status();
        } catch (...) {
            if (c->own) (void)hipStreamDestroy(c->own);
            delete c;
            throw;
        }
        *out = c;
        return (int)HSYM_OK;
    });
}

// Advance every context by up to `iters` iterations.  Contexts on different
// streams overlap on the device: each phase is enqueued for all contexts
// before any of them is waited on.

int lobpcg_ctx_step(lobpcg_ctx_t *ctxs, int count, int iters) {
    return ctx_guard([&] {
        if ((!ctxs && count) || count < 0 || iters < 0) fail(HSYM_E_INVALID_ARG, "bad step arguments");
        for (int i = 0; i < count; i++) if (!ctxs[i]) fail(HSYM_E_INVALID_ARG, "NULL context");
        std::vector<Lobpcg *> act;
        for (int k = 0; k < iters; k++) {
            act.clear();
            for (int i = 0; i < count; i++) {
                Lobpcg &L = ctxs[i]->L;
                if (L.done) continue;
                L.sync();
                if (!L.evaluate()) act.push_back(&L);
            }
            if (act.empty()) break;
            // small steady-state contexts of equal block width and storage
            // step together (one launch per step for all of them)
            std::vector<std::vector<Lobpcg *>> groups;
            std::vector<Lobpcg *> solo;
            for (Lobpcg *L : act) {
                if (!batchable(*L)) {
                    solo.push_back(L);
                    continue;
                }
                bool placed = false;
                for (auto &g : groups)
                    if (g[0]->m == L->m && g[0]->H->storage == L->H->storage) {
                        g.push_back(L);
                        placed = true;
                        break;
                    }
                if (!placed) groups.push_back({L});
            }
            for (auto &g : groups)
                if (g.size() < 2) solo.push_back(g[0]);
            for (Lobpcg *L : solo) L->begin_iteration();
            for (auto &g : groups)
                if (g.size() >= 2) step_batched(g);
            for (Lobpcg *L : solo) L->complete_iteration();
        }
        return (int)HSYM_OK;
    });
}

int lobpcg_ctx_status(lobpcg_ctx_t c, int *done, double *evals, lobpcg_report *rep) {
    return ctx_guard([&] {
        if (!c) fail(HSYM_E_INVALID_ARG, "NULL context");
        Lobpcg &L = c->L;
        L.sync();
        bool d = L.evaluate();
        if (done) *done = d ? 1 : 0;
        if (evals) for (int j = 0; j < L.nev; j++) evals[j] = L.st_h->theta[j];
        if (rep) {
            L.rep.seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - L.t0).count();
            *rep = L.rep;
        }
        return d ? L.status : (int)HSYM_NOT_CONVERGED;
    });
}

int lobpcg_ctx_evecs(lobpcg_ctx_t c, double *evecs) {
    return ctx_guard([&] {
        if (!c || !evecs) fail(HSYM_E_INVALID_ARG, "NULL argument");
        Lobpcg &L = c->L;
        sign_fix_copy(L.X, L.m, L.nev, L.n, evecs, L.gram_scr, L.s);
        L.sync();
        return (int)HSYM_OK;
    });
}

int64_t lobpcg_ctx_device_bytes(lobpcg_ctx_t c) { return c ? c->L.bytes : 0; }

int lobpcg_ctx_destroy(lobpcg_ctx_t c) {
    return ctx_guard([&] {
        if (!c) fail(HSYM_E_INVALID_ARG, "NULL context");
        (void)hipStreamSynchronize(c->L.s);
        hipStream_t own = c->own;
        delete c;
        if (own) (void)hipStreamDestroy(own);
        return (int)HSYM_OK;
    });
}

}  // extern "C"
