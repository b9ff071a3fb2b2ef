// Request loop around the solver: continuous batching of LOBPCG solves at
// iteration granularity.  Requests arrive over time (arrival_s), are admitted
// in arrival order while their estimated device memory fits a budget, are
// loaded (tile-format build and context set-up) by loader threads, and every
// active request is advanced by a few iterations per scheduling round, so a
// short request does not wait for a long one to finish.  The paper runs one
// solve per job; this loop is the serving layer around its method.
//
// The scheduler is written once over a small backend interface: the device
// backend drives the library's public entry points, the virtual-clock backend
// (hsym_serve_sim) replays given service times without a GPU so that the
// admission and accounting logic can be checked on the host.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <condition_variable>
#include <cstring>
#include <deque>
#include <limits>
#include <map>
#include <mutex>
#include <thread>
#include <vector>

#include "hsym_internal.h"

namespace hsym {
namespace {

struct Backend {
    virtual ~Backend() {}
    virtual double now() = 0;                               // seconds since the trace started
    virtual int64_t estimate(int r) = 0;                    // device bytes to reserve before loading
    virtual void load(int r) = 0;                           // start loading request r
    virtual void collect(std::vector<int> &ready) = 0;      // loads finished since the last call
    virtual void idle(double until) = 0;                    // nothing to step: wait for a load or `until`
    virtual void step(std::vector<int> &active, int iters) = 0;
    virtual bool finished(int r) = 0;                       // after a step: request r is done
    virtual int64_t actual_bytes(int r) = 0;                // device bytes held once loaded
    virtual void retire(int r) = 0;                         // free the request's device state
};

void run_schedule(hsym_request *q, int count, const hsym_serve_opts &o, Backend &be, hsym_serve_report *rep) {
    std::vector<int> order(count);
    for (int i = 0; i < count; i++) order[i] = i;
    std::stable_sort(order.begin(), order.end(),
                     [&](int a, int b) { return q[a].arrival_s < q[b].arrival_s; });
    std::vector<int64_t> resv(count, 0);
    std::vector<int> active, ready;
    int next = 0, finished = 0, inflight = 0, rounds = 0, max_act = 0;
    int64_t reserved = 0, peak = 0;
    auto finish = [&](int r, double t) {
        q[r].finish_s = t;
        reserved -= resv[r];
        resv[r] = 0;
        finished++;
    };
    while (finished < count) {
        const double t = be.now();
        // admission in arrival order; a request that does not fit holds the queue
        while (next < count) {
            const int r = order[next];
            if (q[r].arrival_s > t) break;
            const int64_t est = be.estimate(r);
            if (est > o.budget_bytes) {
                q[r].status = HSYM_E_OUT_OF_MEMORY;
                q[r].admit_s = t;
                next++;
                finish(r, t);
                continue;
            }
            if (inflight >= o.max_active || reserved + est > o.budget_bytes) break;
            resv[r] = est;
            reserved += est;
            peak = std::max(peak, reserved);
            inflight++;
            q[r].admit_s = t;
            be.load(r);
            next++;
        }
        ready.clear();
        be.collect(ready);
        for (int r : ready) {
            if (q[r].status < 0) {       // load failed
                inflight--;
                finish(r, be.now());
                continue;
            }
            const int64_t b = be.actual_bytes(r);
            q[r].device_bytes = b;
            active.push_back(r);
        }
        if (active.empty()) {
            be.idle(next < count ? q[order[next]].arrival_s : std::numeric_limits<double>::infinity());
            continue;
        }
        max_act = std::max(max_act, (int)active.size());
        be.step(active, o.iters_per_round);
        rounds++;
        std::vector<int> keep;
        for (int r : active) {
            if (be.finished(r)) {
                be.retire(r);
                inflight--;
                finish(r, be.now());
            } else {
                keep.push_back(r);
            }
        }
        active.swap(keep);
    }
    if (rep) {
        double first = std::numeric_limits<double>::infinity(), last = 0.0;
        for (int i = 0; i < count; i++) {
            first = std::min(first, q[i].arrival_s);
            last = std::max(last, q[i].finish_s);
        }
        rep->wall_s = count ? last - first : 0.0;
        rep->rounds = rounds;
        rep->tuned_classes = 0;
        rep->max_active_seen = max_act;
        rep->peak_reserved_bytes = peak;
    }
}

// ---------------------------------------------------------------------------
// Device backend
// ---------------------------------------------------------------------------
// copy the calling thread's last error message into a request
static void note(hsym_request &x) {
    std::strncpy(x.error, hsym_last_error(), sizeof(x.error) - 1);
    x.error[sizeof(x.error) - 1] = 0;
}

struct DeviceBackend : Backend {
    hsym_request *q;
    const hsym_serve_opts &o;
    std::chrono::steady_clock::time_point t0 = std::chrono::steady_clock::now();
    std::vector<hsym_t> H;
    std::vector<lobpcg_ctx_t> C;
    std::mutex mu;
    std::condition_variable cv;
    std::deque<int> jobs, done;
    bool stop = false;
    std::vector<std::thread> loaders;
    // panel geometry per size class (shared by the loader threads)
    std::mutex geom_mu;
    std::map<int64_t, int> geom;
    int tuned = 0;

    DeviceBackend(hsym_request *q_, int count, const hsym_serve_opts &o_) : q(q_), o(o_), H(count), C(count) {
        for (int i = 0; i < o.loaders; i++) loaders.emplace_back([this] { loader_main(); });
    }
    ~DeviceBackend() override {
        {
            std::lock_guard<std::mutex> g(mu);
            stop = true;
        }
        cv.notify_all();
        for (auto &t : loaders) t.join();
        for (size_t r = 0; r < C.size(); r++) retire((int)r);
    }
    double now() override {
        return std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    }
    int64_t estimate(int r) override {
        const hsym_request &x = q[r];
        const int64_t nnz = x.rowptr ? x.rowptr[x.n] : 0;
        const int vb = x.storage == HSYM_FP32 ? 4 : 8;
        // tile streams with slice padding and transposed-half partials, the
        // diagonal, and about 16 n x m fp64 blocks of the iteration
        return (int64_t)(1.3 * (double)nnz * (vb + 4)) + x.n * 16 + x.n * (int64_t)x.block_width * 8 * 16 +
               ((int64_t)8 << 20);
    }
    void load(int r) override {
        {
            std::lock_guard<std::mutex> g(mu);
            jobs.push_back(r);
        }
        cv.notify_all();
    }
    // tile geometry for a request: sized for its block width, or the panel
    // shape the autotuner chose for its size class
    int geometry(const hsym_request &x) {
        const int dflt = HSYM_GEOM_M(x.block_width);
        if (!o.autotune) return dflt;
        int lg = 0;
        while (((int64_t)2 << lg) <= x.n) lg++;
        const int64_t key = ((int64_t)lg << 8) | (x.block_width << 1) | x.storage;
        // one tuning per class: other loaders wait for it
        std::lock_guard<std::mutex> g(geom_mu);
        auto it = geom.find(key);
        if (it == geom.end()) {
            int f = 0;
            if (hsym_autotune_geometry(x.n, x.rowptr, x.colind, x.values, x.values_prec, x.storage, x.block_width, 0,
                                       &f, nullptr, 0, nullptr) == HSYM_OK)
                tuned++;
            else
                f = 0;   // keep the default geometry for this class
            it = geom.emplace(key, f).first;
        }
        return it->second ? it->second : dflt;
    }

    void loader_main() {
        for (;;) {
            int r;
            {
                std::unique_lock<std::mutex> g(mu);
                cv.wait(g, [&] { return stop || !jobs.empty(); });
                if (stop) return;
                r = jobs.front();
                jobs.pop_front();
            }
            hsym_request &x = q[r];
            int st = hsym_create(&H[r], x.n, x.rowptr, x.colind, x.values, x.values_prec, x.storage,
                                 HSYM_HOST_PTRS | geometry(x), nullptr);
            if (st == HSYM_OK) {
                lobpcg_opts op;
                lobpcg_opts_default(&op);
                op.seed = x.seed;
                if (o.maxit > 0) op.maxit = o.maxit;
                op.keep_history = 0;
                // no graph recording: the runtime refuses the loader thread's
                // stream synchronisations while another thread records
                op.graph = 0;
                st = lobpcg_ctx_create(&C[r], H[r], x.nev, x.block_width, x.tol, nullptr, x.precond, &op, nullptr);
            }
            if (st != HSYM_OK) {
                x.status = st;
                note(x);
                if (C[r]) { lobpcg_ctx_destroy(C[r]); C[r] = nullptr; }
                if (H[r]) { hsym_destroy(H[r]); H[r] = nullptr; }
            }
            {
                std::lock_guard<std::mutex> g(mu);
                done.push_back(r);
            }
            cv.notify_all();
        }
    }
    void collect(std::vector<int> &ready) override {
        std::lock_guard<std::mutex> g(mu);
        while (!done.empty()) {
            ready.push_back(done.front());
            done.pop_front();
        }
    }
    void idle(double until) override {
        std::unique_lock<std::mutex> g(mu);
        const double wait = std::min(std::max(until - now(), 0.0), 0.01);
        cv.wait_for(g, std::chrono::duration<double>(wait), [&] { return !done.empty(); });
    }
    void step(std::vector<int> &active, int iters) override {
        std::vector<lobpcg_ctx_t> cs;
        for (int r : active) cs.push_back(C[r]);
        if (lobpcg_ctx_step(cs.data(), (int)cs.size(), iters) == HSYM_OK) return;
        // some context failed: step them one by one and mark the failures
        for (int r : active) {
            const int st = lobpcg_ctx_step(&C[r], 1, iters);
            if (st != HSYM_OK) { q[r].status = st; note(q[r]); }
        }
    }
    bool finished(int r) override {
        hsym_request &x = q[r];
        if (x.status < 0) return true;
        int d = 0;
        lobpcg_report rp;
        const int st = lobpcg_ctx_status(C[r], &d, x.evals, &rp);
        if (st < 0) {
            x.status = st;
            note(x);
            return true;
        }
        if (!d) return false;
        x.iters = rp.iters;
        x.status = rp.converged ? HSYM_OK : HSYM_NOT_CONVERGED;
        return true;
    }
    int64_t actual_bytes(int r) override {
        hsym_info_t inf;
        int64_t b = 0;
        if (H[r] && hsym_info(H[r], &inf) == HSYM_OK) b += inf.device_bytes;
        if (C[r]) b += lobpcg_ctx_device_bytes(C[r]);
        return b;
    }
    void retire(int r) override {
        if (C[r]) { lobpcg_ctx_destroy(C[r]); C[r] = nullptr; }
        if (H[r]) { hsym_destroy(H[r]); H[r] = nullptr; }
    }
};

// ---------------------------------------------------------------------------
// Virtual-clock backend: loads take load_s each on one loader, a round costs
// the longest iteration time among the requests stepped in it.
// ---------------------------------------------------------------------------
struct SimBackend : Backend {
    hsym_request *q;
    const int *iters;
    const double *iter_s;
    const int64_t *bytes;
    double load_s;
    double vt = 0.0, loader_free = 0.0;
    std::vector<double> ready_at;
    std::vector<int> progress;
    std::vector<int> loading;

    SimBackend(hsym_request *q_, int count, const int *it, const double *its, const int64_t *b, double ls)
        : q(q_), iters(it), iter_s(its), bytes(b), load_s(ls), ready_at(count, 0.0), progress(count, 0) {}
    double now() override { return vt; }
    int64_t estimate(int r) override { return bytes[r]; }
    void load(int r) override {
        loader_free = std::max(loader_free, vt) + load_s;
        ready_at[r] = loader_free;
        loading.push_back(r);
    }
    void collect(std::vector<int> &ready) override {
        std::vector<int> keep;
        for (int r : loading) (ready_at[r] <= vt ? ready : keep).push_back(r);
        loading.swap(keep);
    }
    void idle(double until) override {
        double t = until;
        for (int r : loading) t = std::min(t, ready_at[r]);
        if (!std::isfinite(t)) fail(HSYM_E_INVALID_ARG, "simulated schedule cannot make progress");
        vt = std::max(vt, t);
    }
    void step(std::vector<int> &active, int it) override {
        double c = 0.0;
        for (int r : active) c = std::max(c, iter_s[r]);
        vt += c * it;
        for (int r : active) progress[r] += it;
    }
    bool finished(int r) override {
        if (progress[r] < iters[r]) return false;
        q[r].iters = iters[r];
        q[r].status = HSYM_OK;
        return true;
    }
    int64_t actual_bytes(int r) override { return bytes[r]; }
    void retire(int) override {}
};

void check_opts(hsym_serve_opts &o, const hsym_serve_opts *in) {
    hsym_serve_opts_default(&o);
    if (in) {
        if (in->budget_bytes > 0) o.budget_bytes = in->budget_bytes;
        if (in->max_active > 0) o.max_active = in->max_active;
        if (in->iters_per_round > 0) o.iters_per_round = in->iters_per_round;
        if (in->maxit > 0) o.maxit = in->maxit;
        o.autotune = in->autotune ? 1 : 0;
        if (in->loaders > 0) o.loaders = std::min(in->loaders, 16);
    }
}

void reset_outputs(hsym_request *q, int count) {
    for (int i = 0; i < count; i++) {
        q[i].status = HSYM_OK;
        q[i].iters = 0;
        std::memset(q[i].evals, 0, sizeof(q[i].evals));
        q[i].admit_s = q[i].finish_s = 0.0;
        q[i].device_bytes = 0;
        q[i].error[0] = 0;
    }
}

}  // namespace
}  // namespace hsym

using namespace hsym;

template <class F>
static int serve_guard(F &&f) {
    try {
        f();
        set_error("");
        return HSYM_OK;
    } catch (Error &e) {
        set_error(e.msg);
        return e.status;
    } catch (std::bad_alloc &) {
        set_error("host allocation failed");
        return HSYM_E_OUT_OF_MEMORY;
    } catch (std::exception &e) {
        set_error(e.what());
        return HSYM_E_DEVICE;
    }
}

extern "C" {

void hsym_serve_opts_default(hsym_serve_opts *o) {
    o->budget_bytes = (int64_t)200 << 30;
    o->max_active = 64;
    o->iters_per_round = 1;
    o->maxit = 1000;
    o->autotune = 0;
    o->loaders = 2;
}

int hsym_serve(hsym_request *reqs, int count, const hsym_serve_opts *opts, hsym_serve_report *rep) {
    return serve_guard([&] {
        if (count < 0 || (count && !reqs)) fail(HSYM_E_INVALID_ARG, "bad request array");
        for (int i = 0; i < count; i++) {
            const hsym_request &x = reqs[i];
            if (x.n < 1 || !x.rowptr || !x.colind || !x.values || !(x.arrival_s >= 0.0) || x.nev < 1 ||
                x.block_width < x.nev || x.block_width > HSYM_MAX_BLOCK || !(x.tol > 0.0))
                fail(HSYM_E_INVALID_ARG, "request " + std::to_string(i) + " is malformed");
        }
        hsym_serve_opts o;
        check_opts(o, opts);
        reset_outputs(reqs, count);
        DeviceBackend be(reqs, count, o);
        run_schedule(reqs, count, o, be, rep);
        if (rep) {
            // every load has been collected through the queue lock by now
            std::lock_guard<std::mutex> g(be.geom_mu);
            rep->tuned_classes = be.tuned;
        }
    });
}

int hsym_serve_sim(hsym_request *reqs, int count, const hsym_serve_opts *opts, const int *iters,
                   const double *iter_s, const int64_t *bytes, double load_s, hsym_serve_report *rep) {
    return serve_guard([&] {
        if (count < 0 || (count && (!reqs || !iters || !iter_s || !bytes)) || !(load_s >= 0.0))
            fail(HSYM_E_INVALID_ARG, "bad simulation arguments");
        for (int i = 0; i < count; i++)
            if (!(reqs[i].arrival_s >= 0.0) || iters[i] < 1 || !(iter_s[i] >= 0.0) || bytes[i] < 0)
                fail(HSYM_E_INVALID_ARG, "request " + std::to_string(i) + " is malformed");
        hsym_serve_opts o;
        check_opts(o, opts);
        reset_outputs(reqs, count);
        SimBackend be(reqs, count, iters, iter_s, bytes, load_s);
        run_schedule(reqs, count, o, be, rep);
    });
}

}  // extern "C"
