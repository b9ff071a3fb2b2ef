"""Benchmark of the LOBPCG hot path on one MI355X.

Default workload (the configuration the headline metric, mixed against fp64
time to tolerance, is quoted on): the largest single-GPU instance, a seeded
synthetic CI-shaped symmetric matrix with n = 30,000,000 and about 500
nonzeros per full row (7.5e9 stored upper entries), m = 16, nev = 10,
tol = 1e-6, the block-diagonal preconditioner from exact 64x64 diagonal
blocks.  One step = one complete LOBPCG solve of the mixed form (fp32
storage and SpMM; Cholesky-QR, Rayleigh-Ritz and residuals in fp64) with the
matrix resident in HBM; the fp64 form is built and solved once for the
ratio.  The roofline is that of the SpMM launches inside the timed solves
(HIP events on the solve stream); the per-phase split comes from the
solver's own phase events.  cpu_baseline is the oracle on a bounded slab.

--workload C2 gives the n = 500,000 fp64 line with the Lanczos baseline,
the FOM preconditioner, the multi-level start block and the request loop;
--workload C3 the n = 5,000,000 mixed-vs-fp64 line.

Prints one JSON line.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import numpy as np  # noqa: E402

METRIC = "LOBPCG s-to-tol + SpMM HBM GB/s (% peak), mixed vs FP64; solves/s, p99"
HBM_PEAK_GBS = 8000.0
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "spmm_sym_fp64_m16_n500k_traffic.txt")
KERNEL_SOURCES = [os.path.join(ROOT, "paper_1609_01689_amd", "csrc", f) for f in ("spmm.hip", "build.cpp")]
CALIB_BYTES = 512 << 20


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def kernel_source_hash():
    import hashlib
    h = hashlib.sha1()
    for f in KERNEL_SOURCES:
        with open(f, "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def measured_traffic(path, m):
    """HBM bytes per SpMM call from a committed counter summary (FETCH_SIZE
    and WRITE_SIZE of the SpMM's kernels, scaled by the factor the same
    counters give for an elementwise kernel of known size), or None when the
    summary is absent, for another block width, or the kernel sources changed
    since it was taken."""
    if not os.path.exists(path):
        return None
    kv = {}
    with open(path) as fh:
        for line in fh:
            if ":" in line and not line.startswith("#"):
                k, v = line.split(":", 1)
                kv[k.strip()] = v.strip()
    if kv.get("kernel_source_sha1") != kernel_source_hash() or int(kv.get("block_width", -1)) != m:
        return None
    return float(kv["hbm_bytes_per_call"])


def calibration_kernel(torch):
    """An elementwise kernel of known traffic (reads and writes CALIB_BYTES
    each), run so that counter runs of this script can scale FETCH_SIZE and
    WRITE_SIZE."""
    a = torch.ones(CALIB_BYTES // 8, dtype=torch.float64, device="cuda:0")
    b = torch.empty_like(a)
    for _ in range(3):
        torch.mul(a, 1.0000001, out=b)
    torch.cuda.synchronize()
    del a, b


def spmm_algorithmic_bytes(nnz_stored, n, m, val_bytes, x_bytes, y_bytes):
    """What the product must move: every stored entry once (value + int32
    column index), X read once, Y written once."""
    return nnz_stored * (val_bytes + 4) + n * m * x_bytes + n * m * y_bytes


def time_spmm(hs, torch, M, m, reps, dtype):
    n = M.n
    X = torch.randn((n, m), dtype=dtype, device="cuda:0")
    Y = torch.empty_like(X)
    fn = hs.spmm_sym if dtype == torch.float64 else hs.spmm_sym_f32
    for _ in range(3):
        fn(M.h, X, Y)
    torch.cuda.synchronize()
    s = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(s)
    for _ in range(reps):
        fn(M.h, X, Y, stream=s)
    e1.record(s)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / reps


def serving(hs, torch, count, seed=5):
    """Request-loop measurement on a stream of CI-shaped requests: n
    log-uniform in [1e3, 2e6], N = 40, nev ~ U{1..8}, m = 8, tol 1e-6, Jacobi.
    Baseline: the same requests solved one at a time in arrival order with
    fp64 storage (service time = build + solve + free, measured); arrivals
    are Poisson at twice the baseline's solves/s.  The request loop serves
    the trace with fp32 storage (mixed form) on the device, then the same
    requests all present at once (its capacity)."""
    import hsymgen
    rng = np.random.default_rng(seed)
    ns = np.round(10 ** rng.uniform(3, np.log10(2e6), count)).astype(np.int64)
    nevs = rng.integers(1, 9, count)
    t = time.perf_counter()
    mats = []
    for r, n in enumerate(ns):
        mats.append(hsymgen.generate(int(n), 40, 1000 + r))
        if (r + 1) % 250 == 0 and r + 1 < count:
            log("serving: generated %d of %d requests" % (r + 1, count))
    log("serving: generated %d requests (%.0fM stored entries) in %.1fs" %
        (count, sum(A.nnz for A in mats) / 1e6, time.perf_counter() - t))
    svc = []
    for r, A in enumerate(mats):
        torch.cuda.synchronize()
        t = time.perf_counter()
        M = hs.Matrix(A, storage=hs.HSYM_FP64, geom_m=8)
        st, ev, rep = hs.lobpcg_solve(M.h, int(nevs[r]), 8, 1e-6, precond="jacobi",
                                      opts=hs.default_lobpcg_opts(seed=1000 + r, keep_history=0))
        M.close()
        torch.cuda.synchronize()
        svc.append(time.perf_counter() - t)
        if (r + 1) % 250 == 0 and r + 1 < count:
            log("serving: sequential fp64 baseline, %d of %d solved" % (r + 1, count))
    svc = np.array(svc)
    rate = 2.0 * count / svc.sum()
    arr = np.cumsum(np.random.default_rng(seed).exponential(1.0 / rate, count))
    fin = np.zeros(count)
    prev = 0.0
    for r in range(count):
        prev = max(arr[r], prev) + svc[r]
        fin[r] = prev
    lat_fifo = fin - arr
    reqs = [{"csr": A, "storage": hs.HSYM_FP32, "nev": int(nevs[r]), "block_width": 8, "precond": "jacobi",
             "tol": 1e-6, "seed": 1000 + r, "arrival_s": float(arr[r])} for r, A in enumerate(mats)]
    res, rep = hs.hsym_serve(reqs)
    lat = np.array([x["latency_s"] for x in res])
    ok = sum(x["status"] == hs.HSYM_OK for x in res)
    out = {"requests": count, "arrival_rate_per_s": rate,
           "fifo_fp64": {"p50_s": float(np.percentile(lat_fifo, 50)), "p99_s": float(np.percentile(lat_fifo, 99)),
                         "solves_per_s": count / (fin[-1] - arr[0]), "mean_service_s": float(svc.mean())},
           "request_loop_mixed": {"p50_s": float(np.percentile(lat, 50)), "p99_s": float(np.percentile(lat, 99)),
                                  "solves_per_s": count / rep["wall_s"], "converged": ok,
                                  "max_active": rep["max_active_seen"], "rounds": rep["rounds"],
                                  "peak_reserved_GB": rep["peak_reserved_bytes"] / 1e9}}
    # capacity: the same requests all present at t = 0
    for q in reqs:
        q["arrival_s"] = 0.0
    res, rep = hs.hsym_serve(reqs)
    lat = np.array([x["latency_s"] for x in res])
    out["request_loop_saturated"] = {"solves_per_s": count / rep["wall_s"],
                                     "p50_s": float(np.percentile(lat, 50)), "p99_s": float(np.percentile(lat, 99)),
                                     "converged": sum(x["status"] == hs.HSYM_OK for x in res),
                                     "max_active": rep["max_active_seen"]}
    out["fifo_fp64_capacity_solves_per_s"] = float(1.0 / svc.mean())
    log("serving: %s" % json.dumps(out))
    return out


def stream_create(hs, g, storage, dtype, flags, slab=250_000):
    h = hs.hsym_create_begin(g.n, storage, flags)
    t = time.perf_counter()
    for r0 in range(0, g.n, slab):
        rp, ci, v = g.rows(r0, min(g.n, r0 + slab), dtype)
        hs.hsym_create_append(h, rp, ci, v)
        if (r0 // slab) % 20 == 19:
            log("  create: %d of %d rows, %.0fs" % (r0 + slab, g.n, time.perf_counter() - t))
    hs.hsym_create_finish(h)
    return h


def host_info():
    """CPU model, cores this process may use, and RAM of the host."""
    model, mem_kb = "unknown", 0
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
        with open("/proc/meminfo") as fh:
            for line in fh:
                if line.startswith("MemTotal"):
                    mem_kb = int(line.split()[1])
                    break
    except OSError:
        pass
    return {"cpu_model": model, "cores": len(os.sched_getaffinity(0)), "ram_GB": round(mem_kb / 1e6, 1)}


def traffic_file(form, m, n):
    return os.path.join(ROOT, "profiles", "spmm_sym_%s_m%d_n%s_traffic.txt" % (form, m, short_n(n)))


def short_n(n):
    return "%dM" % (n // 1_000_000) if n % 1_000_000 == 0 else "%dk" % (n // 1000)


def solve_timed(hs, torch, h, nev, m, tol, precond, opts, steps, warmup, label):
    """warmup untimed solves, then steps timed ones (synchronised on both
    sides); returns the times, the last report and eigenvalues, and the SpMM
    launch time and the phase split summed over the timed solves."""
    for k in range(warmup):
        t = time.perf_counter()
        st, ev, rep = hs.lobpcg_solve(h, nev, m, tol, precond=precond, opts=opts)
        torch.cuda.synchronize()
        log("%s: warm-up solve %d: status %d, %d iterations, %.2fs" % (label, k, st, rep.iters,
                                                                      time.perf_counter() - t))
    times, iters = [], []
    phase = np.zeros(8)
    spmm_calls = 0
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(steps):
        t = time.perf_counter()
        st, ev, rep = hs.lobpcg_solve(h, nev, m, tol, precond=precond, opts=opts)
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t)
        iters.append(rep.iters)
        phase += np.array(rep.phase_ms[:8])
        spmm_calls += rep.spmm_calls
        log("%s: timed solve %d: status %d, %d iterations, %.2fs" % (label, k, st, rep.iters, times[-1]))
        assert st == hs.HSYM_OK, "%s solve did not converge (status %d)" % (label, st)
    torch.cuda.synchronize()
    total = time.perf_counter() - t0
    return {"times": times, "total": total, "iters": iters, "rep": rep, "evals": ev, "phase_ms": phase,
            "spmm_calls": spmm_calls}


def phase_split(ph, steps):
    names = ["spmm", "preconditioner", "cholesky_qr", "rr_gram", "rr_eigensolve", "update", "host_wait", "other"]
    return {k: float(v) / max(1, steps) for k, v in zip(names, ph)}


def spmm_only(args, name):
    """The SpMM of the workload's timed form alone, for counter runs: the
    handle (built as the benchmark builds it), the calibration kernel and
    three calls."""
    import torch
    import hsymgen
    import paper_1609_01689_amd as hs
    cfg = hsymgen.CONFIGS[name]
    m = 16
    g = hsymgen.Generator(cfg["n"], cfg["N"], cfg["seed"])
    storage = hs.HSYM_FP64 if args.form == "fp64" else hs.HSYM_FP32
    flags = hs.HSYM_GEOM_M(m) | (hs.HSYM_BUILD_BLOCK64 if name == "C4" else 0)
    h = stream_create(hs, g, storage, np.float64 if storage == hs.HSYM_FP64 else np.float32, flags)
    calibration_kernel(torch)
    X = torch.randn((g.n, m), dtype=torch.float64, device="cuda:0")
    Y = torch.empty_like(X)
    for _ in range(3):
        hs.spmm_sym(h, X, Y)
    torch.cuda.synchronize()
    log("spmm-only %s %s: %s" % (name, args.form, hs.hsym_info(h)))
    hs.hsym_destroy(h)


def scale_workload(args, name):
    """The large configurations (C3: n = 5M, N = 400, Jacobi; C4: n = 30M,
    N = 500, block-64 preconditioner): nev = 10, m = 16, tol 1e-6, the mixed
    form (fp32 storage) against the fp64 form.  Each handle is built by
    streaming create from generator slabs and freed before the next.  One
    step = one solve of the mixed form; the fp64 form is solved once for the
    ratio."""
    import torch
    import hsymgen
    import paper_1609_01689_amd as hs
    cfg = hsymgen.CONFIGS[name]
    nev, m, tol = 10, 16, 1e-6
    precond = "block64" if name == "C4" else "jacobi"
    flags = hs.HSYM_GEOM_M(m) | (hs.HSYM_BUILD_BLOCK64 if precond == "block64" else 0)
    g = hsymgen.Generator(cfg["n"], cfg["N"], cfg["seed"])
    dev = torch.device("cuda:0")
    res = {}
    opts = hs.default_lobpcg_opts(seed=1, keep_history=0, timers=1)
    for label, storage, dtype in (("mixed", hs.HSYM_FP32, np.float32), ("fp64", hs.HSYM_FP64, np.float64)):
        t = time.perf_counter()
        h = stream_create(hs, g, storage, dtype, flags)
        torch.cuda.synchronize()
        build_s = time.perf_counter() - t
        info = hs.hsym_info(h)
        log("%s %s: built in %.1fs: %s" % (name, label, build_s, info))
        X = torch.randn((g.n, m), dtype=torch.float64, device=dev)
        Y = torch.empty_like(X)
        hs.spmm_sym(h, X, Y)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        st_ = torch.cuda.current_stream()
        e0.record(st_)
        for _ in range(3):
            hs.spmm_sym(h, X, Y, stream=st_)
        e1.record(st_)
        torch.cuda.synchronize()
        spmm_ms = e0.elapsed_time(e1) / 3
        del X, Y
        vb = 4 if storage == hs.HSYM_FP32 else 8
        alg = info["nnz_stored"] * (vb + 4) + g.n * m * 16
        if label == "mixed":
            steps, warmup = args.steps, args.warmup
        else:
            steps, warmup = 1, 0
        r = solve_timed(hs, torch, h, nev, m, tol, precond, opts, steps, warmup, "%s %s" % (name, label))
        live = r["phase_ms"][0] / max(1, r["spmm_calls"])
        rep = r["rep"]
        res[label] = {"build_s": build_s, "s_to_tol": r["total"] / steps, "times": r["times"],
                      "iters": int(np.median(r["iters"])), "evals": r["evals"].tolist(),
                      "resnorm_max": float(max(rep.resnorm[:nev])), "spmm_ms_microbench": spmm_ms,
                      "spmm_ms_in_solve": live, "spmm_calls_timed": r["spmm_calls"], "algorithmic_bytes": alg,
                      "spmm_GBs_algorithmic": alg / (live * 1e-3) / 1e9, "device_bytes": info["device_bytes"],
                      "phase_ms_per_solve": phase_split(r["phase_ms"], steps), "p_dropped": rep.p_dropped,
                      "nnz_stored": int(info["nnz_stored"])}
        log("%s %s: %s" % (name, label, json.dumps(res[label])))
        hs.hsym_destroy(h)
        torch.cuda.synchronize()
    ev32, ev64 = np.array(res["mixed"]["evals"]), np.array(res["fp64"]["evals"])
    mixed = res["mixed"]
    times = sorted(mixed["times"])
    cpu = None
    if not args.no_cpu:
        cpu = cpu_baseline_slab(g, cfg, m, nev, tol, precond, mixed["iters"], args.cpu_budget)
        log("cpu baseline: %s" % cpu)
    tf = traffic_file("fp32", m, g.n)
    out = {
        "metric": METRIC,
        "value": args.steps / (mixed["s_to_tol"] * args.steps),
        "unit": "solves/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": 1000.0 * mixed["s_to_tol"],
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32-storage/f64", "data": "synthetic",
        "config": {"workload": "GEN n=%d N=%d seed=%d (CI-shaped upper CSR), LOBPCG nev=%d m=%d tol=%g %s, "
                               "mixed (fp32 storage, fp32 SpMM) vs fp64" % (cfg["n"], cfg["N"], cfg["seed"], nev, m,
                                                                            tol, precond),
                   "n": g.n, "nnz_stored": mixed["nnz_stored"], "block_width": m, "nev": nev, "tol": tol},
        "s_to_tol": mixed["s_to_tol"],
        "p50_s": times[len(times) // 2],
        "p99_s": times[min(len(times) - 1, int(0.99 * len(times)))],
        "iters": mixed["iters"],
        "roofline": {"bound": "hbm", "achieved": mixed["spmm_GBs_algorithmic"], "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": mixed["spmm_GBs_algorithmic"] / HBM_PEAK_GBS,
                     "traffic": measured_traffic(tf, m),
                     "kernel": "spmm_sym fp32 storage m=16 (k_zero_rows + k_spmm_panel)",
                     "launch_ms": mixed["spmm_ms_in_solve"], "launches_timed": mixed["spmm_calls_timed"],
                     "algorithmic_bytes": mixed["algorithmic_bytes"]},
        "cpu_baseline": cpu,
        "mixed_vs_fp64_speedup": res["fp64"]["s_to_tol"] / mixed["s_to_tol"],
        "mixed_vs_fp64_spmm_speedup": res["fp64"]["spmm_ms_in_solve"] / mixed["spmm_ms_in_solve"],
        "max_rel_eval_diff_mixed_vs_fp64": float(np.max(np.abs(ev32 - ev64) / np.abs(ev64))),
        "per_pair_rel_diff": (np.abs(ev32 - ev64) / np.abs(ev64)).tolist(),
        "phase_ms_per_solve": mixed["phase_ms_per_solve"],
        "forms": res,
    }
    print(json.dumps(out))


def cpu_baseline_slab(g, cfg, m, nev, tol, precond, gpu_iters, budget_s, rows=1_000_000):
    """The oracle on a bounded slab of the workload: the principal submatrix
    of the first `rows` rows (same generator, same density).  Oracle LOBPCG
    iterations run for about budget_s seconds; the per-iteration time, which
    grows linearly with n at fixed nonzeros per row, is scaled by n / rows
    and by the GPU's iteration count to a full-solve rate."""
    import oracle
    import hsymgen
    rows = min(rows, g.n)
    rp, ci, v = g.rows(0, rows, np.float64)
    keep = ci < rows
    row_of = np.repeat(np.arange(rows, dtype=np.int64), np.diff(rp))
    rp2 = np.zeros(rows + 1, np.int64)
    np.cumsum(np.bincount(row_of[keep], minlength=rows), out=rp2[1:])
    A = hsymgen.UpperCSR(rows, rp2, np.ascontiguousarray(ci[keep]), np.ascontiguousarray(v[keep]))
    H = oracle.SymMatrix.from_csr(A)
    H.full()
    H.norm1()
    X0 = hsymgen.gauss_block(1, rows, m)
    t = time.perf_counter()
    r = oracle.lobpcg(H, nev, m, tol, X0=X0, precond=precond, maxit=2, keep_history=False)
    dt = time.perf_counter() - t
    per_it = dt / max(1, r.iters)
    its = 2 + int(max(0, budget_s - dt) / max(per_it, 1e-9))
    if its > 2:
        t = time.perf_counter()
        r = oracle.lobpcg(H, nev, m, tol, X0=X0, precond=precond, maxit=its, keep_history=False)
        dt = time.perf_counter() - t
        per_it = dt / max(1, r.iters)
    hi = host_info()
    threads = int(os.environ.get("OMP_NUM_THREADS", hi["cores"]))
    solve_s = per_it * (g.n / rows) * gpu_iters
    return {"value": 1.0 / solve_s, "unit": "solves/s", "cores": min(threads, hi["cores"]), "kind": "oracle",
            "cpu_model": hi["cpu_model"], "ram_GB": hi["ram_GB"],
            "sample": "slab: %d oracle LOBPCG iterations (%s, %.1f s, %.3f s/iteration) on the principal "
                      "submatrix of the first %d rows (%d stored entries), per-iteration time scaled by "
                      "n/rows = %.0f and by the %d iterations of the GPU solve" %
                      (r.iters, precond, dt, per_it, rows, int(rp2[-1]), g.n / rows, gpu_iters)}


def cpu_baseline(A, m, nev, tol, gpu_iters, budget_s):
    """The oracle (as it stands) on the same matrix: LOBPCG iterations are run
    for about budget_s seconds and the per-iteration time is scaled to the
    iteration count of a full solve."""
    import oracle
    import hsymgen
    H = oracle.SymMatrix.from_csr(A)
    H.full()
    H.norm1()
    X0 = hsymgen.gauss_block(1, A.n, m)
    t = time.perf_counter()
    its = 2
    r = oracle.lobpcg(H, nev, m, tol, X0=X0, precond="jacobi", maxit=its, keep_history=False)
    dt = time.perf_counter() - t
    per_it = dt / max(1, r.iters)
    more = int(max(0, budget_s - dt) / max(per_it, 1e-9))
    if more > 0:
        its = min(its + more, gpu_iters)
        t = time.perf_counter()
        r = oracle.lobpcg(H, nev, m, tol, X0=X0, precond="jacobi", maxit=its, keep_history=False)
        dt = time.perf_counter() - t
        per_it = dt / max(1, r.iters)
    threads = int(os.environ.get("OMP_NUM_THREADS", len(os.sched_getaffinity(0))))
    solve_s = per_it * gpu_iters
    return {"value": 1.0 / solve_s, "unit": "solves/s", "cores": threads, "kind": "oracle",
            "sample": "%d oracle LOBPCG iterations (%.1f s, %.3f s/iteration) on the same n=%d matrix, "
                      "scaled to the %d iterations of a full solve" % (r.iters, dt, per_it, A.n, gpu_iters)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None, help="timed steps (default 3 for C3/C4, 5 for C2)")
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--m", type=int, default=16, help="block width of the C2 line (8 or 16)")
    ap.add_argument("--spmm-reps", type=int, default=50)
    ap.add_argument("--cpu-budget", type=float, default=20.0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-extras", action="store_true")
    ap.add_argument("--workload", default="C4", choices=["C2", "C3", "C4"],
                    help="C4 (default: n = 30M, the mixed-vs-fp64 line), C3, or C2 (n = 500k, fp64, "
                         "with the Lanczos, FOM, multi-level and serving extras)")
    ap.add_argument("--spmm-only", action="store_true",
                    help="build the workload's handle and run three SpMMs and the calibration kernel "
                         "(for counter runs)")
    ap.add_argument("--form", default="fp32", choices=["fp32", "fp64"], help="storage of --spmm-only")
    ap.add_argument("--serve-requests", type=int, default=150,
                    help="requests of the request-loop measurement of the C2 line (0: skip)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the library has no multi-GPU path "
              "(run with --gpus 1)", file=sys.stderr)
        sys.exit(2)
    if args.steps is None:
        args.steps = 5 if args.workload == "C2" else 3

    import torch
    import hsymgen
    import paper_1609_01689_amd as hs

    assert torch.cuda.is_available(), "bench.py needs a ROCm GPU"
    if args.spmm_only and args.workload != "C2":
        spmm_only(args, args.workload)
        return
    if args.workload != "C2":
        scale_workload(args, args.workload)
        return
    m, nev, tol = args.m, 8, 1e-8
    cfg = hsymgen.CONFIGS["C2"]
    t = time.perf_counter()
    A = hsymgen.config("C2")
    log("generated C2: n=%d nnz_stored=%d in %.1fs" % (A.n, A.nnz, time.perf_counter() - t))
    t = time.perf_counter()
    M = hs.Matrix(A, storage=hs.HSYM_FP64, geom_m=m)
    torch.cuda.synchronize()
    build_s = time.perf_counter() - t
    info = M.info
    log("handle built in %.2fs: %s" % (build_s, info))

    # --- SpMM roofline (dominant kernel) ---
    spmm_ms = time_spmm(hs, torch, M, m, args.spmm_reps, torch.float64)
    alg = spmm_algorithmic_bytes(A.nnz, A.n, m, 8, 8, 8)
    achieved = alg / (spmm_ms * 1e-3) / 1e9
    log("spmm fp64 m=%d: %.3f ms, %.1f GB/s (%.1f%% of 8 TB/s)" % (m, spmm_ms, achieved, 100 * achieved / HBM_PEAK_GBS))

    calibration_kernel(torch)

    # --- timed LOBPCG solves ---
    opts = hs.default_lobpcg_opts(seed=1, keep_history=0)
    for _ in range(args.warmup):
        hs.lobpcg_solve(M.h, nev, m, tol, precond="jacobi", opts=opts)
    torch.cuda.synchronize()
    times, iters = [], []
    spmm_live_ms, spmm_live_calls = 0.0, 0
    t0 = time.perf_counter()
    for _ in range(args.steps):
        ts = time.perf_counter()
        st, ev, rep = hs.lobpcg_solve(M.h, nev, m, tol, precond="jacobi", opts=opts)
        torch.cuda.synchronize()
        times.append(time.perf_counter() - ts)
        iters.append(rep.iters)
        spmm_live_ms += rep.phase_ms[0]
        spmm_live_calls += rep.spmm_calls
        assert st == hs.HSYM_OK, "solve did not converge"
    torch.cuda.synchronize()
    total = time.perf_counter() - t0
    ms_per_step = 1000.0 * total / args.steps
    # SpMM launch duration inside the timed solves (HIP events on the solve stream)
    live_ms = spmm_live_ms / max(1, spmm_live_calls)
    achieved = alg / (live_ms * 1e-3) / 1e9
    log("spmm inside the solves: %d calls, %.4f ms/call, %.1f GB/s" % (spmm_live_calls, live_ms, achieved))
    log("lobpcg fp64: %.1f ms/solve, iterations %s, rr bisection rounds max %d, evals %s" % (ms_per_step, iters, rep.rr_rounds_max, ev))

    extras = {}
    if not args.no_extras:
        # Lanczos baseline on the same GPU and matrix, on a handle whose tile
        # geometry is built for its single-vector SpMV
        M1 = hs.Matrix(A, storage=hs.HSYM_FP64, geom_m=1)
        t = time.perf_counter()
        stl, evl, repl = hs.lanczos_solve(M1.h, nev, tol, seed=1)
        torch.cuda.synchronize()
        lan_s = time.perf_counter() - t
        extras["lanczos"] = {"s_to_tol": lan_s, "iters": repl.iters, "status": stl,
                             "max_rel_eval_diff_vs_lobpcg": float(np.max(np.abs(evl - ev) / np.abs(ev)))}
        # SpMV (m=1) bandwidth of the Lanczos baseline
        spmv_ms = time_spmm(hs, torch, M1, 1, args.spmm_reps, torch.float64)
        M1.close()
        extras["spmv_fp64"] = {"ms": spmv_ms, "GB/s": spmm_algorithmic_bytes(A.nnz, A.n, 1, 8, 8, 8) / spmv_ms / 1e6}
        # 16-bit tile-local index codes: handle memory against SpMM time
        M16 = hs.Matrix(A, storage=hs.HSYM_FP64, geom_m=m, flags=hs.HSYM_INDEX16)
        i16 = M16.info
        spmm16_ms = time_spmm(hs, torch, M16, m, args.spmm_reps, torch.float64)
        M16.close()
        extras["spmm_index16"] = {"index_bytes": i16["index_bytes"], "handle_GB": i16["device_bytes"] / 1e9,
                                  "handle_GB_index32": M.info["device_bytes"] / 1e9, "ms": spmm16_ms,
                                  "ms_index32": spmm_ms}
        # mixed precision: fp32 storage and SpMM, fp64 everything else
        Mf = hs.Matrix(A, storage=hs.HSYM_FP32, geom_m=m)
        spmm32_ms = time_spmm(hs, torch, Mf, m, args.spmm_reps, torch.float32)
        alg32 = spmm_algorithmic_bytes(A.nnz, A.n, m, 4, 4, 4)
        for tol_m in (1e-6,):
            t = time.perf_counter()
            stm, evm, repm = hs.lobpcg_solve(Mf.h, nev, m, tol_m, precond="jacobi", opts=opts)
            torch.cuda.synchronize()
            mixed_s = time.perf_counter() - t
            t = time.perf_counter()
            st6, ev6, rep6 = hs.lobpcg_solve(M.h, nev, m, tol_m, precond="jacobi", opts=opts)
            torch.cuda.synchronize()
            fp64_s = time.perf_counter() - t
            extras["mixed_vs_fp64_tol1e-6"] = {
                "mixed_s_to_tol": mixed_s, "mixed_iters": repm.iters, "fp64_s_to_tol": fp64_s,
                "fp64_iters": rep6.iters, "speedup": fp64_s / mixed_s,
                "max_rel_eval_err_mixed_vs_fp64": float(np.max(np.abs(evm - ev6) / np.abs(ev6)))}
        extras["spmm_fp32"] = {"ms": spmm32_ms, "GB/s": alg32 / spmm32_ms / 1e6,
                               "frac": alg32 / spmm32_ms / 1e6 / HBM_PEAK_GBS}
        Mf.close()
        # the paper's preconditioner: FOM on the diagonal group tiles
        gst, _ = hsymgen.Generator(A.n, cfg["N"], cfg["seed"]).blocks()
        t = time.perf_counter()
        hs.hsym_attach_group_tiles(M.h, gst, A)
        attach_s = time.perf_counter() - t
        fom = {"attach_s": attach_s}
        for k in (2, 3):
            t = time.perf_counter()
            stf, evf, repf = hs.lobpcg_solve(M.h, nev, m, tol, precond="fom",
                                             opts=hs.default_lobpcg_opts(seed=1, keep_history=0, fom_iters=k))
            torch.cuda.synchronize()
            fom["fom%d" % k] = {"s_to_tol": time.perf_counter() - t, "iters": repf.iters, "status": stf,
                                "max_rel_eval_diff_vs_jacobi": float(np.max(np.abs(evf - ev) / np.abs(ev)))}
        fom["jacobi"] = {"s_to_tol": ms_per_step / 1e3, "iters": int(np.median(iters))}
        extras["fom_tile_preconditioner"] = fom
        # multi-level start block (eq. 12): the level <= 2 space (60% of the
        # rows of this generator) solved to 1e-3, padded, then the full solve
        lv = hsymgen.levels(A.n, cfg["N"], cfg["seed"])
        X0 = torch.zeros((A.n, m), dtype=torch.float64, device="cuda:0")
        t = time.perf_counter()
        sub_its = hs.lobpcg_guess_multilevel(A, lv, [2], X0, m, 1e-3, precond="jacobi", opts=opts)
        torch.cuda.synchronize()
        guess_s = time.perf_counter() - t
        t = time.perf_counter()
        stg, evg, repg = hs.lobpcg_solve(M.h, nev, m, tol, X0=X0, precond="jacobi", opts=opts)
        torch.cuda.synchronize()
        solve_s = time.perf_counter() - t
        extras["multilevel_guess"] = {
            "caps": [2], "sub_tol": 1e-3, "sub_iters": [int(x) for x in sub_its], "guess_s": guess_s,
            "solve_iters": repg.iters, "solve_s": solve_s, "random_start_iters": int(np.median(iters)),
            "random_start_s": ms_per_step / 1e3, "max_rel_eval_diff": float(np.max(np.abs(evg - ev) / np.abs(ev)))}
        del X0
        if args.serve_requests > 0:
            extras["serving"] = serving(hs, torch, args.serve_requests)
        log("extras: %s" % json.dumps(extras))

    cpu = None
    if not args.no_cpu:
        cpu = cpu_baseline(A, m, nev, tol, int(np.median(iters)), args.cpu_budget)
        log("cpu baseline: %s" % cpu)

    times.sort()
    out = {
        "metric": METRIC,
        "value": args.steps / total,
        "unit": "solves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "GEN n=%d N=%d seed=%d (CI-shaped upper CSR, fp64), LOBPCG nev=%d m=%d "
                               "tol=%g jacobi" % (cfg["n"], cfg["N"], cfg["seed"], nev, m, tol),
                   "n": A.n, "nnz_stored": A.nnz, "block_width": m, "nev": nev, "tol": tol},
        "s_to_tol": ms_per_step / 1000.0,
        "p50_s": times[len(times) // 2],
        "p99_s": times[min(len(times) - 1, int(0.99 * len(times)))],
        "iters": int(np.median(iters)),
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": measured_traffic(TRAFFIC_FILE, m),
                     "kernel": "spmm_sym fp64 m=%d (k_zero_rows + k_spmm_panel)" % m,
                     "launch_ms": live_ms, "launches_timed": spmm_live_calls, "algorithmic_bytes": alg,
                     "microbench_ms": spmm_ms},
        "cpu_baseline": cpu,
        "build_s": build_s,
        "extras": extras,
    }
    M.close()
    print(json.dumps(out))


if __name__ == "__main__":
    main()
