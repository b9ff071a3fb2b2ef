"""Device request loop (hsym_serve): every request of a staggered trace
finishes, each result equals the same request solved alone, and the memory
budget bounds what is in flight."""
import numpy as np
import pytest
import scipy.sparse as sp

import hsymgen

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
import paper_1609_01689_amd as hs  # noqa: E402


def make_requests(k, seed=0, nmax=40000):
    rng = np.random.default_rng(seed)
    reqs = []
    t = 0.0
    for r in range(k):
        n = int(round(10 ** rng.uniform(3, np.log10(nmax))))
        A = hsymgen.generate(n, 40, 1000 + r)
        t += rng.exponential(0.01)
        reqs.append({"csr": A, "storage": hs.HSYM_FP32, "nev": int(rng.integers(1, 9)), "block_width": 8,
                     "precond": "jacobi", "tol": 1e-6, "seed": 1000 + r, "arrival_s": t})
    return reqs


def test_serve_trace_matches_alone():
    reqs = make_requests(12)
    res, rep = hs.hsym_serve(reqs)
    print("serve report", rep)
    assert rep["max_active_seen"] >= 2
    for q, r in zip(reqs, res):
        assert r["status"] == hs.HSYM_OK, r
        assert r["finish_s"] >= r["arrival_s"]
        M = hs.Matrix(q["csr"], storage=q["storage"], geom_m=8)
        st, ev, rep1 = hs.lobpcg_solve(M.h, q["nev"], 8, q["tol"], precond="jacobi",
                                       opts=hs.default_lobpcg_opts(seed=q["seed"]))
        M.close()
        assert st == hs.HSYM_OK
        # alone vs mix: the same solve.  The SpMM's transposed half is summed
        # with workgroup-local atomics, so two runs agree to rounding only;
        # at a converged relative residual tol that moves Ritz values by
        # O((tol ||H||)^2 / gap) and can shift the iteration count when
        # nev = block_width (no guard vectors)
        assert np.max(np.abs(r["evals"] - ev) / np.abs(ev)) <= 1e-7, (r["evals"], ev)
    # the smallest request against LAPACK
    small = min(range(len(reqs)), key=lambda i: reqs[i]["csr"].n)
    A = reqs[small]["csr"]
    U = sp.csr_matrix((A.values.astype(np.float64), A.colind, A.rowptr), shape=(A.n, A.n))
    if A.n <= 4000:
        lam = np.linalg.eigvalsh((U + U.T - sp.diags(U.diagonal())).toarray())
        nev = reqs[small]["nev"]
        # fp32 storage: eigenvalues of the rounded matrix, within its perturbation
        assert np.max(np.abs(res[small]["evals"] - lam[:nev])) <= 1e-5 * np.abs(lam).max()


def estimate(q):
    """The loop's admission estimate of a request (fp32 storage)."""
    A = q["csr"]
    return int(1.3 * A.nnz * 8) + A.n * 16 + A.n * q["block_width"] * 8 * 16 + (8 << 20)


def test_serve_budget_limits_inflight():
    reqs = make_requests(8, seed=1, nmax=20000)
    for q in reqs:
        q["arrival_s"] = 0.0                      # all at once: the budget alone limits admission
    _, free = hs.hsym_serve(reqs)
    largest = max(estimate(q) for q in reqs)
    budget = max(largest, int(0.6 * free["peak_reserved_bytes"]))
    res, rep = hs.hsym_serve(reqs, budget_bytes=budget)
    print("unconstrained", free, "budget", budget, rep)
    assert all(r["status"] == hs.HSYM_OK for r in res), [r["status"] for r in res]
    assert rep["peak_reserved_bytes"] <= budget
    # what each request held on the device (handle + solver context) stays
    # within the estimate it was admitted on
    for r, q in zip(res, reqs):
        print("n=%d held %d estimate %d" % (q["csr"].n, r["device_bytes"], estimate(q)))
        assert 0 < r["device_bytes"] <= estimate(q)
    if budget < free["peak_reserved_bytes"]:
        # fewer requests fit at once than without a budget
        assert rep["peak_reserved_bytes"] < free["peak_reserved_bytes"]
    # a budget below the largest request rejects it at admission, the rest run
    res2, _ = hs.hsym_serve(reqs, budget_bytes=largest - 1)
    big = [estimate(q) >= largest for q in reqs]
    assert all((r["status"] == hs.HSYM_E_OUT_OF_MEMORY) == b for r, b in zip(res2, big))
