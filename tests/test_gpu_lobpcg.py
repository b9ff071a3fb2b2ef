"""GPU parity of lobpcg_solve (through the C ABI) against the CPU oracle,
LAPACK and closed-form spectra."""
import numpy as np
import pytest
import scipy.sparse as sp

import hsymgen
import oracle

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
import paper_1609_01689_amd as hs  # noqa: E402


def dense_of(A):
    U = sp.csr_matrix((A.values.astype(np.float64), A.colind, A.rowptr), shape=(A.n, A.n))
    return (U + U.T - sp.diags(U.diagonal())).toarray()


def solve(A, nev, m, tol, precond="jacobi", storage=hs.HSYM_FP64, X0=None, seed=0, maxit=1000):
    dev = torch.device("cuda:0")
    M = hs.Matrix(A, storage=storage, block64=(precond == "block64"), geom_m=m)
    X0d = None if X0 is None else torch.from_numpy(np.ascontiguousarray(X0)).to(dev)
    ev = torch.zeros((A.n, nev), dtype=torch.float64, device=dev)
    opts = hs.default_lobpcg_opts(seed=seed, maxit=maxit)
    st, evals, rep = hs.lobpcg_solve(M.h, nev, m, tol, X0=X0d, precond=precond, opts=opts, evecs=ev)
    torch.cuda.synchronize()
    vecs = ev.cpu().numpy()
    norm1 = M.info["norm1"]
    M.close()
    print("n=%d m=%d nev=%d %s storage=%d: status %d iters %d spmm %d time %.3fs" %
          (A.n, m, nev, precond, storage, st, rep.iters, rep.spmm_calls, rep.seconds), flush=True)
    return st, evals, vecs, rep, norm1


def certify(A, evals, vecs, tol_rel):
    """fp64 residuals of the returned pairs with the oracle's SpMM."""
    H = oracle.SymMatrix.from_csr(A)
    R = H.spmm(vecs) - vecs * evals[None, :]
    rho = np.linalg.norm(R, axis=0) / H.norm1()
    nrm = np.linalg.norm(vecs, axis=0)
    assert np.allclose(nrm, 1.0, atol=1e-10)
    # sign convention: largest-magnitude entry positive
    idx = np.argmax(np.abs(vecs), axis=0)
    assert np.all(vecs[idx, np.arange(vecs.shape[1])] > 0)
    assert np.max(rho) <= tol_rel, rho
    return rho


@pytest.fixture(scope="module")
def c1():
    A = hsymgen.config("C1")
    return A, np.linalg.eigvalsh(dense_of(A))


@pytest.mark.parametrize("precond", ["none", "jacobi", "block64"])
def test_lobpcg_c1_fp64(c1, precond):
    A, lam = c1
    X0 = hsymgen.gauss_block(1, A.n, 8)
    st, evals, vecs, rep, _ = solve(A, 5, 8, 1e-8, precond=precond, X0=X0)
    assert st == hs.HSYM_OK and rep.converged
    assert np.max(np.abs(evals - lam[:5]) / np.abs(lam[:5])) <= 1e-8
    certify(A, evals, vecs, 1.5e-8)
    # iteration count of the oracle on the same start block, same algorithm
    ref = oracle.lobpcg(oracle.SymMatrix.from_csr(A), 5, 8, 1e-8, X0=X0, precond=precond)
    print("oracle iters", ref.iters, "gpu iters", rep.iters)
    assert abs(rep.iters - ref.iters) <= max(3, 0.2 * ref.iters)


def test_lobpcg_c1_seeded_start(c1):
    A, lam = c1
    st, evals, vecs, rep, _ = solve(A, 5, 8, 1e-8, seed=17)
    assert st == hs.HSYM_OK
    assert np.max(np.abs(evals - lam[:5]) / np.abs(lam[:5])) <= 1e-8


def test_lobpcg_c1_mixed(c1):
    A, lam = c1
    st, evals, vecs, rep, _ = solve(A, 5, 8, 1e-6, storage=hs.HSYM_FP32, X0=hsymgen.gauss_block(1, A.n, 8))
    assert st == hs.HSYM_OK
    err = np.abs(evals - lam[:5]) / np.abs(lam[:5])
    print("mixed C1 eigenvalue errors", err)
    assert np.max(err) <= 1e-6


def test_lobpcg_mixed_weyl_certificate():
    """The mixed form (fp32 storage and SpMM) on an n = 200,000 matrix of the
    benchmark's shape: its eigenvalues are those of H32 = fp64(fp32(H)), so
    by Weyl's inequality |lambda_i(H32) - lambda_i(H)| <= ||H32 - H||_2 <=
    ||H32 - H||_1, computed exactly here from the stored entries.  With the
    residual bound (an eigenvalue lies within ||H v - theta v|| of every
    Ritz pair, v of unit norm), measured in fp64 against H32 for the mixed
    pairs and against H for the fp64 pairs, the certificate is
    |theta_mixed - theta_fp64| <= ||E||_1 + ||r_mixed|| + ||r_fp64||."""
    A = hsymgen.generate(200_000, 300, 6)
    A32 = hsymgen.UpperCSR(A.n, A.rowptr, A.colind, A.values.astype(np.float32))
    E = A32.values.astype(np.float64) - A.values
    rows = np.repeat(np.arange(A.n), np.diff(A.rowptr))
    offd = A.colind != rows
    colsum = np.bincount(rows, weights=np.abs(E), minlength=A.n) + \
        np.bincount(A.colind[offd], weights=np.abs(E[offd]), minlength=A.n)
    normE = float(colsum.max())
    H = oracle.SymMatrix.from_csr(A)
    H32 = oracle.SymMatrix.from_csr(hsymgen.UpperCSR(A.n, A.rowptr, A.colind, A32.values.astype(np.float64)))
    nrm = H.norm1()
    X0 = hsymgen.gauss_block(9, A.n, 16)
    st32, ev32, V32, rep32, _ = solve(A32, 8, 16, 1e-6, storage=hs.HSYM_FP32, X0=X0)
    st64, ev64, V64, rep64, _ = solve(A, 8, 16, 1e-8, X0=X0)
    assert st32 == hs.HSYM_OK and st64 == hs.HSYM_OK
    r32 = np.linalg.norm(H32.spmm(V32) - V32 * ev32[None, :], axis=0)
    r64 = np.linalg.norm(H.spmm(V64) - V64 * ev64[None, :], axis=0)
    bound = normE + r32 + r64
    diff = np.abs(ev32 - ev64)
    print("||E||_1 = %.3e (2^-24 ||H||_1 = %.3e); |theta32 - theta64| = %s; bound %s" %
          (normE, 2.0 ** -24 * nrm, diff, bound), flush=True)
    assert normE <= 2.0 ** -24 * nrm
    assert np.all(diff <= bound)
    assert np.max(r32) <= 5e-6 * nrm     # fp32 products in the computed residual: a few 1e-6
    assert np.max(diff / np.abs(ev64)) <= 1e-6


def test_lobpcg_blockdiag_union():
    g = hsymgen.Generator(6000, 40, 21, variant="blockdiag")
    A = g.matrix()
    st_, _ = g.blocks()
    D = dense_of(A)
    spec = np.sort(np.concatenate([np.linalg.eigvalsh(D[a:b, a:b]) for a, b in zip(st_[:-1], st_[1:])]))
    st, evals, vecs, rep, _ = solve(A, 4, 8, 1e-9)
    assert st == hs.HSYM_OK
    assert np.max(np.abs(evals - spec[:4]) / np.abs(spec[:4])) < 1e-8


def test_lobpcg_laplacian():
    n = 400
    A = hsymgen.laplacian_1d(n)
    st, evals, vecs, rep, _ = solve(A, 3, 6, 1e-9, precond="none", X0=hsymgen.gauss_block(2, n, 6), maxit=3000)
    lam = 2 - 2 * np.cos(np.arange(1, 4) * np.pi / (n + 1))
    assert st == hs.HSYM_OK
    assert np.max(np.abs(evals - lam) / lam) < 1e-8


@pytest.mark.parametrize("m,nev", [(16, 10), (12, 8), (5, 3)])
def test_lobpcg_block_widths(m, nev):
    A = hsymgen.generate(20000, 100, 5)
    H = oracle.SymMatrix.from_csr(A)
    X0 = hsymgen.gauss_block(3, A.n, m)
    st, evals, vecs, rep, _ = solve(A, nev, m, 1e-8, X0=X0)
    assert st == hs.HSYM_OK
    ref = oracle.lobpcg(H, nev, m, 1e-8, X0=X0, precond="jacobi")
    assert ref.converged
    assert np.max(np.abs(evals - ref.evals) / np.abs(ref.evals)) <= 1e-8
    certify(A, evals, vecs, 1.5e-8)


def test_lobpcg_not_converged_status(c1):
    A, _ = c1
    st, evals, vecs, rep, _ = solve(A, 5, 8, 1e-12, maxit=4, X0=hsymgen.gauss_block(1, A.n, 8))
    assert st == hs.HSYM_NOT_CONVERGED and rep.iters == 4
    assert np.all(np.isfinite(evals))


def test_lobpcg_rank_deficient_start(c1):
    """Duplicate columns in X0: the start block is repaired with random columns."""
    A, lam = c1
    X0 = hsymgen.gauss_block(1, A.n, 8)
    X0[:, 5] = X0[:, 2]
    st, evals, vecs, rep, _ = solve(A, 5, 8, 1e-8, X0=X0)
    assert st == hs.HSYM_OK and rep.w_replaced >= 1
    assert np.max(np.abs(evals - lam[:5]) / np.abs(lam[:5])) <= 1e-8


def test_lobpcg_invalid_args(c1):
    A, _ = c1
    M = hs.Matrix(A)
    for nev, m, tol in [(9, 8, 1e-8), (0, 8, 1e-8), (5, 17, 1e-8), (5, 8, 0.0)]:
        with pytest.raises(hs.HsymError) as e:
            hs.lobpcg_solve(M.h, nev, m, tol)
        assert e.value.status == hs.HSYM_E_INVALID_ARG
    with pytest.raises(hs.HsymError):
        hs.lobpcg_solve(M.h, 5, 8, 1e-8, precond="block64")   # factors not built
    M.close()


def test_lobpcg_graph_on_null_and_own_stream(c1):
    """opts.graph replays the steady-state phases as HIP graphs on a stream
    the caller owns, and runs eagerly on the null stream (which cannot be
    captured); all three solves converge to the same pairs."""
    A, lam = c1
    M = hs.Matrix(A, geom_m=8)
    out = []
    st_own = torch.cuda.Stream()
    for graph, stream in ((0, None), (1, None), (1, st_own)):
        opts = hs.default_lobpcg_opts(seed=3, graph=graph)
        s, ev, rep = hs.lobpcg_solve(M.h, 5, 8, 1e-8, opts=opts, stream=stream)
        torch.cuda.synchronize()
        assert s == hs.HSYM_OK
        assert np.max(np.abs(ev - lam[:5]) / np.abs(lam[:5])) <= 1e-8
        out.append(rep.iters)
    M.close()
    print("iterations (eager, graph on the null stream, graph on an own stream):", out)
    assert max(out) - min(out) <= 2


@pytest.mark.parametrize("n", [48, 50, 70, 130])
def test_lobpcg_m16_tiny_n(n):
    """Block width 16 on n = 3m and barely above: one partial per Gram,
    ragged 64-row tiles in the fused update + Gram and Jacobi + Gram passes,
    and (n = 48, 50) a basis that fills the space, where W columns are
    replaced and the coefficient-space P keeps the basis orthonormal."""
    A = hsymgen.generate(n, 20, 40 + n)
    lam = np.linalg.eigvalsh(dense_of(A))
    X0 = hsymgen.gauss_block(7, n, 16)
    st, evals, vecs, rep, _ = solve(A, 4, 16, 1e-9, X0=X0, maxit=500)
    assert st == hs.HSYM_OK
    assert np.max(np.abs(evals - lam[:4]) / np.abs(lam[:4])) <= 1e-8
    certify(A, evals, vecs, 2e-9)


@pytest.mark.parametrize("precond", ["jacobi", "block64"])
def test_lobpcg_phase_timers(precond):
    """opts.timers: the per-phase device times of Section 5.2 (Fig. 7) are
    filled, each phase that ran has time, the device phases fit inside the
    solve's wall time, and the solve is the same as without timers."""
    A = hsymgen.generate(40_000, 60, 12)
    dev = torch.device("cuda:0")
    M = hs.Matrix(A, block64=(precond == "block64"), geom_m=8)
    out = {}
    for timers in (0, 1):
        st, ev, rep = hs.lobpcg_solve(M.h, 5, 8, 1e-8, precond=precond,
                                      opts=hs.default_lobpcg_opts(seed=4, timers=timers))
        torch.cuda.synchronize()
        assert st == hs.HSYM_OK
        out[timers] = (ev, rep)
    M.close()
    ev0, rep0 = out[0]
    ev1, rep1 = out[1]
    ph = np.array(rep1.phase_ms[:8])
    print("phases (ms):", ph, "wall %.1f ms, iterations %d/%d" % (1e3 * rep1.seconds, rep0.iters, rep1.iters))
    assert np.all(np.array(rep0.phase_ms[1:8]) == 0.0)
    assert np.all(ph[:6] > 0.0) and ph[7] > 0.0
    assert ph[0] + ph[1:6].sum() + ph[7] <= 1e3 * rep1.seconds * 1.05
    assert abs(rep1.iters - rep0.iters) <= 2
    assert np.max(np.abs(ev1 - ev0) / np.abs(ev0)) <= 1e-10


def test_lobpcg_c2_bench_configuration():
    """The solve the benchmark times (n = 500,000, about 300 nonzeros per full
    row, fp64, m = 16, nev = 8, tol 1e-8, Jacobi) at full size:
      - against the oracle's LOBPCG from the same start block: eigenvalues to
        1e-8 relative, iteration counts by the C1 rule;
      - certified with the oracle's fp64 SpMM: residual norms within the
        stopping rule, orthonormal eigenvectors, Rayleigh quotients equal to
        the returned eigenvalues, and the Kato-Temple bound
        |theta - lambda| <= ||r||^2 / delta, delta the distance from theta to
        the rest of the spectrum bounded below from the Ritz values and their
        residuals (theta_j - theta_{j-1} - ||r_{j-1}|| below, the next Ritz
        value of the block above: Ritz values are upper bounds);
      - the same eigenvalues from Lanczos on the same matrix (another method)."""
    A = hsymgen.config("C2")
    dev = torch.device("cuda:0")
    M = hs.Matrix(A, geom_m=16)
    X0 = hsymgen.gauss_block(1, A.n, 16)
    V = torch.zeros((A.n, 8), dtype=torch.float64, device=dev)
    st, evals, rep = hs.lobpcg_solve(M.h, 8, 16, 1e-8, X0=torch.from_numpy(X0).to(dev), precond="jacobi",
                                     opts=hs.default_lobpcg_opts(seed=1), evecs=V)
    VL = torch.zeros((A.n, 8), dtype=torch.float64, device=dev)
    st2, e2, rep2 = hs.lanczos_solve(M.h, 8, 1e-8, seed=2, evecs=VL)
    torch.cuda.synchronize()
    M.close()
    print("C2 lobpcg: status %d iters %d (%.3fs); lanczos: status %d iters %d (%.3fs)"
          % (st, rep.iters, rep.seconds, st2, rep2.iters, rep2.seconds), flush=True)
    assert st == hs.HSYM_OK and rep.converged
    assert st2 == hs.HSYM_OK and rep2.converged
    H = oracle.SymMatrix.from_csr(A)
    nrm = H.norm1()
    X = V.cpu().numpy()
    HX = H.spmm(X)
    R = HX - X * evals[None, :]
    rn = np.linalg.norm(R, axis=0)
    rho = rn / nrm
    G = X.T @ X
    q = np.einsum("ij,ij->j", X, HX)
    print("residuals / |H|_1", rho, "orthonormality %.1e" % np.max(np.abs(G - np.eye(8))),
          "rayleigh %.1e" % (np.max(np.abs(q - evals)) / nrm), flush=True)
    assert np.max(rho) <= 1.5e-8
    assert np.max(np.abs(G - np.eye(8))) <= 1e-10
    assert np.max(np.abs(q - evals)) <= 1e-12 * nrm
    # Kato-Temple: the nearest other eigenvalue below lies within ||r_{j-1}||
    # of theta_{j-1}; above, the (j+1)-th Ritz value of the block bounds it
    theta = np.array(rep.theta[:16])
    ktb = []
    for j in range(8):
        below = evals[j] - (evals[j - 1] + rn[j - 1]) if j > 0 else np.inf
        above = theta[j + 1] - evals[j]
        delta = min(below, above)
        assert delta > 0
        ktb.append(rn[j] ** 2 / delta)
    ktb = np.array(ktb)
    print("Kato-Temple bounds / |lambda|", ktb / np.abs(evals), flush=True)
    assert np.max(ktb / np.abs(evals)) <= 1e-8
    # the oracle from the same start block (about a minute on 16 host cores)
    ref = oracle.lobpcg(H, 8, 16, 1e-8, X0=X0, precond="jacobi", keep_history=False)
    print("oracle: converged %s, %d iterations (GPU %d), %.1fs" % (ref.converged, ref.iters, rep.iters,
                                                                   ref.seconds), flush=True)
    assert ref.converged
    assert np.max(np.abs(evals - ref.evals) / np.abs(ref.evals)) <= 1e-8
    assert abs(rep.iters - ref.iters) <= max(3, 0.2 * ref.iters)
    XL = VL.cpu().numpy()
    rl = np.linalg.norm(H.spmm(XL) - XL * e2[None, :], axis=0) / nrm
    print("lanczos residuals / |H|_1", rl, "eigenvalue agreement %.1e" % np.max(np.abs(evals - e2) / np.abs(e2)))
    assert np.max(rl) <= 1e-7
    assert np.all(np.diff(evals) >= 0)
    assert np.max(np.abs(evals - e2) / np.abs(e2)) <= 1e-8


@pytest.mark.parametrize("rep_", range(5))
def test_lobpcg_nearly_full_basis_seed0(rep_):
    """A basis of 24 columns in 30 dimensions from start seed 0.  The solve
    once stalled at a residual of about 5e-5 in some runs: after a near-threshold
    Cholesky pivot of W, [X P] lost orthonormality (to 1e-4) and the
    coefficient-space P, which assumed an orthonormal basis, kept it there.
    The Rayleigh-Ritz step now measures S^T S and orthonormalises the basis in
    coefficient space, so the solve converges in every run (5 repeats: the
    order of the SpMM's sums differs from run to run)."""
    A = hsymgen.generate(30, 12, 63)
    lam = np.linalg.eigvalsh(dense_of(A))
    st, evals, vecs, rep, _ = solve(A, 3, 8, 1e-9, seed=0, maxit=400)
    assert st == hs.HSYM_OK
    assert np.max(np.abs(evals - lam[:3]) / np.abs(lam[:3])) <= 1e-8
