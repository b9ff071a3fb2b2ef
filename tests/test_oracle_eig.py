"""Pins of the oracle's eigensolvers: LAPACK dense spectra, closed-form
spectra, block-diagonal spectra, residual bounds and the invariants of
Algorithm 1 (orthonormal X, X^T R = 0, monotone Ritz values, interlacing)."""
import numpy as np
import pytest
import scipy.linalg as sla
import scipy.sparse as sp

import hsymgen
import oracle


def dense_of(A):
    U = sp.csr_matrix((A.values.astype(np.float64), A.colind, A.rowptr), shape=(A.n, A.n))
    return (U + U.T - sp.diags(U.diagonal())).toarray()


@pytest.fixture(scope="module")
def c1():
    A = hsymgen.config("C1")
    lam = np.linalg.eigvalsh(dense_of(A))
    return A, lam


@pytest.mark.parametrize("pc", ["none", "jacobi", "block64"])
def test_lobpcg_c1_matches_eigh(c1, pc):
    A, lam = c1
    H = oracle.SymMatrix.from_csr(A)
    r = oracle.lobpcg(H, 5, 8, 1e-8, X0=hsymgen.gauss_block(1, A.n, 8), precond=pc)
    assert r.converged
    assert np.max(np.abs(r.evals - lam[:5]) / np.abs(lam[:5])) <= 1e-8
    # invariants at exit: X orthonormal, residual orthogonal to X
    X = r.X
    assert np.max(np.abs(X.T @ X - np.eye(8))) < 1e-12
    R = H.spmm(X) - X * r.history[-1][0][None, :]
    assert np.max(np.abs(X.T @ R)) < 1e-10 * H.norm1()
    # each Ritz value is within ||r_j|| of an eigenvalue (symmetric residual bound)
    for j in range(5):
        rj = np.linalg.norm(R[:, j])
        assert np.min(np.abs(lam - r.evals[j])) <= rj * (1 + 1e-6) + 1e-12


def test_ritz_values_monotone_and_interlaced(c1):
    A, lam = c1
    H = oracle.SymMatrix.from_csr(A)
    r = oracle.lobpcg(H, 5, 8, 1e-8, X0=hsymgen.gauss_block(3, A.n, 8), precond="jacobi")
    th = np.array([h[0] for h in r.history])
    tol = 1e-10 * H.norm1()
    assert np.all(np.diff(th, axis=0) <= tol)          # trace minimisation, eq. 6
    assert np.all(th >= lam[None, :8] - tol)           # Cauchy interlacing


def test_preconditioning_cuts_iterations(c1):
    """Table 2 / Fig. 6 claim, qualitative: preconditioning reduces iterations."""
    A, _ = c1
    H = oracle.SymMatrix.from_csr(A)
    X0 = hsymgen.gauss_block(5, A.n, 8)
    it = {pc: oracle.lobpcg(H, 5, 8, 1e-8, X0=X0, precond=pc).iters
          for pc in ("none", "jacobi", "block64")}
    assert it["jacobi"] < it["none"] and it["block64"] < it["none"]


def test_lobpcg_laplacian_closed_form():
    n = 120
    L = oracle.SymMatrix.from_csr(hsymgen.laplacian_1d(n))
    r = oracle.lobpcg(L, 3, 6, 1e-9, X0=hsymgen.gauss_block(2, n, 6), precond="none")
    lam = 2 - 2 * np.cos(np.arange(1, 4) * np.pi / (n + 1))
    assert r.converged
    assert np.max(np.abs(r.evals - lam) / lam) < 1e-8
    # locally optimal three-term search: far fewer steps than n (a steepest
    # descent on this kappa ~ 6e3 problem needs thousands)
    assert r.iters < 200


def test_lobpcg_blockdiag_union_of_block_spectra():
    g = hsymgen.Generator(4000, 40, 21, variant="blockdiag")
    A = g.matrix()
    st, _ = g.blocks()
    D = dense_of(A)
    spec = np.sort(np.concatenate([np.linalg.eigvalsh(D[a:b, a:b]) for a, b in zip(st[:-1], st[1:])]))
    H = oracle.SymMatrix.from_csr(A)
    r = oracle.lobpcg(H, 4, 8, 1e-9, X0=hsymgen.gauss_block(4, A.n, 8), precond="jacobi")
    assert r.converged
    assert np.max(np.abs(r.evals - spec[:4]) / np.abs(spec[:4])) < 1e-8


def test_lobpcg_rejects_bad_sizes(c1):
    A, _ = c1
    H = oracle.SymMatrix.from_csr(A)
    with pytest.raises(ValueError):
        oracle.lobpcg(H, 9, 8, 1e-8)


def test_lobpcg_not_converged_reports(c1):
    A, _ = c1
    H = oracle.SymMatrix.from_csr(A)
    r = oracle.lobpcg(H, 5, 8, 1e-12, maxit=3, X0=hsymgen.gauss_block(1, A.n, 8))
    assert not r.converged and r.iters == 3


def test_lanczos_matches_eigh(c1):
    A, lam = c1
    H = oracle.SymMatrix.from_csr(A)
    r = oracle.lanczos(H, 5, 1e-8, v0=hsymgen.gauss_vector(1, A.n), keep_basis=True)
    assert r.converged
    assert np.max(np.abs(r.evals - lam[:5]) / np.abs(lam[:5])) <= 1e-8
    V = r.V
    k = V.shape[0]
    assert np.max(np.abs(V @ V.T - np.eye(k))) < 1e-12
    T = V @ dense_of(A) @ V.T
    Tref = np.diag(r.alpha) + np.diag(r.beta[:-1], 1) + np.diag(r.beta[:-1], -1)
    assert np.max(np.abs(T - Tref)) < 1e-10 * H.norm1()
    assert k % 10 == 0          # stopped on a scheduled check


def test_lanczos_check_schedule():
    """Footnote 7: checks every 10 iterations to 100, then every 20 to 200,
    every 40 to 400, ..."""
    checks = [j for j in range(1, 900) if j % oracle.lanczos_check_interval(j) == 0]
    assert checks[:10] == list(range(10, 101, 10))
    assert checks[10:15] == [120, 140, 160, 180, 200]
    assert checks[15:20] == [240, 280, 320, 360, 400]
    assert checks[20:22] == [480, 560]


def test_lobpcg_vs_lanczos_iteration_claim(c1):
    """Section 5.2 claim, qualitative: LOBPCG needs fewer iterations than
    Lanczos but more vector applications of H."""
    A, _ = c1
    H = oracle.SymMatrix.from_csr(A)
    lo = oracle.lobpcg(H, 5, 8, 1e-8, X0=hsymgen.gauss_block(1, A.n, 8), precond="jacobi")
    la = oracle.lanczos(H, 5, 1e-8, v0=hsymgen.gauss_vector(1, A.n))
    assert lo.iters < la.iters
    assert 8 * lo.iters > la.iters


def test_ritz_values_bounded_when_the_basis_nearly_fills_the_space():
    """n = 50 with m = 16: [X W P] spans 48 of 50 dimensions and P turns
    nearly dependent.  Rayleigh-Ritz on an orthonormal basis gives Ritz values
    theta_j >= lambda_j (Cauchy interlacing); a P orthonormalised through a
    tiny QR pivot (with its updated AP) breaks that bound and the iteration
    diverges (Ritz values below -1e3 within 10 iterations).  With both
    orthogonalisation passes the basis stays orthonormal to working precision,
    so the bound holds to 1e-12 ||H||_1 and the solve converges."""
    n = 50
    A = hsymgen.generate(n, 20, 90)
    H = oracle.SymMatrix.from_csr(A)
    lam = np.linalg.eigvalsh(H.dense())
    r = oracle.lobpcg(H, 4, 16, 1e-9, X0=hsymgen.gauss_block(7, n, 16), maxit=60, keep_history=True)
    slack = 1e-12 * H.norm1()
    for theta, _ in r.history:
        assert np.all(theta[:16] >= lam[:16] - slack)
    assert r.converged
    assert np.max(np.abs(r.evals - lam[:4]) / np.abs(lam[:4])) <= 1e-12


def test_lobpcg_fom_c1_matches_eigh(c1):
    """The paper's tile preconditioner (FOM on the diagonal group tiles,
    Section 3.2 end, Section 4.3) inside the oracle's LOBPCG reaches the
    LAPACK spectrum of C1, like the other preconditioners."""
    A, lam = c1
    g = hsymgen.Generator(A.n, 40, 1)
    st, _ = g.blocks()
    H = oracle.SymMatrix.from_csr(A)
    for k in (2, 3):
        r = oracle.lobpcg(H, 5, 8, 1e-8, X0=hsymgen.gauss_block(1, A.n, 8), precond="fom",
                          groups=st, fom_iters=k)
        assert r.converged
        assert np.max(np.abs(r.evals - lam[:5]) / np.abs(lam[:5])) <= 1e-8
        assert np.max(np.abs(r.X.T @ r.X - np.eye(8))) < 1e-12


def test_w_repair_branch_runs_and_reaches_eigh():
    """Algorithm 1 step 7 with rank loss: on n = 30, m = 8 the preconditioned
    residual block turns deficient once the guard columns converge, so the
    oracle replaces its deficient columns (w_replaced > 0) and still reaches
    the LAPACK spectrum with an orthonormal X."""
    n = 30
    A = hsymgen.generate(n, 10, 0)
    H = oracle.SymMatrix.from_csr(A)
    lam = np.linalg.eigvalsh(H.dense())
    for xs in range(3):
        r = oracle.lobpcg(H, 3, 8, 1e-9, X0=hsymgen.gauss_block(xs, n, 8), maxit=100)
        assert r.w_replaced > 0
        assert r.converged
        assert np.max(np.abs(r.evals - lam[:3]) / np.abs(lam[:3])) <= 1e-12
        assert np.max(np.abs(r.X.T @ r.X - np.eye(8))) < 1e-12


def test_basis_stays_orthonormal_when_it_nearly_fills_the_space():
    """n = 50, m = 16: [X W P] spans 48 of 50 dimensions.  A W pivot of about
    1e-8 passes the rank test, and its QR amplifies the rounding left along X
    by 1 / pivot; without the second projection pass X drifts from
    orthonormality (1e-7) and the iteration freezes short of tol (or, for
    some start blocks, diverges).  Every start block must converge to LAPACK
    with X orthonormal to working precision."""
    n = 50
    A = hsymgen.generate(n, 20, 90)
    H = oracle.SymMatrix.from_csr(A)
    lam = np.linalg.eigvalsh(H.dense())
    for xs in range(5):
        r = oracle.lobpcg(H, 4, 16, 1e-9, X0=hsymgen.gauss_block(xs, n, 16), maxit=100)
        assert r.converged, xs
        assert r.w_replaced > 0
        assert np.max(np.abs(r.evals - lam[:4]) / np.abs(lam[:4])) <= 1e-12
        assert np.max(np.abs(r.X.T @ r.X - np.eye(16))) < 1e-12
