"""GPU multi-level start block (Section 3.3.1, eq. 12) through the C ABI,
against the oracle's, and the full solve it starts."""
import numpy as np
import pytest
import scipy.linalg as sla

import hsymgen
import oracle

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
import paper_1609_01689_amd as hs  # noqa: E402


def _guess(A, L, caps, m, tol, **kw):
    X0 = torch.zeros((A.n, m), dtype=torch.float64, device="cuda:0")
    its = hs.lobpcg_guess_multilevel(A, L, caps, X0, m, tol, **kw)
    torch.cuda.synchronize()
    return X0, its


def test_guess_matches_oracle_c1():
    A = hsymgen.config("C1")
    L = hsymgen.levels(2000, 40, 1)
    m = 8
    X0, its = _guess(A, L, [2, 3], m, 1e-10)
    Xg = X0.cpu().numpy()
    H = oracle.SymMatrix.from_csr(A)
    Xo, its_o = oracle.multilevel_guess(H, L, [2, 3], m, 1e-10)
    print("sub-solve iterations gpu", its, "oracle", its_o)
    out = np.flatnonzero(L > 3)
    rows = np.flatnonzero(L <= 3)
    assert np.all(Xg[out] == 0.0)                       # eq. 12: exact zeros
    # same subspace as the oracle's and as LAPACK's m lowest eigenvectors of H11
    D = H.dense()
    _, V = sla.eigh(D[np.ix_(rows, rows)])
    for X in (Xg, Xo):
        Q, _ = np.linalg.qr(X[rows])
        assert np.min(np.linalg.svd(V[:, :m].T @ Q, compute_uv=False)) >= 1 - 1e-8
    # column by column: the Rayleigh quotients (the sub-eigenvalues, eq. 12)
    for j in range(m):
        qg = Xg[:, j] @ D @ Xg[:, j] / (Xg[:, j] @ Xg[:, j])
        qo = Xo[:, j] @ D @ Xo[:, j] / (Xo[:, j] @ Xo[:, j])
        assert abs(qg - qo) <= 1e-9 * abs(qo)


def test_solve_from_guess_c1():
    A = hsymgen.config("C1")
    L = hsymgen.levels(2000, 40, 1)
    X0, _ = _guess(A, L, [2, 3], 8, 1e-6)
    M = hs.Matrix(A, geom_m=8)
    st0, ev0, r0 = hs.lobpcg_solve(M.h, 5, 8, 1e-8, opts=hs.default_lobpcg_opts(seed=0))
    st1, ev1, r1 = hs.lobpcg_solve(M.h, 5, 8, 1e-8, X0=X0, opts=hs.default_lobpcg_opts(seed=0))
    M.close()
    lam = np.linalg.eigvalsh(oracle.SymMatrix.from_csr(A).dense())[:5]
    print("iterations from a Gaussian block %d, from the multi-level guess %d" % (r0.iters, r1.iters))
    assert st0 == hs.HSYM_OK and st1 == hs.HSYM_OK
    assert np.max(np.abs(ev1 - lam) / np.abs(lam)) <= 1e-8
    assert r1.iters < r0.iters


def test_guess_larger_mixed_storage():
    n, N, seed = 100_000, 100, 21
    A = hsymgen.generate(n, N, seed)
    L = hsymgen.levels(n, N, seed)
    X0, its = _guess(A, L, [1, 2], 16, 1e-6, storage=hs.HSYM_FP32)
    Xg = X0.cpu().numpy()
    assert np.all(Xg[L > 2] == 0.0)
    M = hs.Matrix(A, geom_m=16)
    st0, ev0, r0 = hs.lobpcg_solve(M.h, 8, 16, 1e-8, opts=hs.default_lobpcg_opts(seed=1))
    st1, ev1, r1 = hs.lobpcg_solve(M.h, 8, 16, 1e-8, X0=X0, opts=hs.default_lobpcg_opts(seed=1))
    M.close()
    print("n=%d: sub-solves %s; iterations %d from Gaussian, %d from the guess" % (n, its, r0.iters, r1.iters))
    assert st0 == hs.HSYM_OK and st1 == hs.HSYM_OK
    assert np.max(np.abs(ev1 - ev0) / np.abs(ev0)) <= 1e-9
    assert r1.iters < r0.iters


def test_guess_rejects_bad_caps():
    A = hsymgen.config("C1")
    L = hsymgen.levels(2000, 40, 1)
    X0 = torch.zeros((A.n, 8), dtype=torch.float64, device="cuda:0")
    for caps in ([3, 2], [-1]):
        with pytest.raises(hs.HsymError) as e:
            hs.lobpcg_guess_multilevel(A, L, caps, X0, 8, 1e-6)
        assert e.value.status == hs.HSYM_E_INVALID_ARG
