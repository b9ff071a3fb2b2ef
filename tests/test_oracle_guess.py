"""Pins of the oracle's multi-level start block (Section 3.3.1, eq. 12).

Checked against mathematics that fixes it, not against the oracle itself:
  - the zero padding: rows outside the smaller space are exactly 0;
  - eq. 12's identities for an exact eigenvector x1 of H11 (dense LAPACK):
    the Rayleigh quotient of the padded x on H is theta, the residual
    H x - theta x vanishes on the smaller space and equals H21 x1 outside it,
    and ||r|| / (||H|| ||x||) <= ||H21|| / ||H|| (2-norms, dense);
  - Cauchy interlacing: theta_j(H11) >= lambda_j(H);
  - a deliberately wrong padding (a row shift) breaks the identities;
  - the recursive guess equals the eigenvectors of the last smaller space
    (subspace angle), and the full solve from it reaches LAPACK's
    eigenvalues in fewer iterations than from a Gaussian block.
"""
import numpy as np
import pytest
import scipy.linalg as sla

import hsymgen
import oracle


@pytest.fixture(scope="module")
def c1():
    A = hsymgen.config("C1")
    H = oracle.SymMatrix.from_csr(A)
    L = hsymgen.levels(2000, 40, 1)
    return H, L, H.dense()


def test_levels_follow_the_diagonal(c1):
    H, L, D = c1
    # generator recipe: H_ii = 10 q + U(0, 1)
    assert np.array_equal(np.floor(np.diag(D) / 10.0).astype(np.int32), L)


def test_principal_submatrix_is_the_dense_block(c1):
    H, L, D = c1
    rows = np.flatnonzero(L <= 2)
    H11 = oracle.principal_submatrix(H, rows)
    assert np.array_equal(H11.dense(), D[np.ix_(rows, rows)])


@pytest.mark.parametrize("cap", [1, 2, 3])
def test_eq12_identities(c1, cap):
    H, L, D = c1
    rows = np.flatnonzero(L <= cap)
    out = np.flatnonzero(L > cap)
    H11 = D[np.ix_(rows, rows)]
    H21 = D[np.ix_(out, rows)]
    theta, X1 = sla.eigh(H11)
    k = 6
    X0 = oracle.pad_with_zeros(X1[:, :k], rows, H.n)
    assert np.all(X0[out] == 0.0)
    R = D @ X0 - X0 * theta[:k]
    nH = np.linalg.norm(D, 2)
    eps = np.linalg.norm(H21, 2) / nH
    for j in range(k):
        x = X0[:, j]
        assert abs(x @ D @ x - theta[j]) <= 1e-12 * nH
        assert np.linalg.norm(R[rows, j]) <= 1e-11 * nH
        assert np.allclose(R[out, j], H21 @ X1[:, j], atol=1e-12 * nH)
        assert np.linalg.norm(R[:, j]) / (nH * np.linalg.norm(x)) <= eps * (1 + 1e-12)
    lam = np.linalg.eigvalsh(D)
    assert np.all(theta[:k] >= lam[:k] - 1e-12 * nH)


def test_wrong_padding_breaks_the_identities(c1):
    H, L, D = c1
    rows = np.flatnonzero(L <= 2)
    theta, X1 = sla.eigh(D[np.ix_(rows, rows)])
    bad = np.zeros((H.n, 1))
    bad[np.minimum(rows + 1, H.n - 1), 0] = X1[:, 0]       # a planted one-row shift
    x = bad[:, 0]
    assert abs(x @ D @ x / (x @ x) - theta[0]) > 1e-3


def test_recursive_guess_spans_the_last_space(c1):
    H, L, D = c1
    m = 8
    X0, its = oracle.multilevel_guess(H, L, [2, 3], m, 1e-10)
    rows = np.flatnonzero(L <= 3)
    assert np.all(X0[np.flatnonzero(L > 3)] == 0.0)
    _, V = sla.eigh(D[np.ix_(rows, rows)])
    # principal angles between span(X0 on the space) and the m lowest eigenvectors
    Q, _ = np.linalg.qr(X0[rows])
    s = np.linalg.svd(V[:, :m].T @ Q, compute_uv=False)
    assert np.min(s) >= 1 - 1e-8
    assert len(its) == 2 and all(i > 0 for i in its)


def test_full_solve_from_guess_is_shorter(c1):
    H, L, D = c1
    X0, _ = oracle.multilevel_guess(H, L, [2, 3], 8, 1e-6)
    lam = np.linalg.eigvalsh(D)[:5]
    r0 = oracle.lobpcg(H, 5, 8, 1e-8, seed=0, keep_history=False)
    r1 = oracle.lobpcg(H, 5, 8, 1e-8, X0=X0, seed=0, keep_history=False)
    assert r0.converged and r1.converged
    assert np.max(np.abs(r1.evals - lam) / np.abs(lam)) <= 1e-8
    assert r1.iters < r0.iters
