"""Pins of the preconditioner (eq. 11) and of the Section 4.3 rules."""
import numpy as np
import pytest
import scipy.linalg as sla

import hsymgen
import oracle


@pytest.fixture(scope="module")
def H():
    return oracle.SymMatrix.from_csr(hsymgen.config("C1"))


def test_shift_rules_table():
    theta = np.array([1.0, 2.0, 3.0, 4.0, 5.0])
    rnorm = np.array([0.01, 0.02, 0.5, 0.03, 0.04])
    rho = np.array([0.001, 0.002, 0.5, 0.003, 0.004])       # third pair is far
    mu = oracle.shifts(theta, rnorm, rho)
    # rule 3 for the first two, rule 4 carries mu_2 to every later column
    assert np.allclose(mu, [1 - 0.02, 2 - 0.04, 2 - 0.04, 2 - 0.04, 2 - 0.04])
    rho2 = np.full(5, 1e-3)
    assert np.allclose(oracle.shifts(theta, rnorm, rho2), theta - 2 * rnorm)


def test_rules_1_and_2_skip_preconditioning(H):
    pre = oracle.Preconditioner("jacobi", H)
    R = hsymgen.gauss_block(1, H.n, 4)
    theta = np.arange(4.0)
    rn = np.full(4, 1e-3)
    for it, rho0 in [(1, 1e-3), (3, 1e-3), (4, 0.5)]:
        W, mu = oracle.precondition(pre, R, it, theta, rn, np.array([rho0, 1e-3, 1e-3, 1e-3]))
        assert mu is None and np.array_equal(W, R)
    W, mu = oracle.precondition(pre, R, 4, theta, rn, np.full(4, 1e-3))
    assert mu is not None and not np.array_equal(W, R)


def test_guard():
    g = oracle.guard(np.array([-1.0, -1e-9, 0.0, 1e-9, 2.0]), 1e-3)
    assert np.array_equal(g, [-1.0, -1e-3, 1e-3, 1e-3, 2.0])


def test_jacobi_apply(H):
    pre = oracle.Preconditioner("jacobi", H)
    R = hsymgen.gauss_block(2, H.n, 3)
    mu = np.array([-100.0, -50.0, -20.0])          # far below the spectrum: no guard
    W = pre.apply(R, mu)
    d = H.dense().diagonal()
    for j in range(3):
        assert np.allclose(W[:, j] * (d - mu[j]), R[:, j], rtol=1e-14, atol=0)


def test_block64_apply_solves_shifted_blocks(H):
    pre = oracle.Preconditioner("block64", H)
    R = hsymgen.gauss_block(3, H.n, 3)
    mu = np.array([-100.0, -50.0, -20.0])
    W = pre.apply(R, mu)
    D = H.dense()
    for b0 in range(0, H.n, 64):
        b1 = min(H.n, b0 + 64)
        Hb = D[b0:b1, b0:b1]
        for j in range(3):
            ref = sla.solve(Hb - mu[j] * np.eye(b1 - b0), R[b0:b1, j], assume_a="sym")
            assert np.allclose(W[b0:b1, j], ref, rtol=1e-11, atol=1e-13)
