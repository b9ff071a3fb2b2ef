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


# ---- the paper's tile preconditioner: FOM on diagonal group tiles ----------

def _krylov_basis(A, b, k):
    """Orthonormal basis of span{b, A b, ..., A^(k-1) b} by Householder QR of
    the (explicit) Krylov matrix, independent of the Arnoldi process."""
    K = np.empty((b.size, k))
    K[:, 0] = b / np.linalg.norm(b)
    for i in range(1, k):
        v = A @ K[:, i - 1]
        K[:, i] = v / np.linalg.norm(v)
    Q, _ = np.linalg.qr(K)
    return Q


def test_fom_full_krylov_space_is_the_exact_solve():
    rng = np.random.default_rng(4)
    for s in (1, 2, 3):
        B = rng.standard_normal((s, s))
        A = B @ B.T + s * np.eye(s)             # SPD, well conditioned
        b = rng.standard_normal(s)
        x = oracle.fom_solve(A, b, 3, 1e-12)
        assert np.allclose(x, np.linalg.solve(A, b), rtol=1e-12, atol=1e-14)


def test_fom_galerkin_condition():
    # k steps: x lies in K_k(A, b) and b - A x is orthogonal to K_k (Saad, Prop. 6.x)
    rng = np.random.default_rng(5)
    s = 40
    B = rng.standard_normal((s, s))
    A = 0.5 * (B + B.T) - 3.0 * np.eye(s)       # symmetric indefinite (a shifted tile)
    b = rng.standard_normal(s)
    for k in (1, 2, 3):
        x = oracle.fom_solve(A, b, k, 1e-12)
        Q = _krylov_basis(A, b, k)
        assert np.linalg.norm(x - Q @ (Q.T @ x)) <= 1e-10 * np.linalg.norm(x)
        assert np.linalg.norm(Q.T @ (b - A @ x)) <= 1e-10 * np.linalg.norm(b)


def test_fom_one_step_is_the_rayleigh_scaling():
    # k = 1: x = (b.b / b.A b) b
    rng = np.random.default_rng(6)
    A = np.diag(rng.uniform(1, 2, 10))
    b = rng.standard_normal(10)
    x = oracle.fom_solve(A, b, 1, 1e-12)
    assert np.allclose(x, (b @ b) / (b @ A @ b) * b, rtol=1e-13)


def test_fom_invariant_space_stops_early():
    # b an eigenvector: K_1 is invariant, the answer is b / lambda whatever k
    A = np.diag([2.0, 3.0, 5.0])
    b = np.array([0.0, 4.0, 0.0])
    for k in (1, 2, 3):
        assert np.allclose(oracle.fom_solve(A, b, k, 1e-12), [0.0, 4.0 / 3.0, 0.0], rtol=1e-14)


def test_fom_tile_apply_uses_the_shifted_tiles(H):
    g = hsymgen.Generator(2000, 40, 1)
    st, _ = g.blocks()
    pre = oracle.Preconditioner("fom", H, groups=st, fom_iters=3)
    assert np.all(np.diff(pre.starts) <= 64) and pre.starts[0] == 0 and pre.starts[-1] == H.n
    R = hsymgen.gauss_block(4, H.n, 3)
    mu = np.array([-3.5, -3.0, 0.5])
    W = pre.apply(R, mu)
    D = H.dense()
    for a, b in zip(pre.starts[:-1], pre.starts[1:]):
        T = D[a:b, a:b]
        for j in range(3):
            A = T - mu[j] * np.eye(b - a)
            Q = _krylov_basis(A, R[a:b, j], min(3, b - a))
            r = R[a:b, j] - A @ W[a:b, j]
            assert np.linalg.norm(Q.T @ r) <= 1e-8 * np.linalg.norm(R[a:b, j])
            # a planted sign error in the shift breaks the Galerkin condition
            Ab = T + mu[j] * np.eye(b - a)
            rb = R[a:b, j] - Ab @ W[a:b, j]
            if j == 0:
                assert np.linalg.norm(_krylov_basis(Ab, R[a:b, j], 3).T @ rb) > 1e-6 * np.linalg.norm(R[a:b, j])
