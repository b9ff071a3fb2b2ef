"""Step-level GPU parity (through the C ABI): block inner products, linear
combinations, Cholesky-QR orthonormalisation, Rayleigh-Ritz and the
preconditioner apply, each against a plain fp64 computation."""
import numpy as np
import pytest

import hsymgen
import oracle

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
import paper_1609_01689_amd as hs  # noqa: E402

U = 2.0 ** -53


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")


@pytest.mark.parametrize("n,m,na,nb", [(10007, 8, 3, 3), (4097, 16, 2, 3), (777, 5, 1, 2), (64, 16, 3, 1),
                                       (3, 1, 1, 1)])
def test_gram(n, m, na, nb):
    A = [hsymgen.gauss_block(10 + i, n, m) for i in range(na)]
    B = [hsymgen.gauss_block(20 + i, n, m) for i in range(nb)]
    G = torch.zeros((na * m, nb * m), dtype=torch.float64, device="cuda:0")
    hs.hsym_kernel_gram([dev(a) for a in A], [dev(b) for b in B], G)
    Ac, Bc = np.hstack(A), np.hstack(B)
    ref = Ac.T @ Bc
    bound = n * U / (1 - n * U) * (np.abs(Ac).T @ np.abs(Bc))
    assert np.all(np.abs(G.cpu().numpy() - ref) <= 2 * bound)
    # fixed reduction order: bitwise reproducible
    G2 = torch.zeros_like(G)
    hs.hsym_kernel_gram([dev(a) for a in A], [dev(b) for b in B], G2)
    assert torch.equal(G, G2)


@pytest.mark.parametrize("n,m,nin,nout", [(5003, 8, 3, 2), (1000, 16, 2, 1), (300, 3, 1, 1)])
def test_lincomb(n, m, nin, nout):
    In = [hsymgen.gauss_block(30 + i, n, m) for i in range(nin)]
    C = hsymgen.gauss_block(40, nin * m, nout * m)
    Out = [torch.zeros((n, m), dtype=torch.float64, device="cuda:0") for _ in range(nout)]
    hs.hsym_kernel_lincomb([dev(a) for a in In], Out, dev(C))
    torch.cuda.synchronize()
    S = np.hstack(In)
    ref = S @ C
    bound = (nin * m) * U * 2 * (np.abs(S) @ np.abs(C))
    for q in range(nout):
        assert np.all(np.abs(Out[q].cpu().numpy() - ref[:, q * m:(q + 1) * m]) <= bound[:, q * m:(q + 1) * m])


def test_lincomb_in_place():
    n, m = 2000, 8
    X = hsymgen.gauss_block(1, n, m)
    C = hsymgen.gauss_block(2, m, m)
    Xd = dev(X)
    hs.hsym_kernel_lincomb([Xd], [Xd], dev(C))
    torch.cuda.synchronize()
    assert np.allclose(Xd.cpu().numpy(), X @ C, rtol=1e-13, atol=1e-13)


def _rr(nblk, m, S, A):
    """Run the Rayleigh-Ritz kernel on the basis S (rows x k) for the
    symmetric A (rows x rows): G = [S^T S | S^T A S]."""
    k = nblk * m
    G = np.hstack([S.T @ S, S.T @ (A @ S)])
    th = torch.zeros(m, dtype=torch.float64, device="cuda:0")
    ev = torch.zeros(k, dtype=torch.float64, device="cuda:0")
    coef = torch.zeros((k, 2 * m), dtype=torch.float64, device="cuda:0")
    dropped = hs.hsym_kernel_rayleigh_ritz(nblk, m, dev(G), th, ev, coef)
    torch.cuda.synchronize()
    return th.cpu().numpy(), ev.cpu().numpy(), coef.cpu().numpy(), dropped


@pytest.mark.parametrize("nblk,m", [(3, 16), (3, 8), (2, 8), (1, 8), (3, 5), (2, 1)])
def test_rayleigh_ritz(nblk, m):
    """Orthonormal basis (S^T S = I): the Ritz pairs of the k x k projected
    matrix against LAPACK, and the search-direction coefficients."""
    k = nblk * m
    A = hsymgen.gauss_block(7 + k, k, k)
    A = A + A.T + np.diag(np.arange(k, dtype=float))
    th, ev, C, dropped = _rr(nblk, m, np.eye(k), 0.5 * (A + A.T))
    assert dropped == 0
    A = 0.5 * (A + A.T)
    lam = np.linalg.eigvalsh(A)
    nA = np.linalg.norm(A, 2)
    assert np.max(np.abs(ev - lam)) <= 50 * k * U * nA
    assert np.max(np.abs(th - lam[:m])) <= 50 * k * U * nA
    CX, CP = C[:, :m], C[:, m:]
    assert np.max(np.abs(A @ CX - CX * lam[None, :m])) <= 100 * k * U * nA
    assert np.max(np.abs(CX.T @ CX - np.eye(m))) <= 100 * k * U
    if nblk > 1:
        assert np.max(np.abs(CP.T @ CP - np.eye(m))) <= 1e-12
        assert np.max(np.abs(CX.T @ CP)) <= 1e-12
        # span{C_X, C_P} contains the W,P-components of C_X (search direction of step 10)
        Y = CX.copy()
        Y[:m] = 0
        Q, _ = np.linalg.qr(np.hstack([CX, CP]))
        assert np.linalg.norm(Y - Q @ (Q.T @ Y)) <= 1e-11 * max(1.0, np.linalg.norm(Y))
    else:
        assert np.all(CP == 0)


@pytest.mark.parametrize("nblk,m,skew", [(3, 16, 1e-3), (3, 8, 0.3), (2, 8, 1e-6), (3, 5, 0.5)])
def test_rayleigh_ritz_measured_basis(nblk, m, skew):
    """A basis S that is not orthonormal (columns perturbed away from an
    orthonormal set by `skew`): the kernel orthonormalises it in coefficient
    space from S^T S (Algorithm 1, step 7), so that S C_X are the Ritz
    vectors of span(S): against LAPACK's generalized eigenproblem
    (S^T A S) c = theta (S^T S) c, with S C_X and S C_P orthonormal, S C_P
    orthogonal to S C_X, and span{S C_X, S C_P} holding the part of S C_X
    outside the first block (step 10)."""
    import scipy.linalg as sla
    k = nblk * m
    rows = 400
    Q, _ = np.linalg.qr(hsymgen.gauss_block(31 + k, rows, k))
    S = Q + skew * hsymgen.gauss_block(32 + k, rows, k)
    B = hsymgen.gauss_block(33 + k, rows, rows)
    A = 0.5 * (B + B.T) + np.diag(np.linspace(-3, 3, rows))
    th, ev, C, dropped = _rr(nblk, m, S, A)
    assert dropped == 0
    Ah, Bh = S.T @ A @ S, S.T @ S
    lam = sla.eigh(0.5 * (Ah + Ah.T), 0.5 * (Bh + Bh.T), eigvals_only=True)
    nA = np.linalg.norm(A, 2)
    kap = np.linalg.cond(Bh)
    assert np.max(np.abs(th - lam[:m])) <= 100 * k * U * nA * kap
    X = S @ C[:, :m]
    P = S @ C[:, m:]
    assert np.max(np.abs(X.T @ X - np.eye(m))) <= 100 * k * U * kap
    R = A @ X - X * th[None, :]
    # Ritz residuals are orthogonal to span(S)
    assert np.max(np.abs(S.T @ R)) <= 100 * k * U * nA * kap * np.linalg.norm(S, 2)
    if nblk > 1:
        assert np.max(np.abs(P.T @ P - np.eye(m))) <= 1e-10 * kap
        assert np.max(np.abs(X.T @ P)) <= 1e-10 * kap
        Q1, _ = np.linalg.qr(S[:, :m])
        Yo = X - Q1 @ (Q1.T @ X)
        Qxp, _ = np.linalg.qr(np.hstack([X, P]))
        assert np.linalg.norm(Yo - Qxp @ (Qxp.T @ Yo)) <= 1e-9 * kap * max(1.0, np.linalg.norm(Yo))


def test_rayleigh_ritz_drops_dependent_p():
    """A third block nearly inside the span of the first two (a pivot of its
    normalised projection below 1e-4) is dropped for the iteration, as the
    oracle drops P: its coefficient rows are zero and the Ritz values are
    those of span[X W]."""
    import scipy.linalg as sla
    m, rows = 8, 300
    Q, _ = np.linalg.qr(hsymgen.gauss_block(41, rows, 2 * m))
    mix = hsymgen.gauss_block(42, 2 * m, m)
    Pn = Q @ mix
    Pn = Pn + 1e-7 * hsymgen.gauss_block(43, rows, m)
    S = np.hstack([Q, Pn])
    B = hsymgen.gauss_block(44, rows, rows)
    A = 0.5 * (B + B.T)
    th, ev, C, dropped = _rr(3, m, S, A)
    assert dropped == 1
    assert np.all(C[2 * m:] == 0)
    lam = np.linalg.eigvalsh(Q.T @ A @ Q)
    assert np.max(np.abs(th - lam[:m])) <= 1e-12 * np.linalg.norm(A, 2)


@pytest.mark.parametrize("nb,m", [(0, 8), (1, 8), (2, 16), (2, 5)])
def test_orthonormalize(nb, m):
    n = 20011
    Bs = []
    if nb:
        Q, _ = np.linalg.qr(hsymgen.gauss_block(3, n, nb * m))
        Bs = [Q[:, i * m:(i + 1) * m] for i in range(nb)]
    V0 = hsymgen.gauss_block(4, n, m) * np.logspace(0, -9, m)[None, :]   # wildly scaled columns
    if nb:
        V0 = V0 + Bs[0] @ hsymgen.gauss_block(5, m, m)
    Vd = dev(V0)
    rep = hs.hsym_kernel_orthonormalize(Vd, [dev(b) for b in Bs], seed=1)
    V = Vd.cpu().numpy()
    assert rep == 0
    Full = np.hstack(Bs + [V])
    assert np.max(np.abs(Full.T @ Full - np.eye(Full.shape[1]))) <= 1e-14 * n ** 0.5 * 10
    # span preserved: V0 lies in span(B, V)
    resid = V0 - Full @ (Full.T @ V0)
    assert np.all(np.linalg.norm(resid, axis=0) <= 1e-9 * np.linalg.norm(V0, axis=0))


def test_orthonormalize_repairs_dependent_columns():
    n, m = 5000, 8
    V0 = hsymgen.gauss_block(6, n, m)
    V0[:, 3] = V0[:, 1]
    Vd = dev(V0)
    rep = hs.hsym_kernel_orthonormalize(Vd, [], seed=2)
    V = Vd.cpu().numpy()
    assert rep >= 1
    assert np.max(np.abs(V.T @ V - np.eye(m))) <= 1e-13


@pytest.mark.parametrize("kind", ["jacobi", "block64"])
def test_precond_apply(kind):
    A = hsymgen.generate(3001, 40, 9)
    H = oracle.SymMatrix.from_csr(A)
    pre = oracle.Preconditioner(kind, H)
    R = hsymgen.gauss_block(8, A.n, 8)
    theta = np.linspace(-3.6, -2.5, 8)
    mu = theta - 2e-3            # shifts inside the spectrum: the guard is exercised too
    M = hs.Matrix(A, block64=(kind == "block64"), geom_m=8)
    Wd = dev(R)
    delta = oracle.GUARD * H.norm1()
    hs.hsym_kernel_precond(M.h, kind, Wd, dev(mu), delta)
    torch.cuda.synchronize()
    ref = pre.apply(R, mu)
    W = Wd.cpu().numpy()
    # the block64 factors differ by algorithm (host QR vs LAPACK) within O(u kappa)
    rt = 1e-12 if kind == "jacobi" else 1e-8
    assert np.linalg.norm(W - ref) <= rt * np.linalg.norm(ref)
    M.close()
