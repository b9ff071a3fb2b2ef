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


@pytest.mark.parametrize("nblk,m", [(3, 16), (3, 8), (2, 8), (1, 8), (3, 5), (2, 1)])
def test_rayleigh_ritz(nblk, m):
    k = nblk * m
    A = hsymgen.gauss_block(7 + k, k, k)
    A = A + A.T + np.diag(np.arange(k, dtype=float))
    th = torch.zeros(m, dtype=torch.float64, device="cuda:0")
    ev = torch.zeros(k, dtype=torch.float64, device="cuda:0")
    coef = torch.zeros((k, 2 * m), dtype=torch.float64, device="cuda:0")
    hs.hsym_kernel_rayleigh_ritz(nblk, m, dev(A), th, ev, coef)
    torch.cuda.synchronize()
    lam = np.linalg.eigvalsh(0.5 * (A + A.T))
    nA = np.linalg.norm(A, 2)
    assert np.max(np.abs(ev.cpu().numpy() - lam)) <= 50 * k * U * nA
    assert np.max(np.abs(th.cpu().numpy() - lam[:m])) <= 50 * k * U * nA
    C = coef.cpu().numpy()
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
