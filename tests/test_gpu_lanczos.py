"""GPU parity of lanczos_solve (through the C ABI) against LAPACK and the oracle."""
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


def test_lanczos_c1():
    A = hsymgen.config("C1")
    lam = np.linalg.eigvalsh(dense_of(A))
    dev = torch.device("cuda:0")
    M = hs.Matrix(A, geom_m=1)
    v0 = hsymgen.gauss_vector(1, A.n)
    ev = torch.zeros((A.n, 5), dtype=torch.float64, device=dev)
    st, evals, rep = hs.lanczos_solve(M.h, 5, 1e-8, v0=torch.from_numpy(v0).to(dev), evecs=ev)
    torch.cuda.synchronize()
    print("lanczos C1: status", st, "iters", rep.iters, "time", rep.seconds)
    assert st == hs.HSYM_OK and rep.converged
    assert np.max(np.abs(evals - lam[:5]) / np.abs(lam[:5])) <= 1e-8
    ref = oracle.lanczos(oracle.SymMatrix.from_csr(A), 5, 1e-8, v0=v0)
    assert rep.iters == ref.iters          # same check schedule, same convergence point
    X = ev.cpu().numpy()
    H = oracle.SymMatrix.from_csr(A)
    R = H.spmm(X) - X * evals[None, :]
    assert np.max(np.linalg.norm(R, axis=0)) / H.norm1() <= 1e-7
    M.close()


def test_lanczos_agrees_with_lobpcg():
    A = hsymgen.generate(40000, 150, 6)
    dev = torch.device("cuda:0")
    M = hs.Matrix(A, geom_m=16)
    st1, e1, r1 = hs.lanczos_solve(M.h, 8, 1e-9, seed=2)
    st2, e2, r2 = hs.lobpcg_solve(M.h, 8, 12, 1e-9, precond="jacobi", opts=hs.default_lobpcg_opts(seed=3))
    print("lanczos iters", r1.iters, "lobpcg iters", r2.iters)
    assert st1 == hs.HSYM_OK and st2 == hs.HSYM_OK
    assert np.max(np.abs(e1 - e2) / np.abs(e2)) <= 1e-8
    assert r2.iters < r1.iters
    M.close()
