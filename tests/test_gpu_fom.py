"""The paper's preconditioner on the GPU (end of Section 3.2, Section 4.3):
diagonal group tiles, FOM per tile and right-hand side, against the oracle,
and LOBPCG with it against LAPACK and the oracle."""
import numpy as np
import pytest

import hsymgen
import oracle

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
import paper_1609_01689_amd as hs  # noqa: E402


def dev(a):
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda:0")


def _setup(n, N, seed, m=8):
    A = hsymgen.generate(n, N, seed)
    st, _ = hsymgen.Generator(n, N, seed).blocks()
    M = hs.Matrix(A, geom_m=m)
    hs.hsym_attach_group_tiles(M.h, st, A)
    return A, st, M


@pytest.mark.parametrize("m", [1, 5, 8, 16])
def test_fom_apply_matches_oracle(m):
    A, st, M = _setup(3001, 40, 9, m)
    H = oracle.SymMatrix.from_csr(A)
    pre = oracle.Preconditioner("fom", H, groups=st, fom_iters=3)
    R = hsymgen.gauss_block(8, A.n, m)
    mu = np.linspace(-3.6, -2.5, m) - 2e-3           # inside the spectrum: pivots near zero occur
    delta = oracle.GUARD * H.norm1()
    Wd = dev(R)
    hs.hsym_kernel_precond(M.h, "fom", Wd, dev(mu), delta)
    torch.cuda.synchronize()
    W = Wd.cpu().numpy()
    ref = pre.apply(R, mu)
    err = np.linalg.norm(W - ref) / np.linalg.norm(ref)
    print("m=%d: relative difference %.2e" % (m, err))
    assert err <= 1e-10
    M.close()


def test_lobpcg_with_fom_c1():
    A, st, M = _setup(2000, 40, 1)
    H = oracle.SymMatrix.from_csr(A)
    lam = np.linalg.eigvalsh(H.dense())[:5]
    s, ev, rep = hs.lobpcg_solve(M.h, 5, 8, 1e-8, precond="fom", opts=hs.default_lobpcg_opts(seed=0))
    ro = oracle.lobpcg(H, 5, 8, 1e-8, precond="fom", groups=st, keep_history=False)
    sj, evj, repj = hs.lobpcg_solve(M.h, 5, 8, 1e-8, precond="jacobi", opts=hs.default_lobpcg_opts(seed=0))
    print("iterations: fom %d (oracle %d), jacobi %d" % (rep.iters, ro.iters, repj.iters))
    assert s == hs.HSYM_OK and ro.converged
    assert np.max(np.abs(ev - lam) / np.abs(lam)) <= 1e-8
    assert abs(rep.iters - ro.iters) <= 2
    assert rep.iters < repj.iters
    M.close()


def test_fom_iters_option_and_errors():
    A, st, M = _setup(4000, 40, 3)
    its = []
    for k in (1, 2, 3, 4):
        s, ev, rep = hs.lobpcg_solve(M.h, 4, 8, 1e-8, precond="fom", opts=hs.default_lobpcg_opts(seed=1, fom_iters=k))
        assert s == hs.HSYM_OK
        its.append(rep.iters)
    print("iterations for 1..4 FOM steps:", its)
    with pytest.raises(hs.HsymError) as e:
        hs.lobpcg_solve(M.h, 4, 8, 1e-8, precond="fom", opts=hs.default_lobpcg_opts(fom_iters=5))
    assert e.value.status == hs.HSYM_E_INVALID_ARG
    # a handle without tiles
    M2 = hs.Matrix(A, geom_m=8)
    with pytest.raises(hs.HsymError) as e:
        hs.lobpcg_solve(M2.h, 4, 8, 1e-8, precond="fom")
    assert e.value.status == hs.HSYM_E_INVALID_ARG
    # bad boundaries
    bad = st.copy()
    bad[-1] = A.n - 1
    with pytest.raises(hs.HsymError) as e:
        hs.hsym_attach_group_tiles(M2.h, bad, A)
    assert e.value.status == hs.HSYM_E_INVALID_ARG
    M2.close()
    M.close()
