"""Context/step API: several solves advanced together give the same results
as each solve alone (within the stated tolerance)."""
import numpy as np
import pytest

import hsymgen

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
import paper_1609_01689_amd as hs  # noqa: E402


def test_ctx_alone_vs_mix():
    cases = [(2000, 40, 1, 5), (6000, 40, 2, 3), (15000, 60, 3, 8), (3000, 40, 4, 1)]
    mats = [hs.Matrix(hsymgen.generate(n, N, seed), storage=hs.HSYM_FP32, geom_m=8) for n, N, seed, _ in cases]
    tol = 1e-6
    alone = []
    for M, (n, N, seed, nev) in zip(mats, cases):
        st, ev, rep = hs.lobpcg_solve(M.h, nev, 8, tol, opts=hs.default_lobpcg_opts(seed=seed))
        assert st == hs.HSYM_OK
        alone.append(ev)
    ctxs = [hs.lobpcg_ctx_create(M.h, nev, 8, tol, opts=hs.default_lobpcg_opts(seed=seed))
            for M, (n, N, seed, nev) in zip(mats, cases)]
    for _ in range(1000):
        hs.lobpcg_ctx_step(ctxs, iters=3)
        if all(hs.lobpcg_ctx_status(c, nev)[0] for c, (_, _, _, nev) in zip(ctxs, cases)):
            break
    for c, (n, N, seed, nev), ev0 in zip(ctxs, cases, alone):
        done, st, ev, rep = hs.lobpcg_ctx_status(c, nev)
        assert done and st == hs.HSYM_OK
        print("n=%d: alone %s mix %s iters %d" % (n, ev0, ev, rep.iters))
        assert np.max(np.abs(ev - ev0) / np.abs(ev0)) <= 1e-6
        vec = torch.zeros((n, nev), dtype=torch.float64, device="cuda:0")
        hs.lobpcg_ctx_evecs(c, vec)
        assert torch.allclose(vec.norm(dim=0), torch.ones(nev, dtype=torch.float64, device="cuda:0"))
        assert hs.lobpcg_ctx_device_bytes(c) > 0
        hs.lobpcg_ctx_destroy(c)
    for M in mats:
        M.close()
