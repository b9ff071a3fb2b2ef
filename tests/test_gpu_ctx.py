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


def test_graph_replays_match_eager():
    """Steady-state iterations recorded once as HIP graphs and replayed: every
    replayed iteration is checked against the same solve run launch by launch
    (residual history; the SpMM's workgroup-local atomics make runs agree to
    rounding), with eager work and synchronisation of another context between
    the replays, and the final eigenpairs agree."""
    A = hsymgen.generate(6000, 40, 7)
    B = hsymgen.generate(3000, 40, 8)
    MA = hs.Matrix(A, geom_m=8)
    MB = hs.Matrix(B, geom_m=8)
    tol = 1e-9
    eager = hs.lobpcg_ctx_create(MA.h, 5, 8, tol, opts=hs.default_lobpcg_opts(seed=4, graph=0))
    graph = hs.lobpcg_ctx_create(MA.h, 5, 8, tol, opts=hs.default_lobpcg_opts(seed=4, graph=1))
    other = hs.lobpcg_ctx_create(MB.h, 3, 8, tol, opts=hs.default_lobpcg_opts(seed=5))
    for _ in range(1000):
        hs.lobpcg_ctx_step([eager], iters=1)
        hs.lobpcg_ctx_step([graph], iters=1)
        hs.lobpcg_ctx_step([other], iters=1)          # eager work in between
        torch.cuda.synchronize()
        de = hs.lobpcg_ctx_status(eager, 5)
        dg = hs.lobpcg_ctx_status(graph, 5)
        if de[0] and dg[0]:
            break
    _, st_e, ev_e, rep_e = hs.lobpcg_ctx_status(eager, 5)
    _, st_g, ev_g, rep_g = hs.lobpcg_ctx_status(graph, 5)
    assert st_e == hs.HSYM_OK and st_g == hs.HSYM_OK
    k = min(rep_e.history_len, rep_g.history_len, 25)
    he = np.array(rep_e.history[:k])
    hg = np.array(rep_g.history[:k])
    print("graph vs eager: iterations %d / %d, history %s / %s" % (rep_g.iters, rep_e.iters, hg[:6], he[:6]))
    assert k > 5
    assert np.all(np.abs(hg - he) <= 1e-6 * he)
    assert np.max(np.abs(ev_g - ev_e) / np.abs(ev_e)) <= 1e-10
    for c in (eager, graph, other):
        hs.lobpcg_ctx_destroy(c)
    MA.close()
    MB.close()
