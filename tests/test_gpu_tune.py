"""Tile-shape autotuner and explicit panel geometry (through the C ABI):
the tuner times every candidate that fits, returns the fastest, and a handle
built with any explicit geometry gives the oracle's H X; the request loop
with autotuning solves every request as it is solved alone."""
import numpy as np
import pytest

import hsymgen
import oracle

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
import paper_1609_01689_amd as hs  # noqa: E402
from test_gpu_serve import make_requests  # noqa: E402

U64 = 2.0 ** -53


def _spmm(A, X, flags, storage=hs.HSYM_FP64):
    dev = torch.device("cuda:0")
    h = hs.hsym_create(A.n, A.rowptr, A.colind, A.values, storage, flags)
    Xd = torch.from_numpy(X).to(dev)
    Yd = torch.empty_like(Xd)
    hs.spmm_sym(h, Xd, Yd)
    torch.cuda.synchronize()
    info = hs.hsym_info(h)
    hs.hsym_destroy(h)
    return Yd.cpu().numpy(), info


def _check(A, X, Y):
    H = oracle.SymMatrix(A.n, A.rowptr, A.colind, A.values.astype(np.float64))
    ref = H.spmm(X)
    Habs = oracle.SymMatrix(A.n, A.rowptr, A.colind, np.abs(A.values.astype(np.float64)))
    # terms in a full row: its stored entries plus the stored entries of its column
    k = int(np.max(np.diff(A.rowptr) + np.bincount(A.colind, minlength=A.n))) + 1
    bound = (k * U64 / (1 - k * U64)) * Habs.spmm(np.abs(X))
    assert np.all(np.abs(Y - ref) <= bound + 1e-300)


@pytest.mark.parametrize("r64,lc", [(1, 3), (4, 5), (8, 7), (12, 6), (16, 6)])
def test_explicit_geometry_parity(r64, lc):
    A = hsymgen.generate(30_000, 60, 11)
    X = hsymgen.gauss_block(12, A.n, 8)
    Y, info = _spmm(A, X, hs.HSYM_GEOM_M(8) | hs.HSYM_GEOM_PANEL(r64, lc))
    assert (info["panel_rows"], info["chunk_cols"]) == (64 * r64, 1 << lc)
    _check(A, X, Y)


def test_explicit_geometry_rejected():
    A = hsymgen.config("C1")
    with pytest.raises(hs.HsymError) as e:
        hs.hsym_create(A.n, A.rowptr, A.colind, A.values, hs.HSYM_FP64, hs.HSYM_GEOM_PANEL(4, 9))
    assert e.value.status == hs.HSYM_E_INVALID_ARG
    # fits at m = 8 but not at m = 16: the SpMM refuses it
    h = hs.hsym_create(A.n, A.rowptr, A.colind, A.values, hs.HSYM_FP64,
                       hs.HSYM_GEOM_M(8) | hs.HSYM_GEOM_PANEL(16, 6))
    X = torch.zeros((A.n, 16), dtype=torch.float64, device="cuda:0")
    with pytest.raises(hs.HsymError) as e:
        hs.spmm_sym(h, X, torch.empty_like(X))
    assert e.value.status == hs.HSYM_E_UNSUPPORTED
    hs.hsym_destroy(h)


@pytest.mark.parametrize("storage,m", [(hs.HSYM_FP64, 16), (hs.HSYM_FP32, 8)])
def test_autotune_picks_fastest_and_is_correct(storage, m):
    A = hsymgen.generate(200_000, 120, 5)
    flags, table = hs.hsym_autotune_geometry(A.n, A.rowptr, A.colind, A.values, storage, m, sample_rows=100_000)
    print("candidates (R, C, ms):", table)
    timed = [t for t in table if t[2] > 0]
    assert len(timed) >= 3
    R, C, ms = min(timed, key=lambda t: t[2])
    assert flags == hs.HSYM_GEOM_M(m) | hs.HSYM_GEOM_PANEL(R // 64, C.bit_length() - 1)
    # every candidate fits the LDS at width m: an fp64 accumulator and an X
    # row in the arithmetic precision per panel and chunk row
    Mr = 1 << (m - 1).bit_length()
    sa = 8 if storage == hs.HSYM_FP64 else 4
    for R_, C_, _ in table:
        assert (R_ + C_) * Mr * (8 + sa) <= 160 * 1024
    X = hsymgen.gauss_block(13, A.n, m)
    if storage == hs.HSYM_FP32:
        X = X.astype(np.float32).astype(np.float64)
    Y, info = _spmm(A, X, flags, storage)
    assert (info["panel_rows"], info["chunk_cols"]) == (R, C)
    if storage == hs.HSYM_FP64:
        _check(A, X, Y)
    else:
        # fp32 arithmetic on the fp32 operator and the fp32 block
        v32 = A.values.astype(np.float32).astype(np.float64)
        H = oracle.SymMatrix(A.n, A.rowptr, A.colind, v32)
        ref = H.spmm(X)
        Habs = oracle.SymMatrix(A.n, A.rowptr, A.colind, np.abs(v32))
        k = int(np.max(np.diff(A.rowptr) + np.bincount(A.colind, minlength=A.n))) + 1
        u32 = 2.0 ** -24
        assert np.all(np.abs(Y - ref) <= (k * u32 / (1 - k * u32)) * Habs.spmm(np.abs(X)) + 1e-300)


def test_autotune_rejects_bad_input():
    A = hsymgen.config("C1")
    with pytest.raises(hs.HsymError) as e:
        hs.hsym_autotune_geometry(A.n, A.rowptr, A.colind, A.values, hs.HSYM_FP64, 17)
    assert e.value.status == hs.HSYM_E_INVALID_ARG
    rp = A.rowptr.copy()
    rp[5] = rp[6] + 1
    with pytest.raises(hs.HsymError) as e:
        hs.hsym_autotune_geometry(A.n, rp, A.colind, A.values, hs.HSYM_FP64, 8)
    assert e.value.status == hs.HSYM_E_INVALID_ARG


def test_serve_with_autotune_matches_alone():
    reqs = make_requests(8, seed=3, nmax=30000)
    res, rep = hs.hsym_serve(reqs, autotune=True)
    print("serve report", rep)
    assert rep["tuned_classes"] >= 1
    for q, r in zip(reqs, res):
        assert r["status"] == hs.HSYM_OK, r
        M = hs.Matrix(q["csr"], storage=q["storage"], geom_m=8)
        st, ev, _ = hs.lobpcg_solve(M.h, q["nev"], 8, q["tol"], precond="jacobi",
                                    opts=hs.default_lobpcg_opts(seed=q["seed"]))
        M.close()
        assert st == hs.HSYM_OK
        assert np.max(np.abs(r["evals"] - ev) / np.abs(ev)) <= 1e-7, (r["evals"], ev)
