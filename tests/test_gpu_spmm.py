"""GPU parity of spmm_sym against the CPU oracle (through the C ABI)."""
import numpy as np
import pytest

import hsymgen
import oracle

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
import paper_1609_01689_amd as hs  # noqa: E402

U64 = 2.0 ** -53
U32 = 2.0 ** -24


def _dev():
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    return torch.device("cuda:0")


def _run(A, X, storage=hs.HSYM_FP64, geom_m=16, ldpad=0, f32=False):
    dev = _dev()
    M = hs.Matrix(A, storage=storage, geom_m=geom_m)
    n, m = X.shape
    if f32:
        Xd = torch.zeros((n, m + ldpad), dtype=torch.float32, device=dev)
        Xd[:, :m] = torch.from_numpy(X.astype(np.float32))
        Yd = torch.full((n, m + ldpad), 7.0, dtype=torch.float32, device=dev)
        hs.spmm_sym_f32(M.h, Xd[:, :m], Yd[:, :m])
    else:
        Xd = torch.zeros((n, m + ldpad), dtype=torch.float64, device=dev)
        Xd[:, :m] = torch.from_numpy(X)
        Yd = torch.full((n, m + ldpad), 7.0, dtype=torch.float64, device=dev)
        hs.spmm_sym(M.h, Xd[:, :m], Yd[:, :m])
    torch.cuda.synchronize()
    Y = Yd[:, :m].cpu().numpy().astype(np.float64)
    if ldpad:
        assert torch.all(Yd[:, m:] == 7.0), "padding columns of Y were written"
    info = M.info
    M.close()
    return Y, info


def _abs_bound(H, X, k, u):
    """Componentwise forward-error bound gamma_k (|H| |X|) (Higham, Thm 3.5)."""
    Habs = oracle.SymMatrix(H.n, H.rowptr, H.colind, np.abs(H.values))
    return (k * u / (1 - k * u)) * Habs.spmm(np.abs(X))


@pytest.mark.parametrize("m", [1, 5, 8, 16])
def test_spmm_fp64_c1(m):
    A = hsymgen.config("C1")
    H = oracle.SymMatrix.from_csr(A)
    X = hsymgen.gauss_block(10 + m, A.n, m)
    Y, info = _run(A, X)
    Yref = H.spmm(X)
    assert np.linalg.norm(Y - Yref) <= 1e-12 * np.linalg.norm(Yref)
    k = int(np.diff(H.full()[0]).max()) + 1
    assert np.all(np.abs(Y - Yref) <= 2 * _abs_bound(H, X, k, U64) + 1e-300)
    assert abs(info["norm1"] - H.norm1()) <= 1e-12 * H.norm1()
    assert info["nnz_stored"] == A.nnz


def test_spmm_fp64_ragged_and_ld():
    # n not a multiple of any tile size, several panels, leading dimension > m
    A = hsymgen.generate(7001, 120, 33)
    H = oracle.SymMatrix.from_csr(A)
    X = hsymgen.gauss_block(5, A.n, 12)
    Y, info = _run(A, X, ldpad=3)
    assert info["npanels"] >= 3
    Yref = H.spmm(X)
    assert np.linalg.norm(Y - Yref) <= 1e-12 * np.linalg.norm(Yref)


@pytest.mark.parametrize("geom_m,m", [(1, 1), (8, 8), (16, 8), (8, 4), (4, 2), (1, 2), (2, 4), (4, 8)])
def test_spmm_geometries(geom_m, m):
    A = hsymgen.generate(20000, 200, 44)
    H = oracle.SymMatrix.from_csr(A)
    X = hsymgen.gauss_block(6, A.n, m)
    Y, info = _run(A, X, geom_m=geom_m)
    Yref = H.spmm(X)
    assert np.linalg.norm(Y - Yref) <= 1e-12 * np.linalg.norm(Yref)


def test_spmm_uniform_window_variant():
    # partner tiles anywhere above the diagonal: many external chunks per panel
    A = hsymgen.generate(12000, 60, 8, variant="uniform")
    H = oracle.SymMatrix.from_csr(A)
    X = hsymgen.gauss_block(7, A.n, 16)
    Y, _ = _run(A, X)
    Yref = H.spmm(X)
    assert np.linalg.norm(Y - Yref) <= 1e-12 * np.linalg.norm(Yref)


def test_spmm_edge_cases():
    # 1x1, diagonal-only, missing diagonal entries, a row with no entries
    one = hsymgen.UpperCSR(1, np.array([0, 1]), np.array([0], np.int32), np.array([3.0]))
    Y, _ = _run(one, np.array([[2.0, -1.0]]))
    assert np.array_equal(Y, [[6.0, -3.0]])
    n = 300
    rp = np.arange(n + 1, dtype=np.int64)
    diag = hsymgen.UpperCSR(n, rp, np.arange(n, dtype=np.int32), np.linspace(1, 2, n))
    X = hsymgen.gauss_block(1, n, 4)
    Y, _ = _run(diag, X)
    assert np.allclose(Y, X * np.linspace(1, 2, n)[:, None], rtol=1e-15, atol=0)
    # strictly upper pairs only, no diagonal, last rows empty
    rows = np.array([0, 0, 5, 100, 150])
    cols = np.array([1, 299, 200, 101, 151], np.int32)
    vals = np.array([1.0, -2.0, 0.5, 4.0, 3.0])
    rp = np.zeros(n + 1, np.int64)
    np.add.at(rp, rows + 1, 1)
    rp = np.cumsum(rp)
    A = hsymgen.UpperCSR(n, rp, cols, vals)
    Y, _ = _run(A, X)
    Yref = oracle.SymMatrix.from_csr(A).spmm(X)
    assert np.allclose(Y, Yref, rtol=1e-15, atol=1e-15)


def test_spmm_fp32_storage():
    """The mixed form: fp32 values, X staged in fp32, products and run sums in
    fp32 (run sums added across runs in fp64).  Against the fp64 oracle the
    error is the rounding of H and X plus an fp32 sum of at most k terms:
    gamma_{k+2}(u32) |H||X| (plus one more rounding for fp32 output)."""
    A = hsymgen.config("C1")
    H = oracle.SymMatrix.from_csr(A)
    X = hsymgen.gauss_block(3, A.n, 16)
    k = int(np.diff(H.full()[0]).max()) + 1
    for f32 in (False, True):
        Y, info = _run(A, X, storage=hs.HSYM_FP32, f32=f32)
        Yref = H.spmm(X)
        assert np.all(np.abs(Y - Yref) <= _abs_bound(H, X, k + 3, U32))
        assert np.linalg.norm(Y - Yref) <= 1e-5 * np.linalg.norm(Yref)
        # and the error is that of fp32 arithmetic, not of fp64: the
        # fp64 result on the fp32-rounded operator is clearly closer
        assert np.linalg.norm(Y - Yref) > 1e-9 * np.linalg.norm(Yref)


def test_spmm_c2_size():
    """Full C2 size (n=500k, ~300 nnz/row) in the geometry the bench times."""
    A = hsymgen.config("C2")
    H = oracle.SymMatrix.from_csr(A)
    for m in (8, 16):
        X = hsymgen.gauss_block(2, A.n, m)
        Y, info = _run(A, X, geom_m=m)
        Yref = H.spmm(X)
        assert np.linalg.norm(Y - Yref) <= 1e-12 * np.linalg.norm(Yref)
        print("C2 m=%d info %s" % (m, info), flush=True)


def test_invalid_csr_rejected():
    _dev()
    bad = [
        (3, [0, 1, 2, 3], [0, 0, 2], [1.0, 1.0, 1.0]),      # lower entry
        (3, [0, 2, 3, 4], [1, 1, 1, 2], [1.0] * 4),           # duplicate column
        (3, [0, 1, 2, 3], [0, 1, 3], [1.0, 1.0, 1.0]),      # column >= n
        (3, [0, 1, 2, 3], [0, 1, 2], [1.0, np.nan, 1.0]),   # NaN
        (3, [0, 2, 1, 3], [0, 1, 1], [1.0] * 3),              # rowptr decreases
    ]
    for n, rp, ci, v in bad:
        with pytest.raises(hs.HsymError) as e:
            hs.hsym_create(n, np.array(rp), np.array(ci, np.int32), np.array(v))
        assert e.value.status == hs.HSYM_E_INVALID_ARG


def test_streaming_create_matches_whole():
    dev = _dev()
    g = hsymgen.Generator(9000, 80, 12)
    A = g.matrix()
    X = hsymgen.gauss_block(9, A.n, 8)
    Yw, _ = _run(A, X)
    h = hs.hsym_create_begin(A.n, hs.HSYM_FP64, hs.HSYM_GEOM_M(8))
    for r0, r1 in [(0, 1), (1, 700), (700, 5000), (5000, 5001), (5001, 9000)]:
        rp, ci, v = g.rows(r0, r1)
        hs.hsym_create_append(h, rp, ci, v)
    hs.hsym_create_finish(h)
    Xd = torch.from_numpy(X).to(dev)
    Yd = torch.empty_like(Xd)
    hs.spmm_sym(h, Xd, Yd)
    torch.cuda.synchronize()
    hs.hsym_destroy(h)
    Ys = Yd.cpu().numpy()
    assert np.linalg.norm(Ys - Yw) <= 1e-13 * np.linalg.norm(Yw)


@pytest.mark.parametrize("storage", [hs.HSYM_FP64, hs.HSYM_FP32])
def test_index_code_widths(storage):
    """16-bit tile-local codes wherever R * C <= 2^16 (the default geometries
    at widths of 4 and more), 32-bit otherwise; the product is the same
    within rounding either way."""
    A = hsymgen.generate(9001, 150, 17)
    H = oracle.SymMatrix.from_csr(A)
    X = hsymgen.gauss_block(4, A.n, 16)
    Yref = H.spmm(X)
    tol = 1e-12 if storage == hs.HSYM_FP64 else 1e-5
    G = hs.HSYM_GEOM_PANEL
    cases = [(0, 2, 16),                  # automatic
             (G(4, 6), 2, 16),            # R = 256, C = 64
             (G(16, 6), 2, 8),            # R * C = 2^16 exactly
             (G(16, 7), 4, 4)]            # 2^17: 32-bit codes
    for flags, width, m in cases:
        M = hs.Matrix(A, storage=storage, geom_m=m, flags=flags)
        info = M.info
        assert info["index_bytes"] == width, (flags, info)
        Xd = torch.from_numpy(X[:, :m].copy()).to(_dev())
        Yd = torch.empty_like(Xd)
        hs.spmm_sym(M.h, Xd, Yd)
        torch.cuda.synchronize()
        Y = Yd.cpu().numpy()
        assert np.linalg.norm(Y - Yref[:, :m]) <= tol * np.linalg.norm(Yref[:, :m])
        M.close()


def test_create_from_device_csr():
    """HSYM_DEVICE_PTRS: the same handle from CSR arrays held in device memory."""
    dev = _dev()
    A = hsymgen.generate(7001, 120, 33)
    X = hsymgen.gauss_block(5, A.n, 16)
    Yh, ih = _run(A, X)
    rp = torch.from_numpy(np.ascontiguousarray(A.rowptr, np.int64)).to(dev)
    ci = torch.from_numpy(np.ascontiguousarray(A.colind, np.int32)).to(dev)
    va = torch.from_numpy(np.ascontiguousarray(A.values, np.float64)).to(dev)
    h = hs.hsym_create_device(A.n, rp, ci, va, flags=hs.HSYM_GEOM_M(16))
    info = hs.hsym_info(h)
    Xd = torch.from_numpy(X).to(dev)
    Yd = torch.empty_like(Xd)
    hs.spmm_sym(h, Xd, Yd)
    torch.cuda.synchronize()
    hs.hsym_destroy(h)
    for k in ("nnz_stored", "norm1", "npanels", "ntiles", "padded_entries", "device_bytes"):
        assert info[k] == ih[k], k
    assert np.linalg.norm(Yd.cpu().numpy() - Yh) <= 1e-15 * np.linalg.norm(Yh)
    # the streaming create takes host arrays only
    with pytest.raises(hs.HsymError) as e:
        hs.hsym_create_begin(A.n, hs.HSYM_FP64, hs.HSYM_DEVICE_PTRS)
    assert e.value.status == hs.HSYM_E_INVALID_ARG
