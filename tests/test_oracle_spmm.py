"""Pins of the oracle's sparse kernels against things other than itself:
SciPy sparse/dense products, unit-vector extraction, closed-form Laplacian
modes and row sums."""
import numpy as np
import pytest
import scipy.sparse as sp

import hsymgen
import oracle


def scipy_full(A):
    U = sp.csr_matrix((A.values.astype(np.float64), A.colind, A.rowptr), shape=(A.n, A.n))
    return (U + U.T - sp.diags(U.diagonal())).tocsr()


@pytest.fixture(scope="module")
def c1():
    return hsymgen.config("C1")


@pytest.mark.parametrize("m", [1, 8, 16])
def test_half_full_dense_agree(c1, m):
    H = oracle.SymMatrix.from_csr(c1)
    X = hsymgen.gauss_block(2, c1.n, m)
    D = scipy_full(c1).toarray()
    Yd = D @ X
    Yh = H.spmm_half(X)
    Yf = H.spmm(X)
    scale = np.abs(D) @ np.abs(X)
    assert np.all(np.abs(Yh - Yd) <= 64 * 2.2e-16 * scale + 1e-300)
    assert np.all(np.abs(Yf - Yd) <= 64 * 2.2e-16 * scale + 1e-300)


def test_unit_vectors_extract_columns(c1):
    """H e_j is column j of H: entries above the diagonal come from the stored
    row j's partners (transposed half), entries at/below from row j itself."""
    H = oracle.SymMatrix.from_csr(c1)
    cols = np.array([0, 1, 777, 1999])
    X = np.zeros((c1.n, len(cols)))
    X[cols, np.arange(len(cols))] = 1.0
    Y = H.spmm_half(X)
    for k, j in enumerate(cols):
        ref = np.zeros(c1.n)
        # stored (j, c) for c >= j gives H_cj; stored (r, j) for r < j gives H_rj
        s, e = c1.rowptr[j], c1.rowptr[j + 1]
        ref[c1.colind[s:e]] = c1.values[s:e]
        rows = np.repeat(np.arange(c1.n), np.diff(c1.rowptr))
        hit = (c1.colind == j) & (rows != j)
        ref[rows[hit]] = c1.values[hit]
        assert np.array_equal(Y[:, k], ref)


def test_ones_give_row_sums(c1):
    H = oracle.SymMatrix.from_csr(c1)
    F = scipy_full(c1)
    y = H.spmm(np.ones(c1.n))
    assert np.allclose(y, np.asarray(F.sum(axis=1)).ravel(), rtol=0, atol=1e-12)


def test_laplacian_sine_modes():
    n = 500
    L = oracle.SymMatrix.from_csr(hsymgen.laplacian_1d(n))
    k = np.array([1, 2, 50, 499])
    i = np.arange(1, n + 1)[:, None]
    V = np.sin(i * k[None, :] * np.pi / (n + 1))
    lam = 2 - 2 * np.cos(k * np.pi / (n + 1))
    for Y in (L.spmm(V), L.spmm_half(V)):
        assert np.max(np.abs(Y - V * lam[None, :])) < 1e-12


def test_norm1_and_diagonal(c1):
    H = oracle.SymMatrix.from_csr(c1)
    D = scipy_full(c1).toarray()
    assert abs(H.norm1() - np.abs(D).sum(axis=1).max()) < 1e-12
    assert np.array_equal(H.diagonal(), np.diag(D))
    B = H.diag_blocks(64)
    for b in (0, 5, B.shape[0] - 1):
        r0, r1 = 64 * b, min(c1.n, 64 * b + 64)
        assert np.array_equal(B[b, : r1 - r0, : r1 - r0], D[r0:r1, r0:r1])


def test_dense_builder_matches_scipy(c1):
    H = oracle.SymMatrix.from_csr(c1)
    assert np.array_equal(H.dense(), scipy_full(c1).toarray())


def test_spmm_rows_from_slab_matches_full():
    """Rows of H X from a slab of the stored triangle (the form used for
    sampled parity at sizes where the full product is not formed) agree with
    the full product, including rows whose transposed entries come from rows
    far above them."""
    g = hsymgen.Generator(12000, 60, 21)
    A = g.matrix()
    X = hsymgen.gauss_block(5, A.n, 8)
    Yref = oracle.SymMatrix.from_csr(A).spmm(X)
    for lo, hi in [(0, 64), (6000, 6100), (11950, 12000)]:
        s0 = max(0, lo - 4200)
        rp, ci, v = g.rows(s0, hi)
        Y = oracle.spmm_rows(s0, rp, ci, v, X, np.arange(lo, hi))
        assert np.max(np.abs(Y - Yref[lo:hi])) <= 1e-12 * np.max(np.abs(Yref))
