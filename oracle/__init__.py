"""CPU FP64 oracle of the LOBPCG hot path.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and
the ``cpu_baseline`` leg of ``bench.py`` may import this package.  It shares
no code with the GPU library: its sparse kernels are the plain C loops in
``csr_oracle.c``; everything else is NumPy/SciPy (LAPACK) in fp64, written
step by step after the paper:

* SpMM with one stored triangle (Section 4.1): Y = H X, H_ij = H_ji.
* LOBPCG (Section 3.1, eqs. 6-9, Algorithm 1) with preconditioning
  (Section 3.2, eq. 11) and the conservative shift rules of Section 4.3.
* Lanczos with full re-orthogonalisation (Section 3, opening paragraph) and
  the convergence-check schedule of footnote 7 (Section 5.2).
* The multi-level start block of Section 3.3.1 (eq. 12, used recursively).

Readings taken where the paper is silent (each is listed with its reason in
the design notes of the repository): the relative residual is
||r_j|| / (||H||_1 ||x_j||); only the first nev columns gate convergence;
Householder QR orthonormalises blocks here (the GPU uses Cholesky-QR, same
span); a deficient W column is replaced by a seeded Gaussian column, a
deficient P is dropped for one iteration; the preconditioner shift guard is
delta = 1e-4 ||H||_1; "nearly converged" means relative residual <= 0.1.

Pins: see tests/test_oracle_*.py (dense products, closed-form spectra,
LAPACK eigensolvers, invariants).  Paper-printed values: parity unpinned --
the paper prints no eigenvalue, residual or matrix that can be regenerated.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import time
from dataclasses import dataclass, field

import numpy as np
import scipy.linalg as sla

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "csr_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lib = None

NEAR = 1e-1          # Section 4.3 rule 2 threshold; also "nearly converged" (rules 3-4)
GUARD = 1e-4         # shifted-denominator guard, as a fraction of ||H||_1
DEFICIENT = 1e-10    # rank test on the R factor of a column-normalised block
# P is orthonormalised through its QR factor and AP follows by the same
# (updated, not recomputed) transformation: a pivot r amplifies the rounding
# of both by 1 / r, so P is dropped for the iteration below this pivot
P_DEFICIENT = 1e-4
NO_PRECOND_ITERS = 3 # Section 4.3 rule 1


def build(force: bool = True) -> str:
    if not force and os.path.exists(_LIB) and os.path.getmtime(_LIB) >= os.path.getmtime(_SRC):
        return _LIB
    tmp = _LIB + ".tmp%d" % os.getpid()
    subprocess.run(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-o", tmp, _SRC, "-lm"],
                   check=True)
    os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB):
        build()
    lib = ctypes.CDLL(_LIB)
    i64, vp = ctypes.c_int64, ctypes.c_void_p
    lib.oracle_spmm_half.argtypes = [i64, vp, vp, vp, i64, vp, vp]
    lib.oracle_full_counts.argtypes = [i64, vp, vp, vp]
    lib.oracle_full_fill.argtypes = [i64, vp, vp, vp, vp, vp, vp]
    lib.oracle_spmm_full.argtypes = [i64, vp, vp, vp, i64, vp, vp]
    lib.oracle_norm1.argtypes = [i64, vp, vp, vp]
    lib.oracle_norm1.restype = ctypes.c_double
    lib.oracle_diagonal.argtypes = [i64, vp, vp, vp, vp]
    lib.oracle_diag_blocks.argtypes = [i64, vp, vp, vp, i64, vp]
    _lib = lib
    return lib


def _p(a):
    return ctypes.c_void_p(a.ctypes.data)


class SymMatrix:
    """H given by its stored upper triangle (upper CSR, fp64 or fp32 values).

    Values are promoted to fp64 once; every product is fp64."""

    def __init__(self, n, rowptr, colind, values):
        self.n = int(n)
        self.rowptr = np.ascontiguousarray(rowptr, np.int64)
        self.colind = np.ascontiguousarray(colind, np.int32)
        self.values = np.ascontiguousarray(values, np.float64)
        self._full = None
        self._norm1 = None
        self._diag = None

    @classmethod
    def from_csr(cls, A):
        return cls(A.n, A.rowptr, A.colind, A.values)

    @property
    def nnz_stored(self):
        return int(self.rowptr[-1])

    def full(self):
        """Mirrored full CSR (rowptr, colind, values)."""
        if self._full is None:
            lib = _load()
            cnt = np.empty(self.n, np.int64)
            lib.oracle_full_counts(self.n, _p(self.rowptr), _p(self.colind), _p(cnt))
            frp = np.zeros(self.n + 1, np.int64)
            np.cumsum(cnt, out=frp[1:])
            fci = np.empty(int(frp[-1]), np.int32)
            fv = np.empty(int(frp[-1]), np.float64)
            lib.oracle_full_fill(self.n, _p(self.rowptr), _p(self.colind), _p(self.values),
                                 _p(frp), _p(fci), _p(fv))
            self._full = (frp, fci, fv)
        return self._full

    def spmm(self, X):
        """Y = H X through the mirrored full CSR (rows in parallel)."""
        X = np.ascontiguousarray(X, np.float64)
        vec = X.ndim == 1
        X2 = X.reshape(self.n, -1)
        m = X2.shape[1]
        Y = np.empty((self.n, m), np.float64)
        frp, fci, fv = self.full()
        _load().oracle_spmm_full(self.n, _p(frp), _p(fci), _p(fv), m, _p(X2), _p(Y))
        return Y.reshape(-1) if vec else Y

    def spmm_half(self, X):
        """Y = H X straight from the stored triangle (sequential)."""
        X = np.ascontiguousarray(X, np.float64)
        vec = X.ndim == 1
        X2 = X.reshape(self.n, -1)
        m = X2.shape[1]
        Y = np.empty((self.n, m), np.float64)
        _load().oracle_spmm_half(self.n, _p(self.rowptr), _p(self.colind), _p(self.values),
                                 m, _p(X2), _p(Y))
        return Y.reshape(-1) if vec else Y

    def norm1(self):
        if self._norm1 is None:
            self._norm1 = float(_load().oracle_norm1(self.n, _p(self.rowptr), _p(self.colind),
                                                     _p(self.values)))
        return self._norm1

    def diagonal(self):
        if self._diag is None:
            d = np.empty(self.n, np.float64)
            _load().oracle_diagonal(self.n, _p(self.rowptr), _p(self.colind), _p(self.values), _p(d))
            self._diag = d
        return self._diag

    def diag_blocks(self, bs=64):
        nb = (self.n + bs - 1) // bs
        out = np.empty((nb, bs, bs), np.float64)
        _load().oracle_diag_blocks(self.n, _p(self.rowptr), _p(self.colind), _p(self.values),
                                   bs, _p(out))
        return out

    def dense(self):
        """Dense H (small n only), built from the stored triplets."""
        A = np.zeros((self.n, self.n))
        rows = np.repeat(np.arange(self.n), np.diff(self.rowptr))
        A[rows, self.colind] = self.values
        A[self.colind, rows] = self.values
        return A


# --------------------------------------------------------------------------
# preconditioner (Section 3.2 eq. 11; rules of Section 4.3)
# --------------------------------------------------------------------------

def spmm_rows(row0, rowptr, colind, values, X, rows):
    """Rows `rows` of Y = H X from a slab of the stored upper triangle
    (Section 4.1: each stored entry (r, c, a) gives Y_r += a X_c and, when
    r != c, Y_c += a X_r).

    The slab holds rows [row0, row0 + len(rowptr) - 1) in CSR form with
    global column indices; it must contain every row of the matrix that
    holds an entry in a column listed in `rows` (for the synthetic CI
    matrices: all rows within the coupling window before them) as well as
    the rows themselves.  X is the full n x m block.  Plain definition,
    fp64, one requested row at a time."""
    rowptr = np.asarray(rowptr, np.int64)
    colind = np.asarray(colind, np.int64)
    values = np.asarray(values, np.float64)
    X = np.asarray(X, np.float64)
    rows = np.asarray(rows, np.int64)
    nr = len(rowptr) - 1
    r_of = np.repeat(np.arange(row0, row0 + nr, dtype=np.int64), np.diff(rowptr))
    out = np.zeros((len(rows), X.shape[1]))
    for k, i in enumerate(rows):
        # U X and the diagonal: entries stored in row i
        a, b = rowptr[i - row0], rowptr[i - row0 + 1]
        out[k] += values[a:b] @ X[colind[a:b]]
        # U^T X: entries (r, i) with r < i
        sel = (colind == i) & (r_of != i)
        out[k] += values[sel] @ X[r_of[sel]]
    return out


def shifts(theta, rnorm, rho):
    """Per-column shifts mu_j (Section 4.3, rules 3 and 4).

    Rule 3: a nearly converged pair (rho_j <= NEAR) gets mu_j = theta_j - 2||r_j||
    (||x_j|| = 1).  Rule 4: from the first pair that is far from converged on,
    every later column reuses the shift of the pair before it.  Rule 2 makes
    sure rho_1 <= NEAR whenever shifts are needed."""
    m = len(theta)
    mu = np.empty(m)
    far = False
    for j in range(m):
        if not far and rho[j] > NEAR:
            far = True
        if far:
            mu[j] = mu[j - 1]
        else:
            mu[j] = theta[j] - 2.0 * rnorm[j]
    return mu


def guard(d, delta):
    """Keep a shifted denominator away from zero: |d| >= delta, sign kept (0 -> +)."""
    d = np.asarray(d, np.float64)
    return np.where(np.abs(d) >= delta, d, np.where(d >= 0, delta, -delta))


def fom_solve(A, b, k, delta):
    """Approximate solution of A x = b by k steps of the full orthogonalization
    method (Saad, Iterative Methods for Sparse Linear Systems, Algorithm 6.4):
    Arnoldi with modified Gram-Schmidt builds V_k and the Hessenberg H_k from
    v_1 = b / ||b||, then x = V_k y with H_k y = ||b|| e_1.  The Arnoldi
    process stops early when the next basis vector vanishes (the Krylov space
    is invariant).  H_k y = ||b|| e_1 is solved by Gaussian elimination with
    partial pivoting whose pivots are kept at least delta from zero (the
    guard of the shifted denominators)."""
    n = b.shape[0]
    beta = np.linalg.norm(b)
    if beta == 0.0:
        return np.zeros(n)
    V = np.zeros((n, k + 1))
    Hh = np.zeros((k + 1, k))
    V[:, 0] = b / beta
    kk = k
    for i in range(k):
        w = A @ V[:, i]
        for l in range(i + 1):
            Hh[l, i] = w @ V[:, l]
            w = w - Hh[l, i] * V[:, l]
        Hh[i + 1, i] = np.linalg.norm(w)
        if Hh[i + 1, i] <= 1e-14 * beta or i + 1 == k:
            kk = i + 1
            if Hh[i + 1, i] > 1e-14 * beta:
                V[:, i + 1] = w / Hh[i + 1, i]
            break
        V[:, i + 1] = w / Hh[i + 1, i]
    T = Hh[:kk, :kk].copy()
    rhs = np.zeros(kk)
    rhs[0] = beta
    # Gaussian elimination with partial pivoting, guarded pivots
    for c in range(kk):
        p = c + int(np.argmax(np.abs(T[c:, c])))
        if p != c:
            T[[c, p]] = T[[p, c]]
            rhs[[c, p]] = rhs[[p, c]]
        T[c, c] = float(guard(T[c, c], delta))
        for r in range(c + 1, kk):
            f = T[r, c] / T[c, c]
            T[r, c:] -= f * T[c, c:]
            rhs[r] -= f * rhs[c]
    y = np.zeros(kk)
    for c in range(kk - 1, -1, -1):
        y[c] = (rhs[c] - T[c, c + 1:] @ y[c + 1:]) / T[c, c]
    return V[:, :kk] @ y


class Preconditioner:
    """T_j = Htilde - mu_j I with Htilde = diag(H) ('jacobi') or the dense 64x64
    diagonal blocks of H ('block64'), solved directly (eq. 11), or the
    diagonal group tiles of H ('fom', Section 3.2 end and Section 4.3: the
    tiles of the many-body groups, each system solved by fom_iters steps of
    FOM per right-hand side with its own shift)."""

    def __init__(self, kind, A: SymMatrix, bs=64, groups=None, fom_iters=3):
        self.kind = kind
        self.A = A
        self.delta = GUARD * A.norm1()
        self.bs = bs
        if kind == "fom":
            # groups: ascending starts [0, ..., n]; groups above 64 rows are cut in 64-row pieces
            st = [0]
            g = np.asarray(groups, np.int64)
            for a, b in zip(g[:-1], g[1:]):
                for c in range(int(a), int(b), 64):
                    st.append(min(int(b), c + 64))
            self.starts = np.array(st, np.int64)
            self.tiles = []
            for a, b in zip(self.starts[:-1], self.starts[1:]):
                self.tiles.append(principal_submatrix(A, np.arange(a, b)).dense())
            self.fom_iters = fom_iters
        elif kind == "jacobi":
            self.d = A.diagonal()
        elif kind == "block64":
            blocks = A.diag_blocks(bs)
            n = A.n
            nb = blocks.shape[0]
            self.lam = np.empty((nb, bs))
            self.Q = np.empty((nb, bs, bs))
            for b in range(nb):
                sz = min(bs, n - b * bs)
                lam, Q = np.linalg.eigh(blocks[b, :sz, :sz])
                self.lam[b, :sz] = lam
                self.lam[b, sz:] = 1.0
                self.Q[b] = np.eye(bs)
                self.Q[b, :sz, :sz] = Q
        elif kind != "none":
            raise ValueError(kind)

    def apply(self, R, mu):
        if self.kind == "jacobi":
            return R / guard(self.d[:, None] - mu[None, :], self.delta)
        if self.kind == "fom":
            W = np.empty_like(R)
            for t, (a, b) in enumerate(zip(self.starts[:-1], self.starts[1:])):
                Ht = self.tiles[t]
                for j in range(R.shape[1]):
                    W[a:b, j] = fom_solve(Ht - mu[j] * np.eye(b - a), R[a:b, j], self.fom_iters, self.delta)
            return W
        n, m = R.shape
        bs = self.bs
        W = np.empty_like(R)
        for b in range(self.lam.shape[0]):
            r0, r1 = b * bs, min(n, (b + 1) * bs)
            sz = r1 - r0
            Q = self.Q[b, :sz, :sz]
            lam = self.lam[b, :sz]
            C = Q.T @ R[r0:r1]
            C = C / guard(lam[:, None] - mu[None, :], self.delta)
            W[r0:r1] = Q @ C
        return W


def precondition(pre, R, it, theta, rnorm, rho):
    """Step 6 of Algorithm 1 under the Section 4.3 rules; returns (W, mu or None)."""
    if pre is None or pre.kind == "none" or it <= NO_PRECOND_ITERS or rho[0] > NEAR:
        return R.copy(), None
    mu = shifts(theta, rnorm, rho)
    return pre.apply(R, mu), mu


# --------------------------------------------------------------------------
# LOBPCG (Algorithm 1)
# --------------------------------------------------------------------------

@dataclass
class LobpcgResult:
    evals: np.ndarray
    X: np.ndarray
    iters: int
    converged: bool
    rho: np.ndarray
    history: list = field(default_factory=list)   # per iteration: (theta, rho)
    p_dropped: int = 0
    w_replaced: int = 0
    seconds: float = 0.0


def _normalise_columns(V):
    nrm = np.linalg.norm(V, axis=0)
    ok = nrm > 0
    V = V.copy()
    V[:, ok] /= nrm[ok]
    return V, ok


def _householder(V):
    Q, R = np.linalg.qr(V)
    return Q, np.abs(np.diag(R))


def _project(V, bases):
    for B in bases:
        V = V - B @ (B.T @ V)
    return V


def lobpcg(A: SymMatrix, nev, m, tol, X0=None, precond="jacobi", maxit=1000, seed=0,
           keep_history=True, spmm=None, groups=None, fom_iters=3):
    """Lowest nev eigenpairs of H by LOBPCG with block width m (m >= nev).

    Follows Algorithm 1: Rayleigh quotient of the start block (step 1); per
    iteration residual (step 4), convergence test (step 5), preconditioned
    residual (step 6), orthogonalisation and Rayleigh-Ritz on span{X, W, P}
    (steps 7-9) and the new search direction P = (I - X_old X_old^T) X_new
    (step 10, with the index read as the next iterate)."""
    t0 = time.perf_counter()
    n = A.n
    if not (1 <= nev <= m and 3 * m <= n):
        raise ValueError("need 1 <= nev <= m and 3m <= n")
    Hx = spmm or A.spmm
    normH = A.norm1()
    pre = None if precond == "none" else Preconditioner(precond, A, groups=groups, fom_iters=fom_iters)
    if X0 is None:
        from hsymgen import gauss_block
        X0 = gauss_block(seed, n, m)
    X, _ = _householder(np.asarray(X0, np.float64))
    AX = Hx(X)
    Ah = X.T @ AX
    theta, C = np.linalg.eigh(0.5 * (Ah + Ah.T))
    X = X @ C
    AX = AX @ C
    P = AP = None
    res = LobpcgResult(theta[:nev].copy(), X, 0, False, None)
    rng_ctr = 0
    for it in range(1, maxit + 1):
        R = AX - X * theta[None, :]
        rnorm = np.linalg.norm(R, axis=0)
        rho = rnorm / normH
        if keep_history:
            res.history.append((theta.copy(), rho.copy()))
        res.rho = rho
        res.iters = it - 1
        if np.max(rho[:nev]) <= tol:
            res.converged = True
            break
        W, _ = precondition(pre, R, it, theta, rnorm, rho)
        # W <- W - X (X^T W), twice; then orthonormalise (rank-revealing test)
        W = _project(W, [X, X])
        for attempt in range(4):
            Wn, nz = _normalise_columns(W)
            Q, diagR = _householder(Wn)
            bad = (~nz) | (diagR < DEFICIENT)
            if not bad.any():
                break
            rng_ctr += 1
            from hsymgen import gauss_block
            G = gauss_block(seed * 1000003 + it * 101 + rng_ctr, n, m)
            W = Wn
            W[:, bad] = G[:, bad]
            W = _project(W, [X, X])
            res.w_replaced += int(bad.sum())
        # second pass: a QR pivot r leaves the rounding of the projection,
        # amplified by 1 / r, along X; projecting again and re-factoring
        # restores X^T W = 0 to working precision (twice is enough)
        W, _ = _householder(_project(Q, [X]))
        AW = Hx(W)
        if P is not None:
            for _ in range(2):
                C1 = X.T @ P
                C2 = W.T @ P
                P = P - X @ C1 - W @ C2
                AP = AP - AX @ C1 - AW @ C2
            nrm = np.linalg.norm(P, axis=0)
            if np.any(nrm == 0):
                P = AP = None
            else:
                P = P / nrm
                AP = AP / nrm
                Qp, Rp = np.linalg.qr(P)
                if np.min(np.abs(np.diag(Rp))) < P_DEFICIENT:
                    P = AP = None
                    res.p_dropped += 1
                else:
                    AP = sla.solve_triangular(Rp, AP.T, trans="T", lower=False).T
                    P = Qp
                    # second pass against [X W], the same transforms on AP
                    C1 = X.T @ P
                    C2 = W.T @ P
                    P = P - X @ C1 - W @ C2
                    AP = AP - AX @ C1 - AW @ C2
                    Qp, Rp = np.linalg.qr(P)
                    AP = sla.solve_triangular(Rp, AP.T, trans="T", lower=False).T
                    P = Qp
        if P is None:
            S = np.hstack([X, W])
            AS = np.hstack([AX, AW])
        else:
            S = np.hstack([X, W, P])
            AS = np.hstack([AX, AW, AP])
        Ah = S.T @ AS
        vals, C = np.linalg.eigh(0.5 * (Ah + Ah.T))
        Cx = C[:, :m]
        theta = vals[:m]
        X = S @ Cx
        AX = AS @ Cx
        Cp = Cx.copy()
        Cp[:m, :] = 0.0
        P = S @ Cp
        AP = AS @ Cp
    else:
        res.iters = maxit
    res.evals = theta[:nev].copy()
    res.X = X
    res.seconds = time.perf_counter() - t0
    return res


# --------------------------------------------------------------------------
# Multi-level initial guess (Section 3.3.1)
# --------------------------------------------------------------------------
def principal_submatrix(A: SymMatrix, rows):
    """H11: the rows and columns of H in the ascending index set `rows`,
    renumbered in order (the Hamiltonian of the smaller configuration space)."""
    rows = np.asarray(rows, np.int64)
    pos = np.full(A.n, -1, np.int64)
    pos[rows] = np.arange(rows.size)
    rp = [0]
    ci, vals = [], []
    for i in rows:
        for p in range(A.rowptr[i], A.rowptr[i + 1]):
            j = pos[A.colind[p]]
            if j >= 0:
                ci.append(j)
                vals.append(A.values[p])
        rp.append(len(ci))
    return SymMatrix(rows.size, np.array(rp, np.int64), np.array(ci, np.int32), np.array(vals, np.float64))


def pad_with_zeros(X1, rows, n):
    """Eq. 12: X0 = [X1; 0], the rows of the smaller space keep X1."""
    X0 = np.zeros((n, X1.shape[1]))
    X0[np.asarray(rows, np.int64)] = X1
    return X0


def multilevel_guess(A: SymMatrix, level, caps, m, tol, precond="jacobi", maxit=1000, seed=0):
    """Start block for the full solve, built recursively over the smaller
    spaces {i : level_i <= cap} for the ascending caps: the m lowest
    eigenvectors of each space (LOBPCG, every column gating convergence),
    started from a Gaussian block on the first space and from the previous
    space's eigenvectors padded with zeros (eq. 12) on the others; the last
    space's eigenvectors padded with zeros are returned, with each sub-solve's
    iteration count."""
    level = np.asarray(level)
    prev_rows, prev_X = None, None
    iters = []
    for cap in caps:
        rows = np.flatnonzero(level <= cap)
        H11 = principal_submatrix(A, rows)
        X0 = None
        if prev_rows is not None:
            pos = np.full(A.n, -1, np.int64)
            pos[rows] = np.arange(rows.size)
            X0 = pad_with_zeros(prev_X, pos[prev_rows], rows.size)
        r = lobpcg(H11, m, m, tol, X0=X0, precond=precond, maxit=maxit, seed=seed, keep_history=False)
        iters.append(r.iters)
        prev_rows, prev_X = rows, r.X[:, :m]
    return pad_with_zeros(prev_X, prev_rows, A.n), iters


# --------------------------------------------------------------------------
# Lanczos with full re-orthogonalisation
# --------------------------------------------------------------------------

def lanczos_check_interval(j):
    """Footnote 7: every 10 iterations up to 100, every 20 up to 200, every 40
    up to 400, and so on (the interval doubles with each doubling of j)."""
    iv, lim = 10, 100
    while j > lim:
        iv *= 2
        lim *= 2
    return iv


@dataclass
class LanczosResult:
    evals: np.ndarray
    X: np.ndarray
    iters: int
    converged: bool
    resid: np.ndarray
    alpha: np.ndarray
    beta: np.ndarray
    V: np.ndarray = None
    seconds: float = 0.0


def lanczos(A: SymMatrix, nev, tol, v0=None, maxit=2000, seed=0, keep_basis=False, spmm=None):
    """Lowest nev eigenpairs by single-vector Lanczos with full (twice repeated
    classical Gram-Schmidt) re-orthogonalisation; Ritz pairs from the
    tridiagonal T_j at the scheduled checks.  Converged when every one of the
    nev Ritz residuals beta_j |s_{j,i}| is <= tol ||H||_1."""
    t0 = time.perf_counter()
    n = A.n
    Hx = spmm or A.spmm
    normH = A.norm1()
    if v0 is None:
        from hsymgen import gauss_vector
        v0 = gauss_vector(seed, n)
    kmax = min(maxit, n)
    V = np.zeros((kmax + 1, n))      # rows are basis vectors
    V[0] = v0 / np.linalg.norm(v0)
    alpha = np.zeros(kmax)
    beta = np.zeros(kmax)
    evals = X = resid = None
    conv = False
    j = 0
    for j in range(1, kmax + 1):
        w = Hx(V[j - 1])
        if j > 1:
            w = w - beta[j - 2] * V[j - 2]
        alpha[j - 1] = w @ V[j - 1]
        w = w - alpha[j - 1] * V[j - 1]
        for _ in range(2):
            w = w - V[:j].T @ (V[:j] @ w)
        beta[j - 1] = np.linalg.norm(w)
        invariant = beta[j - 1] < 1e-14 * normH
        if j % lanczos_check_interval(j) == 0 or invariant or j == kmax:
            k = min(nev, j)
            th, S = sla.eigh_tridiagonal(alpha[:j], beta[:j - 1])
            resid = beta[j - 1] * np.abs(S[j - 1, :k])
            evals = th[:k]
            if np.all(resid <= tol * normH) or invariant or j == kmax:
                conv = bool(np.all(resid <= tol * normH)) and k == nev
                X = V[:j].T @ S[:, :k]
                break
        V[j] = w / beta[j - 1]
    res = LanczosResult(evals, X, j, conv, resid, alpha[:j].copy(), beta[:j].copy())
    if keep_basis:
        res.V = V[:j].copy()
    res.seconds = time.perf_counter() - t0
    return res
