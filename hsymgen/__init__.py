"""Seeded synthetic inputs shared by the CPU oracle and the GPU library.

The generator draws sparse symmetric matrices shaped like nuclear
configuration-interaction Hamiltonians (the tile picture of Section 2.2 and
Fig. 2: groups of basis states, nonzero tiles only between groups whose level
labels are close, densest tiles on the diagonal) and emits the upper triangle,
diagonal included, as CSR with int64 row pointers, int32 column indices and
fp64 or fp32 values.  It also draws Gaussian start blocks.

Nothing here computes any part of the eigensolver; both the oracle and the
GPU path read the arrays written here.  The C source is ``hsymgen.c``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "hsymgen.c")
_LIB = os.path.join(_HERE, "libhsymgen.so")
_lib = None

# Shapes of the synthetic workloads: (n, full-row nonzeros N incl. diagonal, seed)
CONFIGS = {
    "C1": dict(n=2_000, N=40, seed=1),
    "C2": dict(n=500_000, N=300, seed=2),
    "C3": dict(n=5_000_000, N=400, seed=3),
    "C4": dict(n=30_000_000, N=500, seed=4),
}

WINDOW_BLOCKS = 64      # coupling window in blocks (about 2,560 rows)
RHO_OFF = 0.24          # entry density of a present off-diagonal tile
RHO_DIAG = 0.5          # entry density of a diagonal tile
SIGMA = 0.3             # std dev of off-diagonal values

VARIANTS = {"banded": 0, "uniform": 1, "blockdiag": 2}


def build(force: bool = True) -> str:
    """Compile libhsymgen.so in place with gcc/OpenMP."""
    if not force and os.path.exists(_LIB) and os.path.getmtime(_LIB) >= os.path.getmtime(_SRC):
        return _LIB
    tmp = _LIB + ".tmp%d" % os.getpid()
    cmd = ["gcc", "-O3", "-march=x86-64-v2", "-fopenmp", "-fPIC", "-shared", "-o", tmp, _SRC, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB):
        build()
    lib = ctypes.CDLL(_LIB)
    i64, u64, f64, vp = ctypes.c_int64, ctypes.c_uint64, ctypes.c_double, ctypes.c_void_p
    lib.hsg_create.restype = vp
    lib.hsg_create.argtypes = [i64, f64, u64, i64, f64, f64, f64, ctypes.c_int]
    lib.hsg_destroy.argtypes = [vp]
    lib.hsg_nblocks.restype = i64; lib.hsg_nblocks.argtypes = [vp]
    lib.hsg_ptile.restype = f64; lib.hsg_ptile.argtypes = [vp]
    lib.hsg_rho.restype = f64; lib.hsg_rho.argtypes = [vp]
    lib.hsg_ntiles.restype = i64; lib.hsg_ntiles.argtypes = [vp]
    lib.hsg_blocks.argtypes = [vp, vp, vp]
    lib.hsg_count_rows.argtypes = [vp, i64, i64, vp]
    lib.hsg_fill_rows.argtypes = [vp, i64, i64, vp, vp, vp, vp]
    lib.hsg_gauss_x0.argtypes = [u64, i64, i64, vp]
    lib.hsg_gauss_v0.argtypes = [u64, i64, vp]
    _lib = lib
    return lib


def _ptr(a):
    return ctypes.c_void_p(a.ctypes.data) if a is not None else None


@dataclass
class UpperCSR:
    """Upper triangle (diagonal included) of a symmetric matrix in CSR form."""
    n: int
    rowptr: np.ndarray   # int64[n+1]
    colind: np.ndarray   # int32[nnz]
    values: np.ndarray   # float64 or float32 [nnz]

    @property
    def nnz(self) -> int:
        return int(self.rowptr[-1])


class Generator:
    """Block structure of GEN(n, N, seed); rows can be produced slab by slab."""

    def __init__(self, n: int, N: float, seed: int, variant: str = "banded",
                 window: int = WINDOW_BLOCKS, rho: float = RHO_OFF,
                 rho_diag: float = RHO_DIAG, sigma: float = SIGMA):
        lib = _load()
        self.n = int(n)
        self._h = lib.hsg_create(self.n, float(N), int(seed) & (2**64 - 1), int(window),
                                 float(rho), float(rho_diag), float(sigma), VARIANTS[variant])
        if not self._h:
            raise MemoryError("hsg_create failed")
        self.nblocks = lib.hsg_nblocks(self._h)
        self.p_tile = lib.hsg_ptile(self._h)
        self.rho = lib.hsg_rho(self._h)
        self.ntiles = lib.hsg_ntiles(self._h)

    def __del__(self):
        # at interpreter exit the module globals may already be gone
        if getattr(self, "_h", None) and _load is not None and _lib is not None:
            _lib.hsg_destroy(self._h)
            self._h = None

    def blocks(self):
        """(starts int64[nblocks+1], labels int32[nblocks])"""
        st = np.empty(self.nblocks + 1, np.int64)
        lb = np.empty(self.nblocks, np.int32)
        _load().hsg_blocks(self._h, _ptr(st), _ptr(lb))
        return st, lb

    def levels(self) -> np.ndarray:
        """Level label q of every row (its block's label), int32[n]: the
        stand-in for a configuration's excitation quanta."""
        st, lb = self.blocks()
        return np.repeat(lb, np.diff(st)).astype(np.int32)

    def count_rows(self, r0: int, r1: int) -> np.ndarray:
        c = np.empty(r1 - r0, np.int64)
        _load().hsg_count_rows(self._h, r0, r1, _ptr(c))
        return c

    def rows(self, r0: int, r1: int, dtype=np.float64):
        """Rows [r0, r1): (rowptr relative int64[r1-r0+1], colind int32, values)."""
        c = self.count_rows(r0, r1)
        rp = np.zeros(r1 - r0 + 1, np.int64)
        np.cumsum(c, out=rp[1:])
        nnz = int(rp[-1])
        ci = np.empty(nnz, np.int32)
        dt = np.dtype(dtype)
        v = np.empty(nnz, dt)
        _load().hsg_fill_rows(self._h, r0, r1, _ptr(rp), _ptr(ci),
                              _ptr(v) if dt == np.float64 else None,
                              _ptr(v) if dt == np.float32 else None)
        return rp, ci, v

    def matrix(self, dtype=np.float64) -> UpperCSR:
        rp, ci, v = self.rows(0, self.n, dtype)
        return UpperCSR(self.n, rp, ci, v)


def generate(n: int, N: float, seed: int, dtype=np.float64, variant: str = "banded",
             **kw) -> UpperCSR:
    """GEN(n, N, seed): whole upper-triangle CSR."""
    return Generator(n, N, seed, variant=variant, **kw).matrix(dtype)


def levels(n: int, N: float, seed: int, variant: str = "banded", **kw) -> np.ndarray:
    """Row level labels of GEN(n, N, seed)."""
    return Generator(n, N, seed, variant=variant, **kw).levels()


def config(name: str, dtype=np.float64) -> UpperCSR:
    c = CONFIGS[name]
    return generate(c["n"], c["N"], c["seed"], dtype)


def gauss_block(seed: int, n: int, m: int) -> np.ndarray:
    """i.i.d. N(0,1) start block, n x m row-major (stream 'x0')."""
    out = np.empty((n, m), np.float64)
    _load().hsg_gauss_x0(int(seed) & (2**64 - 1), n, m, _ptr(out))
    return out


def gauss_vector(seed: int, n: int) -> np.ndarray:
    """i.i.d. N(0,1) start vector (stream 'v0')."""
    out = np.empty(n, np.float64)
    _load().hsg_gauss_v0(int(seed) & (2**64 - 1), n, _ptr(out))
    return out


def laplacian_1d(n: int) -> UpperCSR:
    """Upper triangle of tridiag(-1, 2, -1): a matrix with a closed-form spectrum."""
    rp = np.zeros(n + 1, np.int64)
    cnt = np.full(n, 2, np.int64)
    cnt[-1] = 1
    np.cumsum(cnt, out=rp[1:])
    ci = np.empty(int(rp[-1]), np.int32)
    v = np.empty(int(rp[-1]), np.float64)
    ci[rp[:-1]] = np.arange(n, dtype=np.int32)
    v[rp[:-1]] = 2.0
    off = rp[:-1][:-1] + 1
    ci[off] = np.arange(1, n, dtype=np.int32)
    v[off] = -1.0
    return UpperCSR(n, rp, ci, v)
