"""Seeded generator: determinism, slab independence, shape statistics."""
import json
import os
import subprocess
import sys

import numpy as np
import pytest

import hsymgen

HERE = os.path.dirname(os.path.abspath(__file__))


def test_deterministic_and_sorted_upper():
    A = hsymgen.generate(3000, 40, 7)
    B = hsymgen.generate(3000, 40, 7)
    assert np.array_equal(A.rowptr, B.rowptr)
    assert np.array_equal(A.colind, B.colind)
    assert np.array_equal(A.values, B.values)
    rows = np.repeat(np.arange(A.n), np.diff(A.rowptr))
    assert np.all(A.colind >= rows)                       # upper triangle
    # first entry of each row is the diagonal; columns strictly increase
    assert np.all(A.colind[A.rowptr[:-1]] == np.arange(A.n))
    same_row = rows[1:] == rows[:-1]
    assert np.all(np.diff(A.colind)[same_row] > 0)
    C = hsymgen.generate(3000, 40, 8)
    assert not np.array_equal(A.values[: min(A.nnz, C.nnz)], C.values[: min(A.nnz, C.nnz)])


def test_slab_equals_whole():
    g = hsymgen.Generator(5000, 60, 3)
    A = g.matrix()
    for r0, r1 in [(0, 1), (17, 911), (2500, 5000), (4999, 5000)]:
        rp, ci, v = g.rows(r0, r1)
        o0, o1 = A.rowptr[r0], A.rowptr[r1]
        assert np.array_equal(rp, A.rowptr[r0:r1 + 1] - o0)
        assert np.array_equal(ci, A.colind[o0:o1])
        assert np.array_equal(v, A.values[o0:o1])


def test_thread_count_independent():
    code = ("import hsymgen,hashlib;A=hsymgen.generate(4000,50,5);"
            "print(hashlib.sha1(A.colind.tobytes()+A.values.tobytes()).hexdigest())")
    outs = []
    for t in ("1", "4"):
        env = dict(os.environ, OMP_NUM_THREADS=t, PYTHONPATH=os.path.dirname(HERE))
        outs.append(subprocess.run([sys.executable, "-c", code], env=env, check=True,
                                   capture_output=True, text=True).stdout.strip())
    assert outs[0] == outs[1]


def test_fp32_values_are_rounded_fp64():
    g = hsymgen.Generator(2000, 40, 1)
    _, _, v64 = g.rows(0, 2000, np.float64)
    _, _, v32 = g.rows(0, 2000, np.float32)
    assert np.array_equal(v64.astype(np.float32), v32)


@pytest.mark.parametrize("n,N,seed,rtol", [(2000, 40, 1, 0.1), (60000, 300, 2, 0.03)])
def test_structure_statistics(n, N, seed, rtol):
    g = hsymgen.Generator(n, N, seed)
    A = g.matrix()
    st, lb = g.blocks()
    sizes = np.diff(st)
    assert st[0] == 0 and st[-1] == n
    assert np.all(sizes[:-1] >= 16) and np.all(sizes <= 64)
    assert set(np.unique(lb)) <= set(range(5))
    full_per_row = (2 * A.nnz - n) / n
    # expectation is exact; the tolerance covers the tile-presence variance
    assert abs(full_per_row - N) / N < rtol
    rows = np.repeat(np.arange(n), np.diff(A.rowptr))
    bi = np.searchsorted(st, rows, side="right") - 1
    bj = np.searchsorted(st, A.colind, side="right") - 1
    # diagonal H_ii = 10 q + U(0,1)
    dmask = rows == A.colind
    dq = A.values[dmask] - 10.0 * lb[bi[dmask]]
    assert np.all((dq >= 0) & (dq < 1))
    # off-diagonal entries only in tiles with |dq| <= 2 inside the window
    off = ~dmask
    assert np.all(np.abs(lb[bi[off]] - lb[bj[off]]) <= 2)
    assert np.all(bj[off] - bi[off] <= hsymgen.WINDOW_BLOCKS)
    v = A.values[off]
    assert abs(v.mean()) < 0.02 and abs(v.std() - 0.3) < 0.02


def test_blockdiag_variant_has_only_diagonal_tiles():
    g = hsymgen.Generator(3000, 40, 9, variant="blockdiag")
    A = g.matrix()
    st, _ = g.blocks()
    rows = np.repeat(np.arange(A.n), np.diff(A.rowptr))
    assert np.array_equal(np.searchsorted(st, rows, side="right"),
                          np.searchsorted(st, A.colind, side="right"))


def test_generator_constants_match_paper_fig2():
    """The in-tile density of a nonzero off-diagonal tile follows the counts
    printed for the 6Li Nmax=2 example (Section 2.2, Fig. 2)."""
    with open(os.path.join(HERE, "golden", "fig2_li6_nmax2.json")) as f:
        g = json.load(f)
    # the fixture is internally consistent with the paper's own arithmetic
    # the printed tile total equals the strictly-lower tile count 92*91/2,
    # while the element total 800*801/2 includes the diagonal
    assert g["tiles_lower_total"] == g["groups"] * (g["groups"] - 1) // 2
    assert g["states"] * (g["states"] + 1) // 2 == 320400
    assert round(g["nonzero_tiles_lower"] / g["tiles_lower_total"], 2) == 0.44
    assert round(g["nnz_lower"] / 320400, 3) == 0.104
    assert abs(g["states"] / g["groups"] - g["mean_group_size"]) < 0.05
    rho = g["nnz_lower"] / (g["nonzero_tiles_lower"] * g["mean_group_size"] ** 2)
    assert abs(rho - hsymgen.RHO_OFF) / hsymgen.RHO_OFF < 0.03


def test_gauss_block():
    X = hsymgen.gauss_block(4, 20000, 8)
    assert X.shape == (20000, 8)
    assert abs(X.mean()) < 0.02 and abs(X.std() - 1) < 0.02
    assert np.array_equal(X, hsymgen.gauss_block(4, 20000, 8))
    assert np.array_equal(X[:100], hsymgen.gauss_block(4, 100, 8))
