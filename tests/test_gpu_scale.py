"""Parity at the mixed-precision scale configuration: n = 5,000,000, about 400
nonzeros per full row (1.0e9 stored entries), built by streaming create.

Checks (sampled where the full product is not formed on the host):
  - rows of H X at the start, middle and end of the matrix against the
    oracle: for fp32 storage (the mixed form: X staged in fp32, fp32
    products and sums) against the oracle on the fp32 values and the
    fp32-rounded block, to the size of an fp32 sum of some 400 terms; for
    fp64 storage to 1e-12;
  - LOBPCG in the mixed form (fp32 storage) against the fp64 form, nev = 10,
    m = 16, tol 1e-6, Jacobi: both converge, and every eigenvalue of the
    mixed form is within 1e-6 relative of the fp64 one.
"""
import time

import numpy as np
import pytest

import hsymgen
import oracle

pytestmark = [pytest.mark.gpu, pytest.mark.slow]

torch = pytest.importorskip("torch")
import paper_1609_01689_amd as hs  # noqa: E402

SLABS = [(0, 64), (2_500_000, 2_500_064), (4_999_936, 5_000_000)]
WINDOW = 4200   # rows above a row that can hold entries in its column (65 groups of <= 64 rows)


def stream(g, storage, dtype, m=16, slab=250_000):
    t = time.perf_counter()
    h = hs.hsym_create_begin(g.n, storage, hs.HSYM_GEOM_M(m))
    for r0 in range(0, g.n, slab):
        rp, ci, v = g.rows(r0, min(g.n, r0 + slab), dtype)
        hs.hsym_create_append(h, rp, ci, v)
    hs.hsym_create_finish(h)
    print("built %s storage in %.1fs: %s" % ("fp32" if storage == hs.HSYM_FP32 else "fp64",
                                             time.perf_counter() - t, hs.hsym_info(h)), flush=True)
    return h


def reference_rows(g, X, dtype):
    out = []
    for lo, hi in SLABS:
        s0 = max(0, lo - WINDOW)
        rp, ci, v = g.rows(s0, hi, dtype)
        out.append(oracle.spmm_rows(s0, rp, ci, v.astype(np.float64), X, np.arange(lo, hi)))
    return out


def check_rows(Y, ref, rtol):
    for (lo, hi), R in zip(SLABS, ref):
        err = np.max(np.abs(Y[lo:hi] - R)) / np.max(np.abs(R))
        print("rows %d..%d: max rel err %.2e" % (lo, hi, err), flush=True)
        assert err <= rtol


def test_c3_scale_mixed_vs_fp64():
    c = hsymgen.CONFIGS["C3"]
    g = hsymgen.Generator(c["n"], c["N"], c["seed"])
    dev = torch.device("cuda:0")
    X = hsymgen.gauss_block(31, g.n, 16)
    Xd = torch.from_numpy(X).to(dev)
    X32 = X.astype(np.float32).astype(np.float64)
    ref32 = reference_rows(g, X32, np.float32)         # fp32 values, X rounded to fp32

    h32 = stream(g, hs.HSYM_FP32, np.float32)
    Yd = torch.empty_like(Xd)
    hs.spmm_sym(h32, Xd, Yd)
    torch.cuda.synchronize()
    # fp32 values, the block staged in fp32, fp32 products and run sums:
    # against the oracle on the same fp32 operands, within an fp32 sum of
    # about 400 terms (gamma_400 u32 |H||X| is about 2.4e-5 |H||X|)
    check_rows(Yd.cpu().numpy(), ref32, 2e-5)
    Yf = torch.empty((g.n, 16), dtype=torch.float32, device=dev)
    hs.spmm_sym_f32(h32, Xd.float(), Yf)
    torch.cuda.synchronize()
    check_rows(Yf.double().cpu().numpy(), ref32, 2e-5)  # result rounded to fp32
    del Yf
    t = time.perf_counter()
    st, ev32, rep32 = hs.lobpcg_solve(h32, 10, 16, 1e-6, precond="jacobi",
                                      opts=hs.default_lobpcg_opts(seed=3, keep_history=0))
    t32 = time.perf_counter() - t
    print("mixed: status %d, %d iterations, %.2fs, evals %s" % (st, rep32.iters, t32, ev32), flush=True)
    assert st == hs.HSYM_OK and max(rep32.resnorm[:10]) <= 1e-6
    hs.hsym_destroy(h32)

    ref64 = reference_rows(g, X, np.float64)
    h64 = stream(g, hs.HSYM_FP64, np.float64)
    hs.spmm_sym(h64, Xd, Yd)
    torch.cuda.synchronize()
    check_rows(Yd.cpu().numpy(), ref64, 1e-12)
    t = time.perf_counter()
    st, ev64, rep64 = hs.lobpcg_solve(h64, 10, 16, 1e-6, precond="jacobi",
                                      opts=hs.default_lobpcg_opts(seed=3, keep_history=0))
    t64 = time.perf_counter() - t
    print("fp64: status %d, %d iterations, %.2fs, evals %s" % (st, rep64.iters, t64, ev64), flush=True)
    assert st == hs.HSYM_OK and max(rep64.resnorm[:10]) <= 1e-6
    hs.hsym_destroy(h64)
    rel = np.abs(ev32 - ev64) / np.abs(ev64)
    print("per-eigenpair relative difference mixed vs fp64: %s" % rel, flush=True)
    assert np.max(rel) <= 1e-6
