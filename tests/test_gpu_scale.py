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


C4_SLABS = [(0, 64), (15_000_000, 15_000_064), (29_999_936, 30_000_000)]
C4_CHUNKS = [0, 234_375, 468_749]       # 64-row chunks of the block-64 preconditioner (first, middle, last)


def c4_rows(g, X, dtype):
    out = []
    for lo, hi in C4_SLABS:
        s0 = max(0, lo - WINDOW)
        rp, ci, v = g.rows(s0, hi, dtype)
        out.append(oracle.spmm_rows(s0, rp, ci, v.astype(np.float64), X, np.arange(lo, hi)))
    return out


def c4_check_rows(Y, ref, rtol):
    for (lo, hi), R in zip(C4_SLABS, ref):
        err = np.max(np.abs(Y[lo:hi] - R)) / np.max(np.abs(R))
        print("rows %d..%d: max rel err %.2e" % (lo, hi, err), flush=True)
        assert err <= rtol


def c4_check_block64(h, g, dtype, normH, R, dev):
    """The block-64 apply on the whole 30M x 16 block against the oracle's
    Preconditioner on the sampled 64-row chunks (each built from the chunk's
    own diagonal block, with the whole matrix's guard).  An fp32-storage
    handle keeps its factors Q in fp32: Q + E with |E| <= u32 |Q| elementwise,
    so ||E||_2 <= ||E||_F <= 8 u32 (Q orthogonal, 64 x 64), and column j of
    Q D_j Q^T R moves by at most 2 ||E||_2 ||D_j||_2 ||R_j|| (first order;
    D_j = diag(1 / g(lambda_i - mu_j)), g the guard)."""
    mu = np.linspace(-3.0, -2.0, 16)
    Wd = torch.from_numpy(R).to(dev)
    delta = oracle.GUARD * normH
    hs.hsym_kernel_precond(h, "block64", Wd, torch.from_numpy(mu).to(dev), delta)
    torch.cuda.synchronize()
    for c in C4_CHUNKS:
        r0, r1 = 64 * c, min(g.n, 64 * c + 64)
        rp, ci, v = g.rows(r0, r1, dtype)
        keep = ci < r1
        row_of = np.repeat(np.arange(r1 - r0), np.diff(rp))
        rp2 = np.zeros(r1 - r0 + 1, np.int64)
        np.cumsum(np.bincount(row_of[keep], minlength=r1 - r0), out=rp2[1:])
        blk = hsymgen.UpperCSR(r1 - r0, rp2, np.ascontiguousarray(ci[keep] - r0),
                               np.ascontiguousarray(v[keep].astype(np.float64)))
        pre = oracle.Preconditioner("block64", oracle.SymMatrix.from_csr(blk))
        pre.delta = delta
        ref = pre.apply(R[r0:r1], mu)
        W = Wd[r0:r1].cpu().numpy()
        err = np.linalg.norm(W - ref) / np.linalg.norm(ref)
        # host eigendecomposition per block against LAPACK: O(u kappa) of the shifted block
        lim = 1e-8
        if dtype == np.float32:
            dmax = np.max(np.abs(1.0 / oracle.guard(pre.lam[0][:r1 - r0, None] - mu[None, :], delta)), axis=0)
            bound = 2 * 8 * 2.0 ** -24 * np.sqrt(np.sum((dmax * np.linalg.norm(R[r0:r1], axis=0)) ** 2))
            lim += 1.01 * bound / np.linalg.norm(ref)
        print("block64 chunk %d (rows %d..%d): rel err %.2e (limit %.2e)" % (c, r0, r1, err, lim), flush=True)
        assert err <= lim
    del Wd


def test_c4_scale_mixed_vs_fp64_block64():
    """The largest single-GPU instance: n = 30,000,000, about 500 nonzeros
    per full row (7.5e9 stored entries, 64-bit tile offsets), block-64
    preconditioner, both storages by streaming create:
      - sampled rows of H X against the oracle (fp64 storage to 1e-12; fp32
        storage against the oracle on the same fp32 operands, within an fp32
        sum of about 500 terms);
      - the block-64 apply on sampled 64-row chunks against the oracle;
      - LOBPCG nev = 10, m = 16, tol 1e-6 in both forms: every eigenvalue of
        the mixed form within 1e-6 relative of the fp64 one, and the mixed
        eigenvectors' residuals measured with the fp64 SpMM within 1e-5 of
        ||H||_1: the tolerance (met on the fp32 SpMM's own products) plus the
        storage rounding (||fp64(fp32(H)) - H||_2 <= 2^-24 ||H||_1) plus the
        fp32 arithmetic of the products the mixed solve's residuals came
        from (a few 1e-6 of ||H||_1 for sums of about 500 terms)."""
    c = hsymgen.CONFIGS["C4"]
    g = hsymgen.Generator(c["n"], c["N"], c["seed"])
    dev = torch.device("cuda:0")
    flags = hs.HSYM_GEOM_M(16) | hs.HSYM_BUILD_BLOCK64
    X = hsymgen.gauss_block(77, g.n, 16)
    X32 = X.astype(np.float32).astype(np.float64)
    ref32 = c4_rows(g, X32, np.float32)
    t0 = time.perf_counter()

    h32 = stream_c4(g, hs.HSYM_FP32, np.float32, flags)
    info32 = hs.hsym_info(h32)
    assert info32["nnz_stored"] > 2 ** 31          # 64-bit offsets in use
    Xd = torch.from_numpy(X).to(dev)
    Yd = torch.empty_like(Xd)
    hs.spmm_sym(h32, Xd, Yd)
    torch.cuda.synchronize()
    c4_check_rows(Yd.cpu().numpy(), ref32, 2.5e-5)
    del Yd
    c4_check_block64(h32, g, np.float32, info32["norm1"], X, dev)
    V32 = torch.zeros((g.n, 10), dtype=torch.float64, device=dev)
    t = time.perf_counter()
    st, ev32, rep32 = hs.lobpcg_solve(h32, 10, 16, 1e-6, precond="block64",
                                      opts=hs.default_lobpcg_opts(seed=3, keep_history=0), evecs=V32)
    torch.cuda.synchronize()
    print("mixed: status %d, %d iterations, %.2fs, evals %s" % (st, rep32.iters, time.perf_counter() - t, ev32),
          flush=True)
    assert st == hs.HSYM_OK and max(rep32.resnorm[:10]) <= 1e-6
    hs.hsym_destroy(h32)
    torch.cuda.synchronize()

    ref64 = c4_rows(g, X, np.float64)
    h64 = stream_c4(g, hs.HSYM_FP64, np.float64, flags)
    info64 = hs.hsym_info(h64)
    Yd = torch.empty_like(Xd)
    hs.spmm_sym(h64, Xd, Yd)
    torch.cuda.synchronize()
    c4_check_rows(Yd.cpu().numpy(), ref64, 1e-12)
    del Yd, Xd
    c4_check_block64(h64, g, np.float64, info64["norm1"], X, dev)
    del X, X32
    t = time.perf_counter()
    st, ev64, rep64 = hs.lobpcg_solve(h64, 10, 16, 1e-6, precond="block64",
                                      opts=hs.default_lobpcg_opts(seed=3, keep_history=0))
    torch.cuda.synchronize()
    print("fp64: status %d, %d iterations, %.2fs, evals %s" % (st, rep64.iters, time.perf_counter() - t, ev64),
          flush=True)
    assert st == hs.HSYM_OK and max(rep64.resnorm[:10]) <= 1e-6
    # residuals of the mixed eigenpairs against the fp64 matrix
    HV = torch.empty_like(V32)
    hs.spmm_sym(h64, V32, HV)
    torch.cuda.synchronize()
    Rn = torch.linalg.vector_norm(HV - V32 * torch.from_numpy(ev32).to(dev)[None, :], dim=0).cpu().numpy()
    normH = info64["norm1"]
    rho = Rn / normH
    print("mixed eigenpairs, fp64 residuals / |H|_1: %s" % rho, flush=True)
    assert np.max(rho) <= 1e-5
    hs.hsym_destroy(h64)
    rel = np.abs(ev32 - ev64) / np.abs(ev64)
    print("per-eigenpair relative difference mixed vs fp64: %s (%.0fs in all)" % (rel, time.perf_counter() - t0),
          flush=True)
    assert np.max(rel) <= 1e-6


def stream_c4(g, storage, dtype, flags, slab=1_000_000):
    t = time.perf_counter()
    h = hs.hsym_create_begin(g.n, storage, flags)
    for r0 in range(0, g.n, slab):
        rp, ci, v = g.rows(r0, min(g.n, r0 + slab), dtype)
        hs.hsym_create_append(h, rp, ci, v)
        if (r0 // slab) % 10 == 9:
            print("  create: %d of %d rows, %.0fs" % (r0 + slab, g.n, time.perf_counter() - t), flush=True)
    hs.hsym_create_finish(h)
    print("built %s storage in %.1fs: %s" % ("fp32" if storage == hs.HSYM_FP32 else "fp64",
                                             time.perf_counter() - t, hs.hsym_info(h)), flush=True)
    return h
