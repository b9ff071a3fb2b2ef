"""Python binding of libhsym, the MI355X (gfx950) LOBPCG hot path.

Argument marshalling only: every step of every call runs in the HIP library
``libhsym.so`` built from ``csrc/``.  Device buffers are torch tensors on a
ROCm device (torch is used for device memory and streams only).  Importing
this package does not load the library; the first call does, and it raises
``RuntimeError`` if the library was not built -- there is no fallback path.

The functions keep the names of the C ABI in ``include/hsym.h``:
``hsym_create``, ``hsym_create_begin/append/finish``, ``hsym_destroy``,
``hsym_info``, ``spmm_sym``, ``spmm_sym_f32``, ``lobpcg_solve``,
``lanczos_solve``, the ``lobpcg_ctx_*`` step interface and the request loop
``hsym_serve`` / ``hsym_serve_sim``.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("HSYM_LIB", os.path.join(_HERE, "libhsym.so"))

HSYM_OK, HSYM_NOT_CONVERGED = 0, 1
HSYM_E_INVALID_ARG, HSYM_E_OUT_OF_MEMORY, HSYM_E_DEVICE = -1, -2, -3
HSYM_E_BREAKDOWN, HSYM_E_NUMERIC, HSYM_E_UNSUPPORTED = -4, -5, -6
HSYM_FP64, HSYM_FP32 = 0, 1
PRECOND = {"none": 0, "jacobi": 1, "block64": 2, "fom": 3}
HSYM_BUILD_BLOCK64 = 0x2
HSYM_INDEX16 = 0x4
HSYM_DEVICE_PTRS = 0x1
MAX_BLOCK = 16
MAX_HISTORY = 4096


def HSYM_GEOM_M(m: int) -> int:
    return (int(m) & 0xFF) << 8


def HSYM_GEOM_PANEL(r64: int, lc: int) -> int:
    """Explicit panel geometry: 64 * r64 panel rows, 2**lc chunk columns."""
    return ((int(r64) & 0xFF) << 16) | ((int(lc) & 0xF) << 24)


class HsymError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("hsym status %d: %s" % (status, msg))
        self.status = status


class hsym_tune_entry(ctypes.Structure):
    _fields_ = [("panel_rows", ctypes.c_int), ("chunk_cols", ctypes.c_int), ("ms", ctypes.c_double)]


class hsym_info_t(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("nnz_stored", ctypes.c_int64), ("norm1", ctypes.c_double),
                ("storage", ctypes.c_int), ("panel_rows", ctypes.c_int), ("chunk_cols", ctypes.c_int),
                ("npanels", ctypes.c_int64), ("ntiles", ctypes.c_int64), ("nslots", ctypes.c_int64),
                ("padded_entries", ctypes.c_int64), ("device_bytes", ctypes.c_int64),
                ("has_block64", ctypes.c_int), ("index_bytes", ctypes.c_int),
                ("npieces", ctypes.c_int64), ("piece_entries", ctypes.c_int)]


class lobpcg_opts(ctypes.Structure):
    _fields_ = [("maxit", ctypes.c_int), ("seed", ctypes.c_uint64), ("check_every", ctypes.c_int),
                ("no_precond_iters", ctypes.c_int), ("near", ctypes.c_double), ("guard", ctypes.c_double),
                ("keep_history", ctypes.c_int), ("graph", ctypes.c_int), ("fom_iters", ctypes.c_int),
                ("timers", ctypes.c_int)]


class lobpcg_report(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int), ("converged", ctypes.c_int), ("spmm_calls", ctypes.c_int),
                ("p_dropped", ctypes.c_int), ("w_replaced", ctypes.c_int),
                ("theta", ctypes.c_double * MAX_BLOCK), ("resnorm", ctypes.c_double * MAX_BLOCK),
                ("seconds", ctypes.c_double), ("phase_ms", ctypes.c_double * 8),
                ("history_len", ctypes.c_int), ("history", ctypes.c_double * MAX_HISTORY),
                ("rr_rounds_max", ctypes.c_int), ("batched_iters", ctypes.c_int)]


class lanczos_opts(ctypes.Structure):
    _fields_ = [("maxit", ctypes.c_int), ("seed", ctypes.c_uint64)]


class lanczos_report(ctypes.Structure):
    _fields_ = [("iters", ctypes.c_int), ("converged", ctypes.c_int),
                ("resnorm", ctypes.c_double * MAX_BLOCK), ("seconds", ctypes.c_double),
                ("spmv_ms", ctypes.c_double), ("orth_ms", ctypes.c_double)]


class hsym_request(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("rowptr", ctypes.c_void_p), ("colind", ctypes.c_void_p),
                ("values", ctypes.c_void_p), ("values_prec", ctypes.c_int), ("storage", ctypes.c_int),
                ("nev", ctypes.c_int), ("block_width", ctypes.c_int), ("precond", ctypes.c_int),
                ("tol", ctypes.c_double), ("seed", ctypes.c_uint64), ("arrival_s", ctypes.c_double),
                ("status", ctypes.c_int), ("iters", ctypes.c_int), ("evals", ctypes.c_double * MAX_BLOCK),
                ("admit_s", ctypes.c_double), ("finish_s", ctypes.c_double), ("device_bytes", ctypes.c_int64),
                ("error", ctypes.c_char * 128)]


class hsym_serve_opts(ctypes.Structure):
    _fields_ = [("budget_bytes", ctypes.c_int64), ("max_active", ctypes.c_int),
                ("iters_per_round", ctypes.c_int), ("maxit", ctypes.c_int), ("autotune", ctypes.c_int),
                ("loaders", ctypes.c_int)]


class hsym_serve_report(ctypes.Structure):
    _fields_ = [("wall_s", ctypes.c_double), ("rounds", ctypes.c_int), ("tuned_classes", ctypes.c_int),
                ("max_active_seen", ctypes.c_int), ("peak_reserved_bytes", ctypes.c_int64)]


_lib = None
_vp, _i64, _int, _dbl = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int, ctypes.c_double

_SIGS = {
    "hsym_create": [ctypes.POINTER(_vp), _i64, _vp, _vp, _vp, _int, _int, _int, _vp],
    "hsym_create_begin": [ctypes.POINTER(_vp), _i64, _int, _int, _vp],
    "hsym_attach_group_tiles": [_vp, _i64, _vp, _vp, _vp, _vp, _int],
    "lobpcg_guess_multilevel": [_i64, _vp, _vp, _vp, _int, _vp, _int, _vp, _int, _int, _dbl, _int,
                                ctypes.POINTER(lobpcg_opts), _vp, _vp, _vp],
    "hsym_autotune_geometry": [_i64, _vp, _vp, _vp, _int, _int, _int, _i64, ctypes.POINTER(_int),
                               ctypes.POINTER(hsym_tune_entry), _int, ctypes.POINTER(_int)],
    "hsym_create_append": [_vp, _i64, _vp, _vp, _vp, _int],
    "hsym_create_finish": [_vp],
    "hsym_destroy": [_vp],
    "hsym_info": [_vp, ctypes.POINTER(hsym_info_t)],
    "spmm_sym": [_vp, _int, _vp, _i64, _vp, _i64, _vp],
    "spmm_sym_f32": [_vp, _int, _vp, _i64, _vp, _i64, _vp],
    "lobpcg_opts_default": [ctypes.POINTER(lobpcg_opts)],
    "lobpcg_solve": [_vp, _int, _int, _dbl, _vp, _int, ctypes.POINTER(lobpcg_opts), _vp, _vp,
                     ctypes.POINTER(lobpcg_report), _vp],
    "lanczos_solve": [_vp, _int, _dbl, _vp, ctypes.POINTER(lanczos_opts), _vp, _vp,
                      ctypes.POINTER(lanczos_report), _vp],
    "lobpcg_ctx_create": [ctypes.POINTER(_vp), _vp, _int, _int, _dbl, _vp, _int,
                          ctypes.POINTER(lobpcg_opts), _vp],
    "lobpcg_ctx_step": [ctypes.POINTER(_vp), _int, _int],
    "lobpcg_ctx_status": [_vp, ctypes.POINTER(_int), _vp, ctypes.POINTER(lobpcg_report)],
    "lobpcg_ctx_evecs": [_vp, _vp],
    "lobpcg_ctx_device_bytes": [_vp],
    "lobpcg_ctx_destroy": [_vp],
    "hsym_serve_opts_default": [ctypes.POINTER(hsym_serve_opts)],
    "hsym_serve": [ctypes.POINTER(hsym_request), _int, ctypes.POINTER(hsym_serve_opts),
                   ctypes.POINTER(hsym_serve_report)],
    "hsym_serve_sim": [ctypes.POINTER(hsym_request), _int, ctypes.POINTER(hsym_serve_opts), _vp, _vp, _vp, _dbl,
                       ctypes.POINTER(hsym_serve_report)],
    "hsym_last_error": [],
    # step-level entry points (include/hsym_kernels.h)
    "hsym_kernel_gram": [_i64, _int, _int, _vp, _int, _vp, _vp, _vp],
    "hsym_kernel_gram_noalloc": [_i64, _int, _int, _vp, _int, _vp, _vp, _vp],
    "hsym_kernel_lincomb": [_i64, _int, _int, _vp, _int, _vp, _vp, _int, _vp],
    "hsym_kernel_rayleigh_ritz": [_int, _int, _vp, _vp, _vp, _vp, ctypes.POINTER(_int), _vp],
    "hsym_kernel_precond": [_vp, _int, _int, _vp, _vp, _dbl, _vp],
    "hsym_kernel_orthonormalize": [_i64, _int, _vp, _int, _vp, ctypes.c_uint64, ctypes.POINTER(_int), _vp],
}


def lib():
    """Load libhsym.so (raises if it is not built: no fallback exists)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError("libhsym.so is not built (run __graft_entry__.build() or "
                           "python paper_1609_01689_amd/build.py); there is no CPU fallback")
    L = ctypes.CDLL(LIB_PATH)
    for name, args in _SIGS.items():
        if not hasattr(L, name):
            continue
        f = getattr(L, name)
        f.argtypes = args
        f.restype = _int
    L.hsym_last_error.restype = ctypes.c_char_p
    if hasattr(L, "lobpcg_opts_default"):
        L.lobpcg_opts_default.restype = None
    if hasattr(L, "lobpcg_ctx_device_bytes"):
        L.lobpcg_ctx_device_bytes.restype = _i64
    if hasattr(L, "hsym_serve_opts_default"):
        L.hsym_serve_opts_default.restype = None
    _lib = L
    return L


def exported_symbols():
    return sorted(_SIGS)


def _check(st):
    if st < 0:
        raise HsymError(st, lib().hsym_last_error().decode())
    return st


def _dptr(t):
    """Device pointer of a torch tensor (None -> NULL)."""
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _hptr(a):
    return None if a is None else ctypes.c_void_p(a.ctypes.data)


def _stream(stream):
    if stream is None:
        import torch
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream)


# ---------------------------------------------------------------------------
# thin wrappers
# ---------------------------------------------------------------------------

def hsym_create(n, rowptr, colind, values, storage=HSYM_FP64, flags=0, stream=None):
    """Device handle from host upper-triangle CSR (numpy arrays)."""
    rowptr = np.ascontiguousarray(rowptr, np.int64)
    colind = np.ascontiguousarray(colind, np.int32)
    values = np.ascontiguousarray(values)
    vp = {np.dtype(np.float64): HSYM_FP64, np.dtype(np.float32): HSYM_FP32}[values.dtype]
    h = ctypes.c_void_p()
    _check(lib().hsym_create(ctypes.byref(h), int(n), _hptr(rowptr), _hptr(colind), _hptr(values), vp,
                             storage, flags, _stream(stream)))
    return h


def hsym_create_device(n, rowptr, colind, values, storage=HSYM_FP64, flags=0, stream=None):
    """Device handle from upper-triangle CSR held in device tensors (int64, int32, fp64/fp32)."""
    vp = {"torch.float64": HSYM_FP64, "torch.float32": HSYM_FP32}[str(values.dtype)]
    h = ctypes.c_void_p()
    _check(lib().hsym_create(ctypes.byref(h), int(n), ctypes.c_void_p(rowptr.data_ptr()),
                             ctypes.c_void_p(colind.data_ptr()), ctypes.c_void_p(values.data_ptr()), vp,
                             storage, flags | HSYM_DEVICE_PTRS, _stream(stream)))
    return h


def hsym_autotune_geometry(n, rowptr, colind, values, storage=HSYM_FP64, m=16, sample_rows=0):
    """Fastest panel geometry for width m on a row sample: (flags, [(R, C, ms), ...])."""
    rowptr = np.ascontiguousarray(rowptr, np.int64)
    colind = np.ascontiguousarray(colind, np.int32)
    values = np.ascontiguousarray(values)
    vp = {np.dtype(np.float64): HSYM_FP64, np.dtype(np.float32): HSYM_FP32}[values.dtype]
    cap = 64
    table = (hsym_tune_entry * cap)()
    flags, ntried = _int(0), _int(0)
    _check(lib().hsym_autotune_geometry(int(n), _hptr(rowptr), _hptr(colind), _hptr(values), vp, storage, int(m),
                                        int(sample_rows), ctypes.byref(flags), table, cap, ctypes.byref(ntried)))
    rows = [(table[i].panel_rows, table[i].chunk_cols, table[i].ms) for i in range(min(ntried.value, cap))]
    return flags.value, rows


def hsym_attach_group_tiles(h, group_start, csr):
    """Diagonal group tiles (FOM preconditioner) from ascending group boundaries [0, ..., n]."""
    gs = np.ascontiguousarray(group_start, np.int64)
    rowptr = np.ascontiguousarray(csr.rowptr, np.int64)
    colind = np.ascontiguousarray(csr.colind, np.int32)
    values = np.ascontiguousarray(csr.values)
    vp = {np.dtype(np.float64): HSYM_FP64, np.dtype(np.float32): HSYM_FP32}[values.dtype]
    _check(lib().hsym_attach_group_tiles(h, len(gs) - 1, _hptr(gs), _hptr(rowptr), _hptr(colind), _hptr(values), vp))


def hsym_create_begin(n, storage=HSYM_FP64, flags=0, stream=None):
    h = ctypes.c_void_p()
    _check(lib().hsym_create_begin(ctypes.byref(h), int(n), storage, flags, _stream(stream)))
    return h


def hsym_create_append(h, rowptr_local, colind, values):
    rowptr_local = np.ascontiguousarray(rowptr_local, np.int64)
    colind = np.ascontiguousarray(colind, np.int32)
    values = np.ascontiguousarray(values)
    vp = {np.dtype(np.float64): HSYM_FP64, np.dtype(np.float32): HSYM_FP32}[values.dtype]
    _check(lib().hsym_create_append(h, len(rowptr_local) - 1, _hptr(rowptr_local), _hptr(colind),
                                    _hptr(values), vp))


def hsym_create_finish(h):
    _check(lib().hsym_create_finish(h))


def hsym_destroy(h):
    _check(lib().hsym_destroy(h))


def hsym_info(h):
    info = hsym_info_t()
    _check(lib().hsym_info(h, ctypes.byref(info)))
    return {f: getattr(info, f) for f, _ in hsym_info_t._fields_}


def spmm_sym(h, X, Y, stream=None):
    """Y = H X on fp64 device tensors (n x m, row-major, any ld >= m via stride)."""
    m = X.shape[1] if X.dim() == 2 else 1
    ldx = X.stride(0) if X.dim() == 2 else 1
    ldy = Y.stride(0) if Y.dim() == 2 else 1
    return _check(lib().spmm_sym(h, m, _dptr(X), ldx, _dptr(Y), ldy, _stream(stream)))


def spmm_sym_f32(h, X, Y, stream=None):
    m = X.shape[1] if X.dim() == 2 else 1
    ldx = X.stride(0) if X.dim() == 2 else 1
    ldy = Y.stride(0) if Y.dim() == 2 else 1
    return _check(lib().spmm_sym_f32(h, m, _dptr(X), ldx, _dptr(Y), ldy, _stream(stream)))


def default_lobpcg_opts(**kw):
    o = lobpcg_opts()
    lib().lobpcg_opts_default(ctypes.byref(o))
    for k, v in kw.items():
        setattr(o, k, v)
    return o


def lobpcg_solve(h, nev, block_width, tol, X0=None, precond="jacobi", opts=None, evecs=None,
                 stream=None):
    """Returns (status, evals numpy[nev], report)."""
    evals = np.zeros(nev, np.float64)
    rep = lobpcg_report()
    o = opts if opts is not None else default_lobpcg_opts()
    st = _check(lib().lobpcg_solve(h, nev, block_width, float(tol), _dptr(X0), PRECOND[precond],
                                   ctypes.byref(o), _hptr(evals), _dptr(evecs), ctypes.byref(rep),
                                   _stream(stream)))
    return st, evals, rep


def lobpcg_guess_multilevel(csr, level, caps, X0, m, tol, storage=HSYM_FP64, precond="jacobi", opts=None,
                            stream=None):
    """Eq. 12 start block over the level caps into the device tensor X0 (n x m); returns the
    sub-solves' iteration counts."""
    rowptr = np.ascontiguousarray(csr.rowptr, np.int64)
    colind = np.ascontiguousarray(csr.colind, np.int32)
    values = np.ascontiguousarray(csr.values)
    vp = {np.dtype(np.float64): HSYM_FP64, np.dtype(np.float32): HSYM_FP32}[values.dtype]
    level = np.ascontiguousarray(level, np.int32)
    caps = np.ascontiguousarray(caps, np.int32)
    iters = np.zeros(len(caps), np.int32)
    o = opts if opts is not None else default_lobpcg_opts()
    _check(lib().lobpcg_guess_multilevel(int(csr.n), _hptr(rowptr), _hptr(colind), _hptr(values), vp,
                                         _hptr(level), len(caps), _hptr(caps), storage, int(m), float(tol),
                                         PRECOND[precond], ctypes.byref(o), _dptr(X0), _hptr(iters),
                                         _stream(stream)))
    return iters


def lanczos_solve(h, nev, tol, v0=None, maxit=2000, seed=0, evecs=None, stream=None):
    evals = np.zeros(nev, np.float64)
    rep = lanczos_report()
    o = lanczos_opts(maxit, seed)
    st = _check(lib().lanczos_solve(h, nev, float(tol), _dptr(v0), ctypes.byref(o), _hptr(evals),
                                    _dptr(evecs), ctypes.byref(rep), _stream(stream)))
    return st, evals, rep


def lobpcg_ctx_create(h, nev, block_width, tol, X0=None, precond="jacobi", opts=None, stream=None):
    c = ctypes.c_void_p()
    o = opts if opts is not None else default_lobpcg_opts()
    _check(lib().lobpcg_ctx_create(ctypes.byref(c), h, nev, block_width, float(tol), _dptr(X0),
                                   PRECOND[precond], ctypes.byref(o), _stream(stream)))
    return c


def lobpcg_ctx_step(ctxs, iters=1):
    arr = (ctypes.c_void_p * len(ctxs))(*[c.value for c in ctxs])
    return _check(lib().lobpcg_ctx_step(arr, len(ctxs), iters))


def lobpcg_ctx_status(c, nev):
    done = ctypes.c_int()
    evals = np.zeros(nev, np.float64)
    rep = lobpcg_report()
    st = _check(lib().lobpcg_ctx_status(c, ctypes.byref(done), _hptr(evals), ctypes.byref(rep)))
    return done.value, st, evals, rep


def lobpcg_ctx_evecs(c, evecs):
    return _check(lib().lobpcg_ctx_evecs(c, _dptr(evecs)))


def lobpcg_ctx_device_bytes(c):
    return lib().lobpcg_ctx_device_bytes(c)


def lobpcg_ctx_destroy(c):
    return _check(lib().lobpcg_ctx_destroy(c))


def _ptr_array(tensors):
    return (ctypes.c_void_p * max(1, len(tensors)))(*[t.data_ptr() for t in tensors])


def hsym_kernel_gram(A, B, G, stream=None):
    """G = [A...]^T [B...] for lists of n x m fp64 device tensors."""
    n, m = A[0].shape
    return _check(lib().hsym_kernel_gram(n, m, len(A), _ptr_array(A), len(B), _ptr_array(B), _dptr(G),
                                         _stream(stream)))


def hsym_kernel_gram_noalloc(A, B, G, stream=None):
    """hsym_kernel_gram with its partials in the library's static device
    scratch (no allocation; asynchronous on `stream`)."""
    n, m = A[0].shape
    return _check(lib().hsym_kernel_gram_noalloc(n, m, len(A), _ptr_array(A), len(B), _ptr_array(B), _dptr(G),
                                                 _stream(stream)))


def hsym_kernel_lincomb(In, Out, C, stream=None):
    n, m = In[0].shape
    return _check(lib().hsym_kernel_lincomb(n, m, len(In), _ptr_array(In), len(Out), _ptr_array(Out), _dptr(C),
                                            C.stride(0), _stream(stream)))


def hsym_kernel_rayleigh_ritz(nblk, m, G, theta, evals, coef, stream=None):
    """Rayleigh-Ritz on a basis S given G = [S^T S | S^T A S] (k x 2k device
    fp64); returns 1 when the third block was dropped, else 0."""
    dropped = _int(0)
    _check(lib().hsym_kernel_rayleigh_ritz(nblk, m, _dptr(G), _dptr(theta), _dptr(evals), _dptr(coef),
                                           ctypes.byref(dropped), _stream(stream)))
    return dropped.value


def hsym_kernel_precond(h, kind, W, mu, delta, stream=None):
    return _check(lib().hsym_kernel_precond(h, PRECOND[kind], W.shape[1], _dptr(W), _dptr(mu), float(delta),
                                            _stream(stream)))


def hsym_kernel_orthonormalize(V, B=(), seed=0, stream=None):
    n, m = V.shape
    rep = ctypes.c_int()
    _check(lib().hsym_kernel_orthonormalize(n, m, _dptr(V), len(B), _ptr_array(list(B)) if B else None,
                                            seed, ctypes.byref(rep), _stream(stream)))
    return rep.value


def _serve_opts(budget_bytes=0, max_active=0, iters_per_round=0, maxit=0, autotune=False, loaders=0):
    o = hsym_serve_opts()
    lib().hsym_serve_opts_default(ctypes.byref(o))
    o.autotune = 1 if autotune else 0
    if loaders:
        o.loaders = int(loaders)
    if budget_bytes:
        o.budget_bytes = int(budget_bytes)
    if max_active:
        o.max_active = int(max_active)
    if iters_per_round:
        o.iters_per_round = int(iters_per_round)
    if maxit:
        o.maxit = int(maxit)
    return o


def _serve_results(arr, count, rep):
    out = []
    for i in range(count):
        r = arr[i]
        out.append({"status": r.status, "iters": r.iters, "evals": np.array(r.evals[:r.nev]),
                    "arrival_s": r.arrival_s, "admit_s": r.admit_s, "finish_s": r.finish_s,
                    "latency_s": r.finish_s - r.arrival_s, "device_bytes": r.device_bytes,
                    "error": r.error.decode(errors="replace")})
    return out, {f: getattr(rep, f) for f, _ in hsym_serve_report._fields_}


def hsym_serve(requests, **opts):
    """Run a request trace through the device request loop.

    requests: list of dicts with keys csr (hsymgen.UpperCSR-like: n, rowptr,
    colind, values), storage, nev, block_width, precond, tol, seed,
    arrival_s.  Returns (per-request result dicts, report dict)."""
    keep = []
    arr = (hsym_request * max(1, len(requests)))()
    for i, q in enumerate(requests):
        A = q["csr"]
        rp = np.ascontiguousarray(A.rowptr, np.int64)
        ci = np.ascontiguousarray(A.colind, np.int32)
        va = np.ascontiguousarray(A.values)
        keep += [rp, ci, va]
        r = arr[i]
        r.n, r.rowptr, r.colind, r.values = int(A.n), rp.ctypes.data, ci.ctypes.data, va.ctypes.data
        r.values_prec = HSYM_FP32 if va.dtype == np.float32 else HSYM_FP64
        r.storage = int(q.get("storage", HSYM_FP64))
        r.nev, r.block_width = int(q["nev"]), int(q["block_width"])
        r.precond = PRECOND[q.get("precond", "jacobi")]
        r.tol, r.seed, r.arrival_s = float(q["tol"]), int(q.get("seed", 0)), float(q["arrival_s"])
    rep = hsym_serve_report()
    o = _serve_opts(**opts)
    _check(lib().hsym_serve(arr, len(requests), ctypes.byref(o), ctypes.byref(rep)))
    return _serve_results(arr, len(requests), rep)


def hsym_serve_sim(arrival_s, iters, iter_s, nbytes, load_s, nev=1, **opts):
    """The request loop's scheduler on a virtual clock (no device)."""
    k = len(arrival_s)
    arr = (hsym_request * max(1, k))()
    for i in range(k):
        arr[i].arrival_s = float(arrival_s[i])
        arr[i].nev = nev
    it = np.ascontiguousarray(iters, np.int32)
    its = np.ascontiguousarray(iter_s, np.float64)
    b = np.ascontiguousarray(nbytes, np.int64)
    rep = hsym_serve_report()
    o = _serve_opts(**opts)
    _check(lib().hsym_serve_sim(arr, k, ctypes.byref(o), _hptr(it), _hptr(its), _hptr(b), float(load_s),
                                ctypes.byref(rep)))
    return _serve_results(arr, k, rep)


class Matrix:
    """Owning wrapper of an hsym handle (create from an upper-triangle CSR)."""

    def __init__(self, csr, storage=HSYM_FP64, block64=False, geom_m=16, stream=None, flags=0):
        flags |= (HSYM_BUILD_BLOCK64 if block64 else 0) | HSYM_GEOM_M(geom_m)
        self.n = csr.n
        self.storage = storage
        self.h = hsym_create(csr.n, csr.rowptr, csr.colind, csr.values, storage, flags, stream)

    @property
    def info(self):
        return hsym_info(self.h)

    def close(self):
        if self.h is not None and self.h.value:
            hsym_destroy(self.h)
        self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
