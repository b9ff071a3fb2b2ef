"""The C ABI library loads and exports every symbol the headers declare
(no GPU needed: nothing is called)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_functions():
    names = set()
    for h in ("hsym.h", "hsym_kernels.h"):
        with open(os.path.join(ROOT, "include", h)) as f:
            src = f.read()
        src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
        for m in re.finditer(r"^\s*(?:int|void|const char \*|int64_t)\s*\*?\s*(\w+)\s*\(", src, flags=re.M):
            names.add(m.group(1))
    return sorted(names)


def test_headers_declare_the_boundary():
    names = declared_functions()
    for required in ("hsym_create", "spmm_sym", "lobpcg_solve", "lanczos_solve", "lobpcg_ctx_step",
                     "hsym_kernel_gram", "hsym_last_error"):
        assert required in names


def test_library_exports_every_declared_symbol():
    import paper_1609_01689_amd as hs
    if not os.path.exists(hs.LIB_PATH):
        pytest.skip("library not built")
    lib = ctypes.CDLL(hs.LIB_PATH)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing
    # the Python binding marshals exactly the declared names
    assert set(declared_functions()) <= set(hs.exported_symbols()) | {"lobpcg_opts_default"}


def test_binding_fails_loudly_without_library(tmp_path, monkeypatch):
    import paper_1609_01689_amd as hs
    monkeypatch.setattr(hs, "LIB_PATH", str(tmp_path / "missing.so"))
    monkeypatch.setattr(hs, "_lib", None)
    with pytest.raises(RuntimeError, match="no CPU fallback"):
        hs.lib()
