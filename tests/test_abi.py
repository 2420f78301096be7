"""The C ABI without a GPU: the shared library loads and exports every function
that include/ssamg.h declares, the ctypes binding declares the same set, and the
Python layer fails loudly (no fallback) when the library is missing."""
import ctypes as C
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "ssamg.h")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(ssamg_[A-Za-z0-9_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def libpath():
    from paper_2205_14273_amd import _build, _lib
    if not os.path.exists(_lib.LIB_PATH):
        _build.build()
    return _lib.LIB_PATH


def test_header_declares_the_boundary():
    names = _declared()
    for must in ("ssamg_problem_create", "ssamg_problem_fv_assemble", "ssamg_problem_fv_grad",
                 "ssamg_setup_symbolic", "ssamg_setup_numeric", "ssamg_solve",
                 "ssamg_apply_A", "ssamg_apply_precond", "ssamg_last_error"):
        assert must in names


def test_library_exports_every_declared_symbol(libpath):
    h = C.CDLL(libpath)
    missing = [n for n in _declared() if not hasattr(h, n)]
    assert not missing, missing


def test_binding_covers_the_header():
    from paper_2205_14273_amd import _lib
    assert sorted(_lib.SIGNATURES) == _declared()


def test_last_error_without_gpu(libpath):
    """A call that fails argument checks before touching the device reports a
    status and a message; no GPU is needed for it."""
    from paper_2205_14273_amd import _lib
    lib = _lib.lib()
    out = C.c_void_p()
    assert lib.ssamg_problem_create(5, 1, C.byref(out)) == _lib.ERR_ARG
    assert b"ndim" in lib.ssamg_last_error() or len(lib.ssamg_last_error()) > 0
    assert lib.ssamg_problem_create(3, 0, C.byref(out)) == _lib.ERR_ARG
    p = _lib.ssamg_params()
    assert lib.ssamg_params_default(C.byref(p)) == _lib.OK
    assert p.max_levels == 64 and p.max_nrhs == 1 and p.tol == 1e-8 and p.use_graph == 1


def test_missing_library_fails_loudly(monkeypatch, tmp_path):
    from paper_2205_14273_amd import _lib
    monkeypatch.setattr(_lib, "_lib", None)
    monkeypatch.setattr(_lib, "LIB_PATH", str(tmp_path / "libssamg.so"))
    with pytest.raises(ImportError):
        _lib.lib()
