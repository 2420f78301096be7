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


def test_binding_checks_buffers_before_the_call(libpath):
    """The ABI takes raw pointers, so the binding refuses a wrong dtype, host
    memory where device memory is expected, or a wrong length, before any call
    that could touch a buffer (no GPU is needed to reach these checks)."""
    import numpy as np
    import torch
    from paper_2205_14273_amd import ssamg as B
    pr = B.Problem(3, [(4, 4, 4), (2, 4, 4)], [(0, 0, 0), (4, 0, 0)])
    assert B.ssamg_problem_num_parts(pr.h) == 2
    offs = np.array([[0, 0, 0], [-1, 0, 0], [1, 0, 0], [0, -1, 0], [0, 1, 0], [0, 0, -1], [0, 0, 1]])
    B.ssamg_problem_set_stencil(pr.h, 0, offs)
    assert B.ssamg_problem_part_size(pr.h, 0) == (7, 64)
    assert B.ssamg_problem_part_size(pr.h, 1) == (0, 32)
    with pytest.raises(ValueError):
        B.ssamg_problem_set_coeffs(pr.h, 0, np.ones(7 * 64 + 1))
    with pytest.raises(ValueError):
        B.ssamg_problem_set_coeffs(pr.h, 0, np.ones(6), constant=1)
    with pytest.raises(ValueError):
        B.ssamg_problem_set_coeffs(pr.h, 1, np.ones(7 * 32))        # no stencil yet
    with pytest.raises(TypeError):
        B.ssamg_problem_fv_assemble(pr.h, torch.ones(96, dtype=torch.float64), np.ones((2, 3)), 7)
    with pytest.raises(TypeError):
        B.ssamg_problem_fv_grad(pr.h, torch.ones(96, dtype=torch.float64),
                                torch.ones(96, dtype=torch.float64), torch.ones(96, dtype=torch.float64))
    with pytest.raises(ValueError):
        B.ssamg_problem_set_coupling(pr.h, [0, 1], [64], [1.0])


def test_new_entry_points_validate_without_gpu(libpath):
    """Argument errors of the boundary's newer calls are reported on the host."""
    import ctypes as C
    from paper_2205_14273_amd import _lib
    lib = _lib.lib()
    prob = C.c_void_p()
    assert lib.ssamg_problem_create(3, 2, C.byref(prob)) == _lib.OK
    n = C.c_int()
    assert lib.ssamg_problem_num_parts(prob, C.byref(n)) == _lib.OK and n.value == 2
    ne, nc = C.c_int(), C.c_int64()
    assert lib.ssamg_problem_part_size(prob, 5, C.byref(ne), C.byref(nc)) == _lib.ERR_ARG
    # bad memory kind for the couplings
    assert lib.ssamg_problem_set_coupling(prob, 0, None, None, None, 7) == _lib.ERR_ARG
    p = _lib.ssamg_params()
    lib.ssamg_params_default(C.byref(p))
    assert p.pb_interp == _lib.PB_ONE
    p.pb_interp = 3
    s = C.c_void_p()
    assert lib.ssamg_solver_create(prob, C.byref(p), None, C.byref(s)) == _lib.ERR_ARG
    assert b"pb_interp" in lib.ssamg_last_error()
    assert lib.ssamg_problem_destroy(prob) == _lib.OK


def test_binding_constants_match_the_header():
    """Every enumerator and every ssamg_params field of the header has its
    twin in the binding, with the same value and in the same order."""
    from paper_2205_14273_amd import _lib
    text = re.sub(r"/\*.*?\*/", "", open(HEADER).read(), flags=re.S)
    enums = re.findall(r"\bSSAMG_([A-Z0-9_]+)\s*=\s*(-?\d+)", text)
    assert len(enums) > 20
    for name, val in enums:
        assert getattr(_lib, name) == int(val), name
    body = re.search(r"typedef struct \{([^}]*)\} ssamg_params;", text, flags=re.S).group(1)
    fields = re.findall(r"\b([a-z_0-9]+)\s*;", body)
    assert [f[0] for f in _lib.ssamg_params._fields_] == fields
