"""ssamg_solve_noalloc: the solve whose PCG vectors and reduction scratch live in
one fixed device array per GPU.  Through the C ABI, two calls in a row (the
second with a smaller problem, then with fewer right-hand sides) must equal
ssamg_solve bit for bit, in both vector layouts; a solve too large for the
array is refused with a clear error."""
import ctypes as C

import numpy as np
import pytest

import workloads as W
from tests.parity_util import gpu_fv

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _cuda(a):
    return torch.as_tensor(np.ascontiguousarray(a), device="cuda", dtype=torch.float64)


def _abi_solve(fn, s, nrhs, b, layout):
    """Call ssamg_solve or ssamg_solve_noalloc directly through ctypes."""
    from paper_2205_14273_amd import _lib as L
    x = torch.full_like(b, float("nan"))
    info = L.ssamg_info()
    st = getattr(L.lib(), fn)(s.h, nrhs, C.c_void_p(b.data_ptr()), C.c_void_p(x.data_ptr()), layout,
                              C.byref(info))
    assert st == 0, (fn, st, L.lib().ssamg_last_error())
    return x, info


def _check_same(s, nrhs, b, layout):
    x0, i0 = _abi_solve("ssamg_solve", s, nrhs, b, layout)
    x1, i1 = _abi_solve("ssamg_solve_noalloc", s, nrhs, b, layout)
    assert torch.equal(x0, x1)
    assert [i0.iters[k] for k in range(nrhs)] == [i1.iters[k] for k in range(nrhs)]
    assert [i0.true_relres[k] for k in range(nrhs)] == [i1.true_relres[k] for k in range(nrhs)]
    assert all(i1.true_relres[k] < 1e-8 for k in range(nrhs))


def test_noalloc_solve_matches_solve_twice_then_smaller():
    from paper_2205_14273_amd import _lib as L
    print("[no alloc] c2_16 fp32 cycle, 4 rhs, then c2_10, then 1 rhs", flush=True)
    big = W.c2(16)
    _, s1 = gpu_fv(big, cycle_precision=1, max_nrhs=4)
    R = np.random.default_rng(41).uniform(-1, 1, (big.geometry.n, 4))
    _check_same(s1, 4, _cuda(R), L.LAYOUT_CELL_MAJOR)
    _check_same(s1, 4, _cuda(R.T), L.LAYOUT_RHS_MAJOR)
    small = W.c2(10)
    _, s2 = gpu_fv(small, cycle_precision=0, max_nrhs=4)
    r2 = np.random.default_rng(42).uniform(-1, 1, (small.geometry.n, 2))
    _check_same(s2, 2, _cuda(r2), L.LAYOUT_CELL_MAJOR)
    _check_same(s2, 1, _cuda(small.b), L.LAYOUT_CELL_MAJOR)
    # the first solver again, after the smaller one used the array
    _check_same(s1, 1, _cuda(big.b), L.LAYOUT_RHS_MAJOR)


def test_noalloc_refuses_a_solve_beyond_the_array():
    from paper_2205_14273_amd import _lib as L
    print("[no alloc] c2 full, 4 rhs: beyond the array", flush=True)
    case = W.c2()
    _, s = gpu_fv(case, max_nrhs=4)
    n = case.geometry.n
    b = torch.zeros(n * 4, dtype=torch.float64, device="cuda")
    x = torch.zeros_like(b)
    info = L.ssamg_info()
    st = L.lib().ssamg_solve_noalloc(s.h, 4, C.c_void_p(b.data_ptr()), C.c_void_p(x.data_ptr()),
                                     L.LAYOUT_CELL_MAJOR, C.byref(info))
    assert st == L.ERR_ARG
    msg = L.lib().ssamg_last_error().decode()
    assert "scratch" in msg and str(L.NOALLOC_SCRATCH_BYTES) in msg
    # one right-hand side of the same problem fits
    x1, _ = _abi_solve("ssamg_solve_noalloc", s, 1, _cuda(case.b), L.LAYOUT_CELL_MAJOR)
    x0, _ = _abi_solve("ssamg_solve", s, 1, _cuda(case.b), L.LAYOUT_CELL_MAJOR)
    assert torch.equal(x0, x1)
