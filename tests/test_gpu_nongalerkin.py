"""The non-Galerkin coarse operator (coarse_op = SSAMG_COARSE_OP_NONGALERKIN; the
option Section 5 plans for isotropic problems, reading R-ng of the oracle) on
the device against the oracle: every level element by element with both
Galerkin kernel layouts (bit for bit against each other), the V-cycle entry by
entry in FP64 and FP32, and PCG iterations; parts whose stencil is not a star
stay Galerkin."""
import numpy as np
import pytest

import workloads as W
from oracle import ssamg as O
from tests.parity_util import (CYCLE_RTOL, assert_cycle_close, compare_hierarchy, gpu_fv, gpu_raw,
                               oracle_fv, oracle_raw, vcycle_scale)

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

NG = 1   # SSAMG_COARSE_OP_NONGALERKIN


def _cuda(a):
    return torch.as_tensor(np.ascontiguousarray(a), device="cuda", dtype=torch.float64)


def _raw():
    g = W.Geometry(3, [(12, 9, 8), (10, 9, 8), (7, 6, 8)], [(0, 0, 0), (12, 0, 0), (12, 9, 0)])
    return W.random_link_case(21, g, 7)


CASES = {"c1_24": lambda: W.c1(24), "c5_13": lambda: W.c5(13), "c2_18": lambda: W.c2(18), "raw": _raw}


def _pair(name, **params):
    case = CASES[name]()
    if name == "raw":
        return case, oracle_raw(case, coarse_op="nongalerkin"), gpu_raw(case, coarse_op=NG, **params)[1]
    return case, oracle_fv(case, coarse_op="nongalerkin"), gpu_fv(case, coarse_op=NG, **params)[1]


@pytest.mark.parametrize("name", list(CASES))
def test_nongalerkin_hierarchy_both_kernels(monkeypatch, name):
    print(f"[gpu nongalerkin] hierarchy {name}", flush=True)
    monkeypatch.setenv("SSAMG_RAP_CELL_MIN", "0")
    case, h, s_cell = _pair(name)
    nparts = len(h.levels[0].dims)
    compare_hierarchy(h, s_cell, nparts)
    assert all(len(lev.pattern[p]) <= 7 for lev in h.levels for p in range(nparts))
    monkeypatch.setenv("SSAMG_RAP_CELL_MIN", str(1 << 40))
    _, _, s_ent = _pair(name)
    for l in range(1, h.nlevels):
        for p in range(nparts):
            assert np.array_equal(s_cell.copy_stencil(l, p), s_ent.copy_stencil(l, p)), (l, p)


@pytest.mark.parametrize("precision", [0, 1])
@pytest.mark.parametrize("name", list(CASES))
def test_nongalerkin_cycle_and_solve(name, precision):
    print(f"[gpu nongalerkin] cycle {name} precision={precision}", flush=True)
    case, h, s = _pair(name, cycle_precision=precision)
    r = np.random.default_rng(23).uniform(-1, 1, h.levels[0].n)
    z = s.apply_precond(_cuda(r)).cpu().numpy()
    assert_cycle_close(z, O.vcycle(h, r), vcycle_scale(h, r), CYCLE_RTOL[precision], name)
    b = case.b if case.b.ndim == 1 else case.b[0]
    ref = O.solve(h, b, tol=1e-8, flexible=(precision == 1))
    x, st, info = s.solve(_cuda(b))
    assert st == 0 and abs(info.iters[0] - ref.iters) <= 1, (info.iters[0], ref.iters)
    assert info.true_relres[0] < 1e-8
    assert np.linalg.norm(x.cpu().numpy() - ref.x) <= 1e-6 * np.linalg.norm(ref.x)


def test_nongalerkin_leaves_27_point_parts_galerkin():
    """A 27-point stencil is not a star: the option gives the Galerkin
    hierarchy bit for bit."""
    print("[gpu nongalerkin] 27-point unchanged", flush=True)
    case = W.c3(9)
    _, s_ng = gpu_fv(case, coarse_op=NG)
    _, s_g = gpu_fv(case)
    assert s_ng.nlevels == s_g.nlevels
    for l in range(s_g.nlevels):
        for p in range(case.geometry.nparts):
            assert np.array_equal(s_ng.copy_stencil(l, p), s_g.copy_stencil(l, p)), (l, p)


def test_coarse_op_is_checked():
    from paper_2205_14273_amd.ssamg import SSAMGError
    with pytest.raises(SSAMGError) as e:
        gpu_fv(W.c1(6), coarse_op=2)
    assert e.value.status == -1
