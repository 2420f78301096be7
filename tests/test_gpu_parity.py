"""Parity of the HIP path (through the C ABI) against the CPU oracle.

Integer results (levels, d*, boxes, stencil patterns, coupling structure) must
match bit for bit; coarse operators, weights and couplings to a row-relative
1e-12; solves to a relative residual of 1e-8 with the oracle's iteration count
+-1.  Sizes span several 256-cell tiles with ragged tails and odd extents.
"""
import math

import numpy as np
import pytest
import scipy.linalg as sla

import workloads as W
from oracle import assemble, ssamg as O
from tests.parity_util import (CYCLE_RTOL, assert_cycle_close, compare_hierarchy, gpu_fv, gpu_raw,
                               oracle_fv, oracle_raw, row_rel_err, vcycle_scale)

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

CASES = {
    "c1_16": lambda: W.c1(16),
    "c2_13": lambda: W.c2(13),
    "c2_20": lambda: W.c2(20),
    "c3_9": lambda: W.c3(9),
    "c4_12": lambda: W.c4(12, nrhs=1),
    "c5_11": lambda: W.c5(11),
}


def _cuda(a):
    return torch.as_tensor(np.ascontiguousarray(a), device="cuda", dtype=torch.float64)


def _print_case(name):
    print(f"[gpu parity] case {name}", flush=True)


@pytest.mark.parametrize("name", list(CASES))
def test_hierarchy_parity(name):
    _print_case(name)
    case = CASES[name]()
    h = oracle_fv(case)
    pr, s = gpu_fv(case)
    # direction sums of Section 3.1 (device reduction vs correctly rounded sums)
    cd = s.direction_sums()
    assert np.allclose(cd, h.cd, rtol=1e-12, atol=0)
    compare_hierarchy(h, s, case.geometry.nparts)


@pytest.mark.parametrize("name", ["c1_16", "c2_20", "c3_9", "c5_11"])
def test_matvec_parity_every_level(name):
    _print_case(name)
    case = CASES[name]()
    h = oracle_fv(case)
    pr, s = gpu_fv(case)
    rng = np.random.default_rng(7)
    for l, lev in enumerate(h.levels):
        x = rng.standard_normal(lev.n)
        y = s.apply_A(l, _cuda(x)).cpu().numpy()
        want = lev.A @ x
        scale = np.abs(lev.A) @ np.abs(x)
        assert np.max(np.abs(y - want) / np.maximum(scale, 1e-300)) <= 1e-13, l


@pytest.mark.parametrize("name", ["c1_16", "c2_20", "c3_9", "c5_11"])
def test_vcycle_parity(name):
    _print_case(name)
    case = CASES[name]()
    h = oracle_fv(case)
    pr, s = gpu_fv(case)
    r = np.random.default_rng(3).uniform(-1, 1, h.levels[0].n)
    z = s.apply_precond(_cuda(r)).cpu().numpy()
    want = O.vcycle(h, r)
    assert_cycle_close(z, want, vcycle_scale(h, r), CYCLE_RTOL[0], name)


@pytest.mark.parametrize("name", list(CASES))
def test_solve_parity(name):
    _print_case(name)
    case = CASES[name]()
    h = oracle_fv(case)
    b = case.b if case.b.ndim == 1 else case.b[0]
    ref = O.solve(h, b, tol=1e-8)
    pr, s = gpu_fv(case)
    x, st, info = s.solve(_cuda(b))
    assert st == 0
    assert abs(info.iters[0] - ref.iters) <= 1, (info.iters[0], ref.iters)
    assert info.relres[0] < 1e-8 and info.true_relres[0] < 1e-8
    xn = x.cpu().numpy()
    tr = np.linalg.norm(b - h.levels[0].A @ xn) / np.linalg.norm(b)
    assert tr < 1e-8
    assert np.linalg.norm(xn - ref.x) <= 1e-6 * np.linalg.norm(ref.x)


def test_solve_matches_dense_direct():
    case = W.c3(5)
    A, _ = assemble.assemble_fv(case.geometry, 27, case.kappa, case.aniso)
    pr, s = gpu_fv(case, tol=1e-12)
    x, st, info = s.solve(_cuda(case.b))
    xd = sla.solve(A.toarray(), case.b, assume_a="pos")
    assert np.linalg.norm(x.cpu().numpy() - xd) <= 1e-9 * np.linalg.norm(xd)


@pytest.mark.parametrize("seed,kind", [(1, 7), (2, 27), (3, 27)])
def test_raw_problem_parity(seed, kind):
    g = W.Geometry(3, [(9, 7, 5), (6, 7, 5), (5, 4, 6)], [(0, 0, 0), (9, 0, 0), (9, 7, 0)])
    case = W.random_link_case(seed, g, kind, junk_outside=True)
    h = oracle_raw(case)
    pr, s = gpu_raw(case)
    compare_hierarchy(h, s, g.nparts)
    ref = O.solve(h, case.b, tol=1e-8)
    x, st, info = s.solve(_cuda(case.b))
    assert st == 0 and abs(info.iters[0] - ref.iters) <= 1


def test_collapse_fallback_parity():
    from tests.test_oracle_pins import den_fallback_case
    case = den_fallback_case()
    h = oracle_raw(case)
    pr, s = gpu_raw(case)
    compare_hierarchy(h, s, 1)
    wm, wp = s.copy_interp(0, 0)
    assert wm[1] == pytest.approx(0.75, abs=1e-15) and wp[1] == pytest.approx(0.25, abs=1e-15)


def test_raw_2d_problem_parity():
    g = W.Geometry(2, [(17, 11, 1), (9, 11, 1)], [(0, 0, 0), (17, 0, 0)])
    case = W.random_link_case(5, g, 9)
    h = oracle_raw(case)
    pr, s = gpu_raw(case)
    compare_hierarchy(h, s, g.nparts)
    ref = O.solve(h, case.b, tol=1e-8)
    x, st, info = s.solve(_cuda(case.b))
    assert st == 0 and abs(info.iters[0] - ref.iters) <= 1


def test_max_levels_and_min_coarse_size():
    case = W.c2(12)
    for kw in ({"max_levels": 4}, {"min_coarse_size": 300}):
        h = oracle_fv(case, **kw)
        pr, s = gpu_fv(case, **kw)
        compare_hierarchy(h, s, 4)
        ref = O.solve(h, case.b, tol=1e-8)
        x, st, info = s.solve(_cuda(case.b))
        assert st == 0 and abs(info.iters[0] - ref.iters) <= 1


@pytest.mark.parametrize("precision", [0, 1])
def test_large_coarsest_level(precision):
    """max_levels = 2 leaves a coarsest level of 16000 cells, too large for the
    LDS-resident coarse end: it runs as a grid kernel on global vectors (one
    sweep from zero), and the cycle and the solve still match the oracle."""
    _print_case(f"large coarsest precision={precision}")
    case = W.c2(20)
    h = oracle_fv(case, max_levels=2)
    pr, s = gpu_fv(case, max_levels=2, cycle_precision=precision)
    assert s.nlevels == 2 and s.level_cells(1) == 16000
    r = np.random.default_rng(12).uniform(-1, 1, h.levels[0].n)
    z = s.apply_precond(_cuda(r)).cpu().numpy()
    want = O.vcycle(h, r)
    assert_cycle_close(z, want, vcycle_scale(h, r), CYCLE_RTOL[precision])
    ref = O.solve(h, case.b, tol=1e-8)
    x, st, info = s.solve(_cuda(case.b))
    assert st == 0 and abs(info.iters[0] - ref.iters) <= 1


def test_solution_buffer_not_16_byte_aligned():
    """x may be any float64 buffer: a view one element into a larger one (8-byte
    aligned only) takes the one-element-per-thread update and gives the same
    solution bitwise."""
    _print_case("unaligned x")
    case = W.c2(9)
    _, s = gpu_fv(case, cycle_precision=1)
    b = _cuda(case.b)
    x0, st0, i0 = s.solve(b)
    buf = torch.zeros(b.numel() + 1, dtype=torch.float64, device="cuda")
    xv = buf[1:]
    assert xv.data_ptr() % 16 == 8
    x1, st1, i1 = s.solve(b, x=xv)
    assert st0 == st1 == 0 and i0.iters[0] == i1.iters[0]
    assert torch.equal(x0, x1)


def test_single_cell_parts():
    # degenerate: every part is one cell, the hierarchy has one level
    g = W.Geometry(3, [(1, 1, 1)] * 3, [(0, 0, 0), (1, 0, 0), (2, 0, 0)])
    case = W.FVCase("t", g, 7, np.array([1.0, 2.0, 3.0]), np.ones((3, 3)), np.array([1.0, -1.0, 0.5]))
    h = oracle_fv(case)
    pr, s = gpu_fv(case)
    assert s.nlevels == 1 == h.nlevels
    ref = O.solve(h, case.b, tol=1e-10)
    x, st, info = s.solve(_cuda(case.b))
    assert np.allclose(x.cpu().numpy(), ref.x, rtol=1e-12)


def test_zero_rhs():
    pr, s = gpu_fv(W.c1(8))
    x, st, info = s.solve(torch.zeros(512, dtype=torch.float64, device="cuda"))
    assert st == 0 and info.iters[0] == 0 and float(x.abs().max()) == 0.0


def test_not_converged_status():
    pr, s = gpu_fv(W.c2(12), max_iter=2)
    x, st, info = s.solve(_cuda(W.c2(12).b))
    assert st == 1 and info.iters[0] == 2 and not info.converged[0]


def test_errors_are_reported():
    from paper_2205_14273_amd import ssamg as B
    from paper_2205_14273_amd._lib import SSAMGError
    pr = B.Problem(3, [(4, 4, 4)])
    B.ssamg_problem_set_stencil(pr.h, 0, W.stencil_offsets(7))
    bad = np.ones((7, 64))
    bad[0, 5] = -1.0      # nonpositive diagonal
    with pytest.raises(SSAMGError) as e:
        B.ssamg_problem_set_coeffs(pr.h, 0, bad)
    assert e.value.status == -4
    s = B.Solver(pr)
    with pytest.raises(SSAMGError) as e:
        B.ssamg_solve(s.h, 1, torch.zeros(64, dtype=torch.float64, device="cuda"),
                      torch.zeros(64, dtype=torch.float64, device="cuda"))
    assert e.value.status == -2
    with pytest.raises(SSAMGError) as e:
        B.ssamg_problem_set_coupling(pr.h, [0], [1], [1.0])   # same part
    assert e.value.status == -1


def test_nan_rhs_is_an_error():
    from paper_2205_14273_amd._lib import SSAMGError
    pr, s = gpu_fv(W.c1(6))
    b = torch.ones(216, dtype=torch.float64, device="cuda")
    b[3] = float("nan")
    with pytest.raises(SSAMGError) as e:
        s.solve(b)
    assert e.value.status == -4


def test_repeatable_bitwise():
    case = W.c3(7)
    pr, s = gpu_fv(case)
    x1, _, i1 = s.solve(_cuda(case.b))
    x2, _, i2 = s.solve(_cuda(case.b))
    assert torch.equal(x1, x2) and i1.iters[0] == i2.iters[0]


def test_graph_and_eager_agree():
    case = W.c2(14)
    pr, s1 = gpu_fv(case, use_graph=1)
    _, s2 = gpu_fv(case, use_graph=0)
    b = _cuda(case.b)
    for _ in range(3):   # replay the captured cycle several times with eager work between
        z1 = s1.apply_precond(b)
        z2 = s2.apply_precond(b)
        torch.cuda.synchronize()
        assert torch.equal(z1, z2)


@pytest.mark.parametrize("precision", [0, 1])
def test_tail_kernel_matches_grid_kernels(monkeypatch, precision):
    """The one-workgroup coarse-end kernel (vectors and descriptors in LDS; the
    levels of up to 4096 elements that fit, set through SSAMG_TAIL_ELEMS) gives
    the V-cycle of the per-level grid kernels (SSAMG_TAIL_ELEMS=0: the coarsest
    level only), for one and for eight right-hand sides; both match the
    oracle's cycle."""
    _print_case(f"tail precision={precision}")
    case = W.c2(13)
    h = oracle_fv(case)
    r = np.random.default_rng(8).uniform(-1, 1, h.levels[0].n)
    monkeypatch.setenv("SSAMG_TAIL_ELEMS", "0")
    _, s0 = gpu_fv(case, cycle_precision=precision, max_nrhs=8)
    monkeypatch.setenv("SSAMG_TAIL_ELEMS", "4096")
    _, s1 = gpu_fv(case, cycle_precision=precision, max_nrhs=8)
    z0 = s0.apply_precond(_cuda(r)).cpu().numpy()
    z1 = s1.apply_precond(_cuda(r)).cpu().numpy()
    want = O.vcycle(h, r)
    scale = vcycle_scale(h, r)
    assert_cycle_close(z1, z0, scale, CYCLE_RTOL[precision], "tail vs grid")
    assert_cycle_close(z1, want, scale, CYCLE_RTOL[precision], "tail vs oracle")
    R = np.random.default_rng(9).uniform(-1, 1, (h.levels[0].n, 8))
    x0, st0, i0 = s0.solve(_cuda(R))
    x1, st1, i1 = s1.solve(_cuda(R))
    assert st0 == st1 == 0
    assert max(abs(i0.iters[k] - i1.iters[k]) for k in range(8)) <= (0 if precision == 0 else 1)
    X0, X1 = x0.cpu().numpy(), x1.cpu().numpy()
    assert np.linalg.norm(X1 - X0) <= 1e-6 * np.linalg.norm(X0)


@pytest.mark.parametrize("cells", ["256", "512"])
@pytest.mark.parametrize("precision", [0, 1])
def test_collapsed_coarse_cycle(monkeypatch, precision, cells):
    """Below the first level of at most SSAMG_COLLAPSE_CELLS cells the cycle is
    one dense matrix formed at setup; the cycle with it matches the cycle
    without it (to rounding), for one and for eight right-hand sides, and the
    oracle's cycle; the solves take the same iterations.  With 512 cells and
    eight right-hand sides the collapse level lies above the coarse-end kernel
    and the matrix is applied by a grid kernel."""
    _print_case(f"collapse precision={precision} cells={cells}")
    case = W.c2(13)
    h = oracle_fv(case)
    r = np.random.default_rng(31).uniform(-1, 1, h.levels[0].n)
    monkeypatch.setenv("SSAMG_COLLAPSE_CELLS", "0")
    _, s0 = gpu_fv(case, cycle_precision=precision, max_nrhs=8)
    monkeypatch.setenv("SSAMG_COLLAPSE_CELLS", cells)
    _, s1 = gpu_fv(case, cycle_precision=precision, max_nrhs=8)
    z0 = s0.apply_precond(_cuda(r)).cpu().numpy()
    z1 = s1.apply_precond(_cuda(r)).cpu().numpy()
    want = O.vcycle(h, r)
    scale = vcycle_scale(h, r)
    assert_cycle_close(z1, z0, scale, CYCLE_RTOL[precision], "collapsed vs full")
    assert_cycle_close(z1, want, scale, CYCLE_RTOL[precision], "collapsed vs oracle")
    R = np.random.default_rng(32).uniform(-1, 1, (h.levels[0].n, 8))
    x0, st0, i0 = s0.solve(_cuda(R))
    x1, st1, i1 = s1.solve(_cuda(R))
    assert st0 == st1 == 0
    assert max(abs(i0.iters[k] - i1.iters[k]) for k in range(8)) <= 1
    X0, X1 = x0.cpu().numpy(), x1.cpu().numpy()
    assert np.linalg.norm(X1 - X0) <= 1e-6 * np.linalg.norm(X0)


@pytest.mark.parametrize("name", ["c2_12", "c3_8"])
def test_host_formed_couplings_match_device(monkeypatch, name):
    """The coupling products of the small coarse levels are formed on the host
    (SSAMG_HOST_SYM records and below): with every level on the device, every
    level on the host and the default split, the hierarchies match the oracle
    and the cycles are bitwise equal.  On the device the records of each
    coarse row are ranked in LDS (rows of at most SSAMG_ROW_SORT records) or
    from memory (SSAMG_ROW_SORT=0: every row); both give the same order."""
    _print_case(f"host couplings {name}")
    case = {"c2_12": lambda: W.c2(12), "c3_8": lambda: W.c3(8)}[name]()
    h = oracle_fv(case)
    r = _cuda(np.random.default_rng(21).uniform(-1, 1, h.levels[0].n))
    out = []
    for hs, rs in (("0", None), ("0", "0"), (str(1 << 40), None), (None, None)):
        for var, val in (("SSAMG_HOST_SYM", hs), ("SSAMG_ROW_SORT", rs)):
            if val is None:
                monkeypatch.delenv(var, raising=False)
            else:
                monkeypatch.setenv(var, val)
        _, s = gpu_fv(case)
        compare_hierarchy(h, s, len(case.geometry.dims))
        out.append(s.apply_precond(r).cpu())
    assert all(torch.equal(out[0], o) for o in out[1:])


def test_update_after_assembly_uses_the_new_values():
    """After ssamg_update_coeffs on an assembled problem, the assembly's
    direction-metric partials and collapse sums no longer describe the
    coefficients: the new setup forms them from the coefficients and matches
    the oracle on the updated operator (part 0's stencil doubled, which keeps
    it symmetric and diagonally dominant)."""
    _print_case("update after assembly")
    case = W.c3(8)
    g = case.geometry
    _, s = gpu_fv(case)
    new0 = s.copy_stencil(0, 0) * 2.0
    s.update_coeffs(0, new0)
    s.setup()
    A, _ = assemble.assemble_fv(g, case.stencil, case.kappa, case.aniso)
    A = A.tocoo()
    n0 = int(np.prod(g.dims[0]))
    inside = (A.row < n0) & (A.col < n0)
    data = np.where(inside, 2.0 * A.data, A.data)
    A2 = type(A)((data, (A.row, A.col)), shape=A.shape).tocsr()
    pat = [W.stencil_offsets(case.stencil, g.ndim)] * g.nparts
    h = O.setup(A2, g.dims, g.face_kinds(), pat, g.ndim, omega=case.omega, max_levels=64, min_coarse_size=0,
                relax=case.relax, coarse="sweep", skip=False, pb="one", hybrid_level=0, coarse_op="galerkin")
    compare_hierarchy(h, s, g.nparts)


@pytest.mark.parametrize("row_sort", [None, "0"])
def test_repeated_device_setups_are_identical(monkeypatch, row_sort):
    """The device coupling product keeps two count buffers at zero between
    calls (each call leaves them so; they are cleared only when allocated):
    three setups of one solver, every level on the device, give the same
    couplings on every level and the same solve bit for bit, with rows
    ranked in LDS or from memory."""
    _print_case(f"repeated device setups row_sort={row_sort}")
    monkeypatch.setenv("SSAMG_HOST_SYM", "0")
    if row_sort is None:
        monkeypatch.delenv("SSAMG_ROW_SORT", raising=False)
    else:
        monkeypatch.setenv("SSAMG_ROW_SORT", row_sort)
    case = W.c3(8)
    _, s = gpu_fv(case)
    b = _cuda(case.b)
    ref_c = [s.copy_coupling(l) for l in range(s.nlevels)]
    ref_x, st, _ = s.solve(b)
    assert st == 0
    for _ in range(2):
        s.setup()
        for l in range(s.nlevels):
            got = s.copy_coupling(l)
            for a, e in zip(got, ref_c[l]):
                assert np.array_equal(a, e), l
        x, st, _ = s.solve(b)
        assert st == 0 and torch.equal(x, ref_x)


@pytest.mark.parametrize("precision", [0, 1])
def test_split_down_sweep_matches_fused(monkeypatch, precision):
    """On large 27-point levels the first sweep and the residual run as two
    kernels; forced on every level here (SSAMG_SPLIT_CELLS=0) it must give the
    fused kernel's cycle, and both the oracle's."""
    _print_case(f"split precision={precision}")
    case = W.c3(9)
    h = oracle_fv(case)
    r = np.random.default_rng(10).uniform(-1, 1, h.levels[0].n)
    monkeypatch.setenv("SSAMG_SPLIT_CELLS", "0")
    _, s0 = gpu_fv(case, cycle_precision=precision)
    monkeypatch.setenv("SSAMG_SPLIT_CELLS", str(1 << 40))
    _, s1 = gpu_fv(case, cycle_precision=precision)
    z0 = s0.apply_precond(_cuda(r)).cpu().numpy()
    z1 = s1.apply_precond(_cuda(r)).cpu().numpy()
    want = O.vcycle(h, r)
    scale = vcycle_scale(h, r)
    assert_cycle_close(z0, want, scale, CYCLE_RTOL[precision], "split vs oracle")
    assert_cycle_close(z1, want, scale, CYCLE_RTOL[precision], "fused vs oracle")
    assert_cycle_close(z0, z1, scale, CYCLE_RTOL[precision], "split vs fused")


@pytest.mark.parametrize("name,precision", [("c1_16", 0), ("c2_13", 1), ("c3_9", 0), ("c5_11", 1)])
def test_direct_coarsest_solve(name, precision):
    """SSAMG_COARSE_DIRECT: the coarsest level is solved exactly; the cycle and
    the solve match the oracle's cycle with a dense solve there."""
    _print_case(f"direct {name} precision={precision}")
    case = CASES[name]()
    h = oracle_fv(case, coarse="direct")
    pr, s = gpu_fv(case, coarse=1, cycle_precision=precision)
    r = np.random.default_rng(15).uniform(-1, 1, h.levels[0].n)
    z = s.apply_precond(_cuda(r)).cpu().numpy()
    want = O.vcycle(h, r)
    assert_cycle_close(z, want, vcycle_scale(h, r), CYCLE_RTOL[precision], name)
    b = case.b if case.b.ndim == 1 else case.b[0]
    ref = O.solve(h, b, tol=1e-8, flexible=(precision == 1))
    x, st, info = s.solve(_cuda(b))
    assert st == 0 and abs(info.iters[0] - ref.iters) <= 1
    assert info.true_relres[0] < 1e-8


def test_direct_single_level_is_exact():
    """One level (max_levels = 1) with the direct option: the preconditioner is
    A^{-1}, so PCG converges in one iteration."""
    case = W.c1(4)
    pr, s = gpu_fv(case, coarse=1, max_levels=1, tol=1e-10)
    x, st, info = s.solve(_cuda(case.b))
    assert st == 0 and info.iters[0] == 1 and info.true_relres[0] < 1e-12


def test_direct_too_large_is_unsupported():
    from paper_2205_14273_amd.ssamg import SSAMGError
    case = W.c2(13)
    with pytest.raises(SSAMGError) as e:
        gpu_fv(case, coarse=1, max_levels=3)
    assert e.value.status == -3


@pytest.mark.parametrize("name,precision", [("c1_16", 0), ("c2_20", 1), ("c3_9", 0), ("c5_11", 1)])
def test_skip_option_parity(name, precision):
    """The skip option of Section 3.4: the same parts skip relaxation on the
    same levels as in the oracle, and the cycle and solve match it."""
    _print_case(f"skip {name} precision={precision}")
    case = CASES[name]()
    h = oracle_fv(case, skip=True)
    pr, s = gpu_fv(case, skip=1, cycle_precision=precision)
    assert s.nlevels == h.nlevels
    nskip = 0
    for l, lev in enumerate(h.levels):
        for p in range(case.geometry.nparts):
            assert s.level_info(l, p)["skip"] == int(lev._cache["skip"][p]), (l, p)
            nskip += int(lev._cache["skip"][p])
    assert nskip > 0
    r = np.random.default_rng(16).uniform(-1, 1, h.levels[0].n)
    z = s.apply_precond(_cuda(r)).cpu().numpy()
    want = O.vcycle(h, r)
    assert_cycle_close(z, want, vcycle_scale(h, r), CYCLE_RTOL[precision], name)
    b = case.b if case.b.ndim == 1 else case.b[0]
    ref = O.solve(h, b, tol=1e-8, flexible=(precision == 1))
    x, st, info = s.solve(_cuda(b))
    assert st == 0 and abs(info.iters[0] - ref.iters) <= 1
    assert info.true_relres[0] < 1e-8


def test_update_coeffs_rebuilds_the_hierarchy():
    """ssamg_update_coeffs: new values of one part (same pattern); the solver
    refuses to solve until set up again, and then equals a solver built on the
    updated problem from scratch (and the oracle on it)."""
    from paper_2205_14273_amd.ssamg import SSAMGError
    g = W.Geometry(3, [(9, 7, 5), (6, 7, 5)], [(0, 0, 0), (9, 0, 0)])
    case = W.random_link_case(4, g, 7)
    pr, s = gpu_raw(case)
    new1 = np.asarray(case.coeffs[1]) * 3.0
    s.update_coeffs(1, new1)
    with pytest.raises(SSAMGError) as e:
        s.solve(_cuda(case.b))
    assert e.value.status == -2
    s.setup()
    case2 = W.random_link_case(4, g, 7)
    case2.coeffs[1] = new1
    h = oracle_raw(case2)
    compare_hierarchy(h, s, g.nparts)
    pr2, s2 = gpu_raw(case2)
    x, st, info = s.solve(_cuda(case.b))
    x2, st2, info2 = s2.solve(_cuda(case.b))
    assert st == st2 == 0 and torch.equal(x, x2)
