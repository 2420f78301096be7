"""Parity on the paths that full-size runs take, and on the boundary's options.

* the one-thread-per-coarse-cell Galerkin kernel (forced on every level with
  SSAMG_RAP_CELL_MIN=0) against the oracle and, bit for bit, against the
  per-(cell, entry) kernel;
* the 27-point heterogeneous workload at 8 x 64^3 (2.1M cells, the largest the
  oracle sets up in well under a minute): every level element by element, the
  rows where the collapse denominator is not positive, the V-cycle entry by
  entry, iterations and the FP32 cycle's distance to the oracle's solution;
* the four-part anisotropic workload at its full size (4 x 64^3);
* the lumped part-boundary reading, right-hand-side-major vectors, couplings
  given in device memory, the symmetry test of given coefficients, the
  multi-column adjoint gradient and the binding's argument checks.
"""
import numpy as np
import pytest

import workloads as W
from oracle import assemble, ssamg as O
from tests.parity_util import (CYCLE_RTOL, assert_cycle_close, compare_hierarchy, gpu_fv, gpu_raw,
                               oracle_fv, oracle_raw, vcycle_scale)

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _cuda(a):
    return torch.as_tensor(np.ascontiguousarray(a), device="cuda", dtype=torch.float64)


def _print_case(name):
    print(f"[gpu parity full] case {name}", flush=True)


SMALL = {"c2_20": lambda: W.c2(20), "c3_9": lambda: W.c3(9), "c5_11": lambda: W.c5(11)}


@pytest.mark.parametrize("name", list(SMALL))
def test_rap_per_cell_kernel_parity(monkeypatch, name):
    """Levels of at least SSAMG_RAP_CELL_MIN coarse cells take the per-cell
    Galerkin kernel (the one that forms every large coarse operator at full
    size, and the interpolation weights of the levels it forms); forced on
    every level it matches the oracle and gives the per-entry kernel's
    operators and the separate weight kernel's weights bit for bit."""
    _print_case(f"rap per cell {name}")
    case = SMALL[name]()
    h = oracle_fv(case)
    monkeypatch.setenv("SSAMG_RAP_CELL_MIN", "0")
    _, s_cell = gpu_fv(case)
    compare_hierarchy(h, s_cell, case.geometry.nparts)
    monkeypatch.setenv("SSAMG_RAP_CELL_MIN", str(1 << 40))
    _, s_ent = gpu_fv(case)
    for l in range(1, h.nlevels):
        for p in range(case.geometry.nparts):
            assert np.array_equal(s_cell.copy_stencil(l, p), s_ent.copy_stencil(l, p)), (l, p)
            if l < h.nlevels - 1:
                for wc, we in zip(s_cell.copy_interp(l, p), s_ent.copy_interp(l, p)):
                    assert np.array_equal(wc, we), ("weights", l, p)
    r = np.random.default_rng(5).uniform(-1, 1, h.levels[0].n)
    z = s_cell.apply_precond(_cuda(r)).cpu().numpy()
    assert_cycle_close(z, O.vcycle(h, r), vcycle_scale(h, r), CYCLE_RTOL[0], name)


def _rden_rows(h):
    """Rows of the oracle hierarchy where the collapse denominator (sum of the
    row's same-part coefficients with zero d* component, F cells only) is not
    positive."""
    total = 0
    for lev in h.levels[:-1]:
        for p in range(len(lev.dims)):
            ds = lev.dstar[p]
            if ds < 0:
                continue
            vals = O.stencil_values_fast(lev, p)
            pat = np.asarray(lev.pattern[p])
            den = vals[pat[:, ds] == 0].sum(axis=0)
            nx, ny, nz = lev.dims[p]
            idx = np.arange(nx * ny * nz)
            coord = [idx % nx, (idx // nx) % ny, idx // (nx * ny)]
            total += int(np.sum((den <= 0) & (coord[ds] % 2 == 1)))
    return total


def test_c3_64_hierarchy_cycle_and_solve():
    """8 x 64^3, 27-point, log-normal kappa with 1e4 jumps: hierarchy, cycle and
    solves against the oracle at a size where the large-level kernels run."""
    _print_case("c3_64")
    case = W.c3(64)
    h = oracle_fv(case)
    assert _rden_rows(h) > 0      # the collapse fallback is exercised on real operators
    pr, s = gpu_fv(case)
    compare_hierarchy(h, s, case.geometry.nparts)
    r = np.random.default_rng(11).uniform(-1, 1, h.levels[0].n)
    z = s.apply_precond(_cuda(r)).cpu().numpy()
    want = O.vcycle(h, r)
    scale = vcycle_scale(h, r)
    worst = assert_cycle_close(z, want, scale, CYCLE_RTOL[0], "fp64 cycle")
    print(f"[gpu parity full] c3_64 fp64 cycle worst error / scale {worst:.2e}", flush=True)
    ref = O.solve(h, case.b, tol=1e-8)
    x, st, info = s.solve(_cuda(case.b))
    assert st == 0 and abs(info.iters[0] - ref.iters) <= 1, (info.iters[0], ref.iters)
    assert info.true_relres[0] < 1e-8
    xn = x.cpu().numpy()
    assert np.linalg.norm(xn - ref.x) <= 1e-6 * np.linalg.norm(ref.x)
    _, s32 = gpu_fv(case, cycle_precision=1)
    z32 = s32.apply_precond(_cuda(r)).cpu().numpy()
    worst32 = assert_cycle_close(z32, want, scale, CYCLE_RTOL[1], "fp32 cycle")
    x32, st32, info32 = s32.solve(_cuda(case.b))
    assert st32 == 0 and abs(info32.iters[0] - ref.iters) <= 1, (info32.iters[0], ref.iters)
    err32 = float(np.linalg.norm(x32.cpu().numpy() - ref.x) / np.linalg.norm(ref.x))
    print(f"[gpu parity full] c3_64 iters oracle {ref.iters} fp64 {info.iters[0]} fp32 {info32.iters[0]}; "
          f"fp32 cycle worst error / scale {worst32:.2e}; fp32-cycle solution vs oracle {err32:.2e}",
          flush=True)
    assert err32 <= 1e-6


def test_c2_full_size_parity():
    """4 x 64^3 with per-part anisotropy, the workload at its full size."""
    _print_case("c2 full")
    case = W.c2()
    h = oracle_fv(case)
    pr, s = gpu_fv(case)
    compare_hierarchy(h, s, case.geometry.nparts)
    r = np.random.default_rng(13).uniform(-1, 1, h.levels[0].n)
    z = s.apply_precond(_cuda(r)).cpu().numpy()
    assert_cycle_close(z, O.vcycle(h, r), vcycle_scale(h, r), CYCLE_RTOL[0], "c2 full")
    ref = O.solve(h, case.b, tol=1e-8)
    x, st, info = s.solve(_cuda(case.b))
    assert st == 0 and abs(info.iters[0] - ref.iters) <= 1
    assert np.linalg.norm(x.cpu().numpy() - ref.x) <= 1e-6 * np.linalg.norm(ref.x)


@pytest.mark.parametrize("name", list(SMALL))
@pytest.mark.parametrize("precision", [0, 1])
def test_lumped_part_boundary_parity(name, precision):
    """pb_interp = SSAMG_PB_LUMP: weights, operators, cycle and solve as the
    oracle's reading R-pb2."""
    _print_case(f"pb lump {name} precision={precision}")
    case = SMALL[name]()
    h = oracle_fv(case, pb="lump")
    h1 = oracle_fv(case, pb="one")
    _, s = gpu_fv(case, pb_interp=1, cycle_precision=precision)
    compare_hierarchy(h, s, case.geometry.nparts)
    # the two readings differ somewhere on this workload
    assert any(not np.array_equal(a, b) for la, lb in zip(h.levels[:-1], h1.levels[:-1])
               for a, b in zip(la.wm, lb.wm))
    r = np.random.default_rng(17).uniform(-1, 1, h.levels[0].n)
    z = s.apply_precond(_cuda(r)).cpu().numpy()
    assert_cycle_close(z, O.vcycle(h, r), vcycle_scale(h, r), CYCLE_RTOL[precision], name)
    b = case.b if case.b.ndim == 1 else case.b[0]
    ref = O.solve(h, b, tol=1e-8, flexible=(precision == 1))
    x, st, info = s.solve(_cuda(b))
    assert st == 0 and abs(info.iters[0] - ref.iters) <= 1 and info.true_relres[0] < 1e-8


def test_lumped_weight_by_hand_on_device():
    """The hand value of R-pb2 next to a Dirichlet face: 2a/(2a+1) for a = 10."""
    from tests.test_oracle_pins import _pb_case
    case = _pb_case(10.0)
    _, s = gpu_fv(case, pb_interp=1)
    wm, _ = s.copy_interp(0, 0)
    fidx = (3 - 1) // 2 + 2 * (0 + 3 * 1)
    assert wm[fidx] == pytest.approx(20.0 / 21.0, rel=1e-15)
    fidx1 = (3 - 1) // 2 + 2 * (1 + 3 * 1)
    assert wm[fidx1] == pytest.approx(1.0, rel=1e-15)


def test_pb_interp_is_checked():
    from paper_2205_14273_amd.ssamg import SSAMGError
    with pytest.raises(SSAMGError) as e:
        gpu_fv(W.c1(6), pb_interp=2)
    assert e.value.status == -1


def test_rhs_major_layout_matches_cell_major():
    """[nrhs][N] vectors give, column by column, the [N][nrhs] solve bit for bit."""
    from paper_2205_14273_amd import _lib as L
    _print_case("rhs-major layout")
    case = W.c2(12)
    _, s = gpu_fv(case, max_nrhs=4, cycle_precision=1)
    R = np.random.default_rng(19).uniform(-1, 1, (4, case.geometry.n))
    xc, st, ic = s.solve(_cuda(R.T))                                  # [N][4]
    xr, st2, ir = s.solve(_cuda(R), layout=L.LAYOUT_RHS_MAJOR)      # [4][N]
    assert st == st2 == 0
    assert torch.equal(xc.t().contiguous(), xr)
    assert [ic.iters[k] for k in range(4)] == [ir.iters[k] for k in range(4)]
    assert ic.t_setup > 0 and ic.t_solve > 0
    x1, _, i1 = s.solve(_cuda(R[2]), layout=L.LAYOUT_RHS_MAJOR)     # one column: plain vector
    assert st == 0 and i1.iters[0] >= 1


def test_couplings_from_device_memory():
    """set_coupling with device COO arrays builds the same problem as host arrays."""
    from paper_2205_14273_amd import ssamg as B
    _print_case("device couplings")
    g = W.Geometry(3, [(9, 7, 5), (6, 7, 5), (5, 4, 6)], [(0, 0, 0), (9, 0, 0), (9, 7, 0)])
    case = W.random_link_case(2, g, 27)
    pr_h, s_h = gpu_raw(case)
    pr_d = B.Problem(g.ndim, g.dims)
    for p in range(g.nparts):
        for f in range(6):
            B.ssamg_problem_set_face(pr_d.h, p, f, int(case.faces[p][f]))
        B.ssamg_problem_set_stencil(pr_d.h, p, case.stencils[p])
        B.ssamg_problem_set_coeffs(pr_d.h, p, _cuda(np.asarray(case.coeffs[p]).reshape(-1)))
    B.ssamg_problem_set_coupling(pr_d.h, torch.as_tensor(case.urow, device="cuda"),
                                 torch.as_tensor(case.ucol, device="cuda"), _cuda(case.uval))
    s_d = B.Solver(pr_d).setup()
    for l in range(s_h.nlevels):
        a, b = s_h.copy_coupling(l), s_d.copy_coupling(l)
        assert all(np.array_equal(u, v) for u, v in zip(a, b)), l
    xh, _, _ = s_h.solve(_cuda(case.b))
    xd, _, _ = s_d.solve(_cuda(case.b))
    assert torch.equal(xh, xd)


def test_asymmetric_coefficients_read_in_full():
    """Given coefficients that break a_s(c) = a_{-s}(c+s) switch the product's
    mirrored reads off: the level-0 product is still exactly S x + U x of the
    given entries (the mirrored product would use the other half)."""
    _print_case("asymmetric input")
    g = W.Geometry(3, [(9, 7, 5), (6, 7, 5)], [(0, 0, 0), (9, 0, 0)])
    case = W.random_link_case(6, g, 27)
    co = [np.array(c, dtype=np.float64, copy=True) for c in case.coeffs]
    pat = [tuple(int(v) for v in t) for t in case.stencils[0]]
    e = pat.index((1, 0, 0))
    co[0][e].reshape(-1)[3 + 9 * (2 + 7 * 2)] *= 1.5       # one in-box entry of part 0
    case.coeffs = co
    A, _ = assemble.assemble_raw(g.dims, case.stencils, case.coeffs, case.urow, case.ucol, case.uval)
    _, s = gpu_raw(case)
    x = np.random.default_rng(23).standard_normal(g.n)
    y = s.apply_A(0, _cuda(x)).cpu().numpy()
    scale = np.abs(A) @ np.abs(x)
    assert np.max(np.abs(y - A @ x) / scale) <= 1e-13


def test_fv_grad_sums_the_columns():
    """The adjoint gradient of several right-hand sides in one kernel pass is the
    sum of the oracle's per-column gradients."""
    from paper_2205_14273_amd.ssamg import Problem
    _print_case("fv_grad nrhs=4")
    case = W.c5(7)
    g = case.geometry
    rng = np.random.default_rng(29)
    lam = rng.standard_normal((g.n, 4))
    x = rng.standard_normal((g.n, 4))
    want = sum(assemble.fv_gradient(g, case.stencil, case.kappa, case.aniso, lam[:, k], x[:, k])
               for k in range(4))
    pr = Problem.from_fv(g, case.stencil, _cuda(case.kappa), case.aniso)
    got = pr.fv_grad(_cuda(lam), _cuda(x)).cpu().numpy()
    assert np.max(np.abs(got - want)) <= 1e-13 * np.max(np.abs(want)) * 4


def test_binding_rejects_bad_vectors():
    """Wrong dtype, host memory or a wrong length is refused before any kernel
    runs (the C ABI cannot see buffer sizes)."""
    case = W.c1(6)
    _, s = gpu_fv(case)
    n = case.geometry.n
    good = torch.zeros(n, dtype=torch.float64, device="cuda")
    with pytest.raises(TypeError):
        s.solve(torch.zeros(n, dtype=torch.float32, device="cuda"))
    with pytest.raises(TypeError):
        s.solve(torch.zeros(n, dtype=torch.float64))
    with pytest.raises(ValueError):
        s.solve(torch.zeros(n + 1, dtype=torch.float64, device="cuda"))
    with pytest.raises(ValueError):
        s.solve(good, x=torch.zeros(n - 1, dtype=torch.float64, device="cuda"))
    with pytest.raises(ValueError):
        s.apply_A(1, good)
    with pytest.raises(TypeError):
        s.apply_precond(good.float())


def _odd_chunks_case():
    """27-point, two parts of 10 x 10 x 6 (600 cells: three 256-cell chunks, so
    the two-cell kernels' last block holds a chunk the one-cell grid lacks)
    and one of 6 x 10 x 6, heterogeneous kappa and a different anisotropy per
    part (which the cross-part conductances of the 27-point stencil read by
    part index: an odd number of parts and links with dz = +1 once decoded a
    wrong part there)."""
    g = W.Geometry(3, [(10, 10, 6), (10, 10, 6), (6, 10, 6)], [(0, 0, 0), (10, 0, 0), (20, 0, 0)])
    rng = np.random.default_rng(77)
    kappa = np.exp(rng.standard_normal(g.n))
    b = rng.uniform(-1, 1, g.n)
    aniso = np.array([[1.0, 2.0, 3.0], [2.0, 1.0, 1.0], [1.0, 1.0, 4.0]])
    return W.FVCase("odd", g, 27, kappa, aniso, b, relax="l1")


@pytest.mark.parametrize("precision", [0, 1])
@pytest.mark.parametrize("name", ["c3_10", "odd"])
def test_multi_cell_product_and_sweeps(monkeypatch, precision, name):
    """Full 27-point levels with even rows run the PCG product two cells per
    thread and, in the FP64 cycle, the finest residual and post-sweep two cells
    per thread: the cycle matches the oracle entry by entry, the solve reaches
    the tolerance with the oracle's iterations (the true residual is formed by
    the same product), and it equals the one-cell kernels' solve to
    rounding.  The product that takes the row neighbours from the adjacent
    lanes (SSAMG_PRODUCT2=2; the odd case's rows cross wave boundaries, so its
    edge lanes load theirs) gives the same solve bit for bit."""
    _print_case(f"multi-cell kernels {name} precision={precision}")
    case = W.c3(10) if name == "c3_10" else _odd_chunks_case()
    h = oracle_fv(case)
    compare_hierarchy(h, gpu_fv(case)[1], case.geometry.nparts)
    b = case.b
    ref = O.solve(h, b, tol=1e-8, flexible=(precision == 1))
    out = {}
    for v in ("2", "1", "0"):
        monkeypatch.setenv("SSAMG_PRODUCT2", v)
        _, s = gpu_fv(case, cycle_precision=precision)
        r = np.random.default_rng(31).uniform(-1, 1, h.levels[0].n)
        z = s.apply_precond(_cuda(r)).cpu().numpy()
        assert_cycle_close(z, O.vcycle(h, r), vcycle_scale(h, r), CYCLE_RTOL[precision], f"product2={v}")
        x, st, info = s.solve(_cuda(b))
        assert st == 0 and info.true_relres[0] < 1e-8 and abs(info.iters[0] - ref.iters) <= 1
        out[v] = (x.cpu().numpy(), info.iters[0])
    assert out["1"][1] == out["0"][1]
    assert np.linalg.norm(out["1"][0] - out["0"][0]) <= 1e-9 * np.linalg.norm(out["0"][0])
    assert out["2"][1] == out["1"][1] and np.array_equal(out["2"][0], out["1"][0])


@pytest.mark.parametrize("precision", [0, 1])
def test_residual_update_forms_first_sweep(monkeypatch, precision):
    """One-column solves whose down-sweeps are split let PCG's residual update
    form the finest level's first sweep from zero, x = w r, and each
    restriction form the next grid level's, x = w b (SSAMG_FUSE_ZERO, on by
    default): the solve equals the one with the separate sweeps bit for bit,
    and the oracle's iterations.  SSAMG_SPLIT_CELLS=0 splits every level, so
    the small case takes those paths."""
    _print_case(f"fused first sweep precision={precision}")
    case = W.c3(10)
    h = oracle_fv(case)
    ref = O.solve(h, case.b, tol=1e-8, flexible=(precision == 1))
    monkeypatch.setenv("SSAMG_SPLIT_CELLS", "0")
    out = {}
    for v in ("1", "0"):
        monkeypatch.setenv("SSAMG_FUSE_ZERO", v)
        _, s = gpu_fv(case, cycle_precision=precision)
        x, st, info = s.solve(_cuda(case.b))
        assert st == 0 and info.true_relres[0] < 1e-8 and abs(info.iters[0] - ref.iters) <= 1
        out[v] = (x, info.iters[0])
        # a preconditioner application right after a solve starts from zero
        r = _cuda(np.random.default_rng(4).uniform(-1, 1, h.levels[0].n))
        out[v + "z"] = s.apply_precond(r)
    assert out["1"][1] == out["0"][1] and torch.equal(out["1"][0], out["0"][0])
    assert torch.equal(out["1z"], out["0z"])


def test_calls_under_another_stream():
    """A solver orders its work on the stream current at its creation; inputs
    made under another stream (the assembled coefficients, b) are waited for
    and its outputs are ready on the caller's stream: the solve equals the one
    made on a single stream, bit for bit."""
    from paper_2205_14273_amd.ssamg import Problem, Solver
    _print_case("calls under another stream")
    case = W.c2(12)
    _, s0 = gpu_fv(case)
    x0, st0, _ = s0.solve(_cuda(case.b))
    side = torch.cuda.Stream()
    with torch.cuda.stream(side):
        kappa = torch.as_tensor(case.kappa, device="cuda")
        pr = Problem.from_fv(case.geometry, case.stencil, kappa, case.aniso)
    s = Solver(pr)
    with torch.cuda.stream(side):
        s.setup()
        b = torch.as_tensor(case.b, device="cuda")
        x, st, _ = s.solve(b)
        y = x * 1.0
        z = s.apply_precond(b) * 1.0
    torch.cuda.synchronize()
    assert st == st0 == 0
    assert torch.equal(y, x0)
    assert torch.equal(z, s0.apply_precond(_cuda(case.b)))
