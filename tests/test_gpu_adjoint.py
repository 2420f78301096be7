"""Adjoint gradient of L(x(kappa)) = 1/2 ||x - x_t||^2 with x = A(kappa)^{-1} b.

* the library's fv_grad kernels against the oracle's gradient formula on the
  same seeded (lambda, x) - 7- and 27-point, several parts, a different
  anisotropy per part, 2D;
* the autograd function end to end against the oracle (exact sparse solves,
  oracle assembly and gradient) on small problems;
* the adjoint gradient against central finite differences of L on sampled
  cells, at the full 3 x 64^3 size (a property that holds at any size).
"""
import numpy as np
import pytest
import scipy.sparse.linalg as spla

import workloads as W
from oracle import assemble

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _cuda(a):
    return torch.as_tensor(np.ascontiguousarray(a), device="cuda", dtype=torch.float64)


def _print_case(name):
    print(f"[gpu adjoint] case {name}", flush=True)


def _fv_case(name):
    return {
        "c5_7": lambda: W.c5(7),
        "c3_6": lambda: W.c3(6),
        "c2_9": lambda: W.c2(9),
        "2d": _case_2d,
        "odd27": _case_odd27,
    }[name]()


def _case_odd27():
    """27-point, three parts of different sizes along x, a different
    anisotropy per part (cross-part conductances read it by part index)."""
    g = W.geometry_along_x(3, [(5, 4, 3), (5, 4, 3), (3, 4, 3)])
    kappa = np.exp(np.random.default_rng(78).standard_normal(g.n))
    aniso = np.array([[1.0, 2.0, 3.0], [2.0, 1.0, 1.0], [1.0, 1.0, 4.0]])
    return W.FVCase("odd27", g, 27, kappa, aniso, np.zeros(g.n))


def _case_2d():
    g = W.geometry_along_x(2, [(9, 7, 1), (6, 7, 1)])
    kappa = np.exp(np.random.default_rng(77).standard_normal(g.n))
    return W.FVCase("2d", g, 9, kappa, np.array([[1.0, 3.0, 1.0], [2.0, 1.0, 1.0]]),
                    np.zeros(g.n))


@pytest.mark.parametrize("name", ["c5_7", "c3_6", "c2_9", "2d", "odd27"])
def test_fv_grad_kernel_parity(name):
    _print_case(name)
    from paper_2205_14273_amd.ssamg import Problem
    case = _fv_case(name)
    g = case.geometry
    rng = np.random.default_rng(12)
    lam = rng.standard_normal(g.n)
    x = rng.standard_normal(g.n)
    want = assemble.fv_gradient(g, case.stencil, case.kappa, case.aniso, lam, x)
    pr = Problem.from_fv(g, case.stencil, _cuda(case.kappa), case.aniso)
    got = pr.fv_grad(_cuda(lam), _cuda(x)).cpu().numpy()
    scale = np.max(np.abs(want))
    assert np.max(np.abs(got - want)) <= 1e-13 * scale


def _loss_and_grad_oracle(case):
    g = case.geometry
    A, _ = assemble.assemble_fv(g, case.stencil, case.kappa, case.aniso)
    At, _ = assemble.assemble_fv(g, case.stencil, case.extra["kappa_target"], case.aniso)
    xt = spla.spsolve(At.tocsc(), case.b)
    x = spla.spsolve(A.tocsc(), case.b)
    lam = spla.spsolve(A.tocsc(), x - xt)
    grad = assemble.fv_gradient(g, case.stencil, case.kappa, case.aniso, lam, x)
    return xt, x, lam, grad


@pytest.mark.parametrize("m,precision", [(8, 0), (11, 1)])
def test_autograd_matches_oracle(m, precision):
    _print_case(f"c5_{m} precision={precision}")
    from paper_2205_14273_amd.autograd import FVSolver
    case = W.c5(m)
    g = case.geometry
    xt, x_ref, lam_ref, grad_ref = _loss_and_grad_oracle(case)
    fv = FVSolver(g, case.stencil, case.aniso, tol=1e-13, max_iter=200, cycle_precision=precision)
    kappa = _cuda(case.kappa).requires_grad_(True)
    b = _cuda(case.b).requires_grad_(True)
    x = fv.solve(kappa, b)
    loss = 0.5 * torch.sum((x - _cuda(xt)) ** 2)
    loss.backward()
    xs = x.detach().cpu().numpy()
    assert np.linalg.norm(xs - x_ref) <= 1e-10 * np.linalg.norm(x_ref)
    gk = kappa.grad.cpu().numpy()
    assert np.max(np.abs(gk - grad_ref)) <= 1e-9 * np.max(np.abs(grad_ref))
    gb = b.grad.cpu().numpy()
    assert np.linalg.norm(gb - lam_ref) <= 1e-10 * np.linalg.norm(lam_ref)


def test_autograd_reuses_hierarchy_and_rebuilds_on_change():
    _print_case("c5_6 cache")
    from paper_2205_14273_amd.autograd import FVSolver
    case = W.c5(6)
    fv = FVSolver(case.geometry, case.stencil, case.aniso, tol=1e-12)
    kappa = _cuda(case.kappa)
    b = _cuda(case.b)
    x1 = fv.solve(kappa, b)
    k1 = fv._kappa
    x2 = fv.solve(kappa, b)
    assert fv._kappa is k1                                # same kappa: no new setup
    assert torch.equal(x1, x2)
    kappa.mul_(2.0)                                       # in place: must re-assemble
    x3 = fv.solve(kappa, b)
    # A(2 kappa) = 2 A(kappa) for the harmonic-mean rule, so x halves
    assert torch.allclose(x3, 0.5 * x1, rtol=1e-9, atol=0)


def test_adjoint_vs_central_fd_full_c5():
    """Full 3 x 64^3 problem: the autograd gradient at 50 sampled cells against
    central differences of L with h = 1e-6 on kappa_c; every solve to 1e-13."""
    _print_case("c5 full FD")
    from paper_2205_14273_amd.autograd import FVSolver
    case = W.c5()
    g = case.geometry
    fv_t = FVSolver(g, case.stencil, case.aniso, tol=1e-13, max_iter=300)
    b = _cuda(case.b)
    xt = fv_t.solve(_cuda(case.extra["kappa_target"]), b).detach()
    fv = FVSolver(g, case.stencil, case.aniso, tol=1e-13, max_iter=300)
    kappa = _cuda(case.kappa).requires_grad_(True)
    x = fv.solve(kappa, b)
    loss = 0.5 * torch.sum((x - xt) ** 2)
    loss.backward()
    grad = kappa.grad.cpu().numpy()
    h = case.extra["fd_h"]
    gmax = np.max(np.abs(grad))
    base = case.kappa.copy()
    worst = 0.0
    for c in case.extra["sample"]:
        L = []
        for sg in (1.0, -1.0):
            k = base.copy()
            k[c] += sg * h
            with torch.no_grad():
                xk = fv.solve(_cuda(k), b)
                L.append(0.5 * float(torch.sum((xk - xt) ** 2)))
        fd = (L[0] - L[1]) / (2 * h)
        worst = max(worst, abs(fd - grad[c]))
    print(f"[gpu adjoint] max |fd - adjoint| = {worst:.3e}, max |grad| = {gmax:.3e}", flush=True)
    assert worst <= 1e-6 * gmax
