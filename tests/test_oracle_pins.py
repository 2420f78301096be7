"""Pins of the CPU oracle against facts fixed by the paper and by mathematics.

None of these re-types the oracle's formulas: each compares it with a
hand-derived value (tests/golden), a closed form, a dense direct solve, finite
differences, or a structural invariant (the theorem of Section 3.3).
"""
import math

import numpy as np
import pytest
import scipy.linalg as sla

import workloads as W
from oracle import assemble, ssamg
from tests.conftest import _frac


def fv_hierarchy(case, **kw):
    A, off = assemble.assemble_fv(case.geometry, case.stencil, case.kappa, case.aniso)
    faces = case.geometry.face_kinds()
    pat = [W.stencil_offsets(case.stencil, case.geometry.ndim)] * case.geometry.nparts
    h = ssamg.setup(A, case.geometry.dims, faces, pat, case.geometry.ndim,
                    omega=kw.pop("omega", case.omega), **kw)
    return A, h


def seq_of(h, p=0):
    return "".join("xyz"[l.dstar[p]] for l in h.levels if l.dstar[p] >= 0)


# ---------------------------------------------------------------------------
# assembly


def test_fv_c1_is_the_seven_point_laplacian():
    # eq:stencilA with alpha = beta = gamma = 1: diagonal 6, off-diagonals -1
    A, _ = assemble.assemble_fv(W.c1().geometry, 7, np.ones(4096), np.ones((1, 3)))
    assert np.all(A.diagonal() == 6.0)
    off = A.copy()
    off.setdiag(0)
    off.eliminate_zeros()
    assert set(np.unique(off.data)) == {-1.0}
    deg = np.diff(off.indptr)
    # an interior cell has 6 neighbours, a corner 3
    assert deg.max() == 6 and deg.min() == 3


def test_fv_interface_is_harmonic_mean():
    case = W.c2(4)
    A, _ = assemble.assemble_fv(case.geometry, 7, case.kappa, case.aniso)
    # part 0 cell (3,1,2) couples to part 1 cell (0,1,2) with H(100, 1) = 200/101
    i = 3 + 4 * (1 + 4 * 2)
    j = 64 + 0 + 4 * (1 + 4 * 2)
    assert A[i, j] == pytest.approx(-200.0 / 101.0, rel=1e-15)
    assert A[j, i] == A[i, j]


def test_raw_assembly_drops_out_of_box_entries():
    g = W.geometry_along_x(2, [(4, 3, 2), (3, 3, 2)])
    clean = W.random_link_case(7, g, 7)
    junk = W.random_link_case(7, g, 7, junk_outside=True)
    A1, _ = assemble.assemble_raw(g.dims, clean.stencils, clean.coeffs, clean.urow, clean.ucol, clean.uval)
    A2, _ = assemble.assemble_raw(g.dims, junk.stencils, junk.coeffs, junk.urow, junk.ucol, junk.uval)
    assert abs(A1 - A2).max() == 0.0
    assert abs(A1 - A1.T).max() == 0.0
    np.linalg.cholesky(A1.toarray())


# ---------------------------------------------------------------------------
# Section 3.1: W and Algorithm 1


def test_W_closed_forms():
    _, h = fv_hierarchy(W.c1(8))
    assert list(h.W0[0]) == [1.0, 1.0, 1.0]
    _, h = fv_hierarchy(W.c2(8))
    # c_d is proportional to the directional factor: W = sqrt(100 / a_d)
    assert list(h.W0[0]) == [1.0, 10.0, 10.0]
    assert list(h.W0[1]) == [10.0, 1.0, 10.0]
    assert list(h.W0[2]) == [10.0, 10.0, 1.0]


@pytest.mark.parametrize("row", range(7))
def test_algorithm1_sequences(golden, row):
    nx, ny, nz, ax, ay, az, seq, levels = golden("algorithm1_sequences.txt")[row]
    dims = [(int(nx), int(ny), int(nz))]
    a = [float(ax), float(ay), float(az)]
    ndim = 3 if int(nz) > 1 else 2
    cd = np.array([a])
    Wm = ssamg.grid_spacing(cd, ndim)
    all_dims, all_dstar, _ = ssamg.coarsen(Wm, dims, ndim)
    got = "".join("xyz"[d[0]] for d in all_dstar if d[0] >= 0)
    assert got == seq
    assert len(all_dims) == int(levels)
    assert all_dims[-1] == [(1, 1, 1)]


def test_algorithm1_from_assembled_operator(golden):
    # the same sequences come out when W is computed from the assembled matrix
    _, h = fv_hierarchy(W.c1())
    assert seq_of(h) == "xyz" * 4 and h.nlevels == 13
    case = W.c2(64)
    case.geometry = W.Geometry(3, [(64, 64, 64)], [(0, 0, 0)])
    case.kappa = np.ones(64 ** 3)
    for aniso, seq in [((100, 1, 1), "xxxxyzxyzxyzyzyzyz")]:
        case.aniso = np.array([aniso], dtype=float)
        _, h = fv_hierarchy(case)
        assert seq_of(h) == seq


def test_coarsest_size_is_number_of_parts():
    # SSAMG-base: the coarsest grid size equals the number of parts (Section 4)
    for case in (W.c2(8), W.c3(4), W.c5(4)):
        _, h = fv_hierarchy(case)
        assert h.levels[-1].n == case.geometry.nparts
        assert all(d == (1, 1, 1) for d in h.levels[-1].dims)


def test_coarse_extent_is_ceil_half():
    _, h = fv_hierarchy(W.c1(13))
    assert h.levels[1].dims[0] == (7, 13, 13)
    assert h.levels[2].dims[0] == (7, 7, 13)


# ---------------------------------------------------------------------------
# Section 3.4: relaxation weights


@pytest.mark.parametrize("row", range(3))
def test_omega_values(golden, row):
    r = golden("omega_values.txt")[row]
    a = [float(v) for v in r[:3]]
    want = [_frac(v) for v in r[3:]]
    Wm = ssamg.grid_spacing(np.array([a]), 3)
    _, _, om = ssamg.coarsen(Wm, [(64, 64, 64)], 3)
    got = [float(o[0]) for o in om[:4]]
    tol = 1e-15 if "/" in r[3] else 5e-5
    assert got == pytest.approx(want, abs=tol)


def test_omega_paper_2d_like_example():
    # Section 3.4: nearly decoupled in k, isotropic in i and j -> omega = 4/5
    Wp = np.array([1.0, 1.0, 1e6])
    assert ssamg.relax_weight(Wp, 0, 3) == pytest.approx(0.8, abs=1e-11)


# ---------------------------------------------------------------------------
# Section 3.2: interpolation


@pytest.mark.parametrize("row", range(8))
def test_interp_weights_c1(golden, row):
    i, j, k, wm, wp = golden("interp_weights.txt")[row]
    A, h = fv_hierarchy(W.c1())
    lev = h.levels[0]
    assert lev.dstar[0] == 0
    fi = (int(i) - 1) // 2
    lin = fi + 8 * (int(j) + 16 * int(k))
    assert lev.wm[0][lin] == pytest.approx(_frac(wm), abs=1e-15)
    assert lev.wp[0][lin] == pytest.approx(_frac(wp), abs=1e-15)


def test_interp_paper_worked_mapping():
    # Section 3.2 example: semicoarsening in i; fine (3,3) takes coarse (1,3) and
    # (2,3); fine (2,3) maps with weight 1 to coarse (1,3).
    g = W.Geometry(2, [(8, 6, 1)], [(0, 0, 0)])
    case = W.FVCase("t", g, 9, np.ones(g.n), np.array([[1.0, 0.5, 1.0]]), np.ones(g.n))
    A, h = fv_hierarchy(case)
    lev = h.levels[0]
    assert lev.dstar[0] == 0
    P = lev.P.tocsr()
    cx = h.levels[1].dims[0][0]
    f33 = 3 + 8 * 3
    cols = sorted(P.indices[P.indptr[f33]:P.indptr[f33 + 1]])
    assert cols == [1 + cx * 3, 2 + cx * 3]
    f23 = 2 + 8 * 3
    assert list(P.indices[P.indptr[f23]:P.indptr[f23 + 1]]) == [1 + cx * 3]
    assert P.data[P.indptr[f23]] == 1.0
    # nine-point collapse: P_W = (A_SW + A_W + A_NW) / -(A_S + A_C + A_N)
    row = A.getrow(f33).toarray().ravel()
    west = row[2 + 8 * 2] + row[2 + 8 * 3] + row[2 + 8 * 4]
    mid = row[3 + 8 * 2] + row[3 + 8 * 3] + row[3 + 8 * 4]
    Pw = P[f33, 1 + cx * 3]
    assert Pw == pytest.approx(-west / mid, rel=1e-14)
    assert Pw > 0


def test_interp_reproduces_constants_on_zero_row_sum_rows():
    case = W.c5(8)
    A, h = fv_hierarchy(case)
    for lev in h.levels[:-1]:
        # P is collapsed from the structured part S alone (Section 3.2), so the
        # rows whose S-row sums to zero (no Dirichlet face, no coupling in U)
        # interpolate constants exactly
        part, i, j, k = assemble.cell_coords(lev.dims, lev.offsets)
        Ac = lev.A.tocoo()
        same = part[Ac.row] == part[Ac.col]
        s_rowsum = np.bincount(Ac.row[same], weights=Ac.data[same], minlength=lev.n)
        p1 = lev.P @ np.ones(lev.P.shape[1])
        interior = np.abs(s_rowsum) < 1e-9 * np.abs(lev.A.diagonal())
        if lev is h.levels[0]:
            assert interior.sum() > 0
        assert np.allclose(p1[interior], 1.0, atol=1e-12)


def test_part_boundary_rule_gives_weight_one():
    # Section 3.2: a weight crossing a part face is zero and the opposite one is 1
    case = W.c2(8)
    A, h = fv_hierarchy(case)
    lev = h.levels[0]
    p = 0                                # +x face is a part face, d* = x
    assert lev.dstar[p] == 0
    wm = lev.wm[p].reshape(8, 8, 4)      # F-box (z, y, x): odd x = 1,3,5,7
    wp = lev.wp[p].reshape(8, 8, 4)
    assert np.all(wm[:, :, 3] == 1.0) and np.all(wp[:, :, 3] == 0.0)
    # part 3: -x face is a part face, +x face physical (even extent: F cell 7 has
    # an in-box -x neighbour and no +x neighbour -> plain collapse there)
    assert lev.dstar[3] == 0
    wm3 = lev.wm[3].reshape(8, 8, 4)
    assert np.all(wm3[:, :, 3] < 1.0) and np.all(lev.wp[3].reshape(8, 8, 4)[:, :, 3] == 0.0)


# ---------------------------------------------------------------------------
# Section 3.3: Galerkin coarse operator


def test_galerkin_closed_form_interior(golden):
    _, h = fv_hierarchy(W.c1())
    lev1 = h.levels[1]
    vals = ssamg.stencil_values(lev1, 0)
    pat = [tuple(int(v) for v in t) for t in lev1.pattern[0]]
    assert len(pat) == 15
    cx, cy, cz = lev1.dims[0]
    # an interior coarse cell: fine rows 2I-1..2I+1 far from every face
    I, J, K = 3, 7, 7
    cell = I + cx * (J + cy * K)
    want = {(int(a), int(b), int(c)): _frac(v) for a, b, c, v in golden("rap_closed_form.txt")}
    got = {pat[e]: vals[e, cell] for e in range(len(pat))}
    assert set(got) == set(want)
    for key in want:
        assert got[key] == pytest.approx(want[key], abs=1e-14)


def test_galerkin_1d_textbook():
    # P^T [-1 2 -1] P = [-1/2 1 -1/2] in the interior (two-point interpolation 1/2)
    g = W.Geometry(2, [(33, 1, 1)], [(0, 0, 0)])
    case = W.FVCase("t", g, 5, np.ones(g.n), np.array([[1.0, 1.0, 1.0]]), np.ones(g.n))
    A, off = assemble.assemble_fv(g, 5, case.kappa, case.aniso)
    A = A.tolil()
    for i in range(33):        # remove the y-ghost contribution: pure 1D operator
        A[i, i] = 2.0
    A = A.tocsr()
    h = ssamg.setup(A, g.dims, g.face_kinds(), [W.stencil_offsets(5, 2)], 2)
    A1 = h.levels[1].A.toarray()
    assert A1[8, 7] == pytest.approx(-0.5) and A1[8, 8] == pytest.approx(1.0)
    assert A1[8, 9] == pytest.approx(-0.5)


def test_stencil_growth_bound():
    # Section 3.3: a 7-point fine stencil grows to at most 27 points, 5 -> 9 in 2D
    _, h = fv_hierarchy(W.c3(4))
    for lev in h.levels:
        for p in range(len(lev.dims)):
            assert len(lev.pattern[p]) <= 27
    _, h = fv_hierarchy(W.c2(8))
    assert max(len(l.pattern[0]) for l in h.levels) == 27
    g = W.Geometry(2, [(16, 16, 1)], [(0, 0, 0)])
    case = W.FVCase("t", g, 5, np.ones(g.n), np.ones((1, 3)), np.ones(g.n))
    _, h = fv_hierarchy(case)
    assert max(len(l.pattern[0]) for l in h.levels) == 9


@pytest.mark.parametrize("mk", [lambda: W.c2(6), lambda: W.c3(5), lambda: W.c5(5)])
def test_coarse_operators_spd_and_theorem(mk):
    case = mk()
    A, h = fv_hierarchy(case)
    for l, lev in enumerate(h.levels):
        Ad = lev.A.toarray()
        assert np.max(np.abs(Ad - Ad.T)) <= 1e-13 * np.max(np.abs(Ad))
        np.linalg.cholesky(Ad)
        # numeric entries lie in the symbolic pattern (raises otherwise)
        for p in range(len(lev.dims)):
            ssamg.stencil_values_fast(lev, p)
        # theorem of Section 3.3: U couples only points on part faces and never
        # two points of one part
        part, i, j, k = assemble.cell_coords(lev.dims, lev.offsets)
        U = lev.ustruct.tocoo()
        assert np.all(part[U.row] != part[U.col])
        dims = np.asarray(lev.dims)[part[U.row]]
        on_face = np.zeros(U.nnz, dtype=bool)
        faces = case.geometry.face_kinds()[part[U.row]]
        for ax, c in enumerate((i, j, k)):
            cr = c[U.row]
            on_face |= (cr == 0) & (faces[:, 2 * ax] == 1)
            on_face |= (cr == dims[:, ax] - 1) & (faces[:, 2 * ax + 1] == 1)
        assert on_face.all()
        # every cross-part entry of the full product is on the symbolic structure
        Af = lev.A.tocoo()
        cross = part[Af.row] != part[Af.col]
        st = lev.ustruct.tocsr()
        assert np.all(np.asarray(st[Af.row[cross], Af.col[cross]]).ravel() == 1.0)


# ---------------------------------------------------------------------------
# Section 3.4 / Section 4: V-cycle and PCG


@pytest.mark.parametrize("mk", [lambda: W.c1(6), lambda: W.c2(5), lambda: W.c3(4)])
def test_vcycle_is_spd(mk):
    case = mk()
    A, h = fv_hierarchy(case)
    n = A.shape[0]
    B = np.column_stack([ssamg.vcycle(h, e) for e in np.eye(n)])
    assert np.max(np.abs(B - B.T)) <= 1e-12 * np.max(np.abs(B))
    assert np.linalg.eigvalsh(0.5 * (B + B.T)).min() > 0


def test_vcycle_contracts():
    # a multigrid cycle: the error propagator I - BA has spectral radius well
    # below 1 (a sign or transfer mistake pushes it to >= 1)
    for case in (W.c1(8), W.c2(6), W.c3(4)):
        A, h = fv_hierarchy(case)
        n = A.shape[0]
        B = np.column_stack([ssamg.vcycle(h, e) for e in np.eye(n)])
        rho = max(abs(np.linalg.eigvals(np.eye(n) - B @ A.toarray())))
        assert rho < 0.7


@pytest.mark.parametrize("mk", [lambda: W.c1(8), lambda: W.c2(6), lambda: W.c3(4), lambda: W.c5(6)])
def test_pcg_matches_dense_solve(mk):
    case = mk()
    A, h = fv_hierarchy(case)
    b = case.b if case.b.ndim == 1 else case.b[0]
    x_direct = sla.solve(A.toarray(), b, assume_a="pos")
    res = ssamg.solve(h, b, tol=1e-10)
    assert res.converged and res.true_relres < 1e-10
    err = np.linalg.norm(res.x - x_direct) / np.linalg.norm(x_direct)
    assert err < 1e-8
    flex = ssamg.solve(h, b, tol=1e-10, flexible=True)
    assert abs(flex.iters - res.iters) <= 1


def test_pcg_zero_rhs():
    _, h = fv_hierarchy(W.c1(4))
    res = ssamg.solve(h, np.zeros(64))
    assert res.iters == 0 and np.all(res.x == 0)


def test_direct_coarse_option_also_spd():
    case = W.c2(5)
    A, h = fv_hierarchy(case, coarse="direct")
    res = ssamg.solve(h, case.b, tol=1e-10)
    assert res.converged


def test_raw_case_hierarchy():
    g = W.geometry_along_x(3, [(5, 4, 3), (4, 4, 3), (3, 5, 2)])
    g.origins = [(0, 0, 0), (5, 0, 0), (9, 0, 0)]
    case = W.random_link_case(3, g, 27, junk_outside=True)
    A, off = assemble.assemble_raw(g.dims, case.stencils, case.coeffs, case.urow, case.ucol, case.uval)
    h = ssamg.setup(A, g.dims, case.faces, case.stencils, 3,
                    ustruct0=assemble.u_structure(case.urow, case.ucol, A.shape[0]))
    x_direct = np.linalg.solve(A.toarray(), case.b)
    res = ssamg.solve(h, case.b, tol=1e-11)
    assert np.linalg.norm(res.x - x_direct) <= 1e-9 * np.linalg.norm(x_direct)


# ---------------------------------------------------------------------------
# adjoint gradient of the FV workload


def test_fv_gradient_matches_finite_differences():
    case = W.c5(3)
    g = case.geometry
    kt = case.extra["kappa_target"]
    At, _ = assemble.assemble_fv(g, 7, kt, case.aniso)
    xt = np.linalg.solve(At.toarray(), case.b)

    def loss(kap):
        A, _ = assemble.assemble_fv(g, 7, kap, case.aniso)
        x = np.linalg.solve(A.toarray(), case.b)
        return 0.5 * np.sum((x - xt) ** 2), x, A

    L0, x, A = loss(case.kappa)
    lam = np.linalg.solve(A.toarray(), x - xt)
    grad = assemble.fv_gradient(g, 7, case.kappa, case.aniso, lam, x)
    h = 1e-6
    for c in range(0, g.n, 7):
        kp = case.kappa.copy()
        km = case.kappa.copy()
        kp[c] += h
        km[c] -= h
        fd = (loss(kp)[0] - loss(km)[0]) / (2 * h)
        assert grad[c] == pytest.approx(fd, rel=1e-5, abs=1e-12)


def test_fv_gradient_27_point_and_anisotropic():
    case = W.c3(2)
    g = case.geometry
    aniso = np.random.default_rng(0).uniform(0.5, 2.0, (8, 3))
    kap = np.random.default_rng(1).uniform(0.5, 2.0, g.n)
    b = np.random.default_rng(2).uniform(-1, 1, g.n)

    def xsol(k):
        A, _ = assemble.assemble_fv(g, 27, k, aniso)
        return np.linalg.solve(A.toarray(), b), A

    x, A = xsol(kap)
    w = np.random.default_rng(3).standard_normal(g.n)     # L = w . x
    lam = np.linalg.solve(A.toarray(), w)
    grad = assemble.fv_gradient(g, 27, kap, aniso, lam, x)
    h = 1e-6
    for c in range(0, g.n, 5):
        kp = kap.copy()
        km = kap.copy()
        kp[c] += h
        km[c] -= h
        fd = (w @ xsol(kp)[0] - w @ xsol(km)[0]) / (2 * h)
        assert grad[c] == pytest.approx(fd, rel=1e-5, abs=1e-10)


# ---------------------------------------------------------------------------
# reading R-den: collapse with a non-positive denominator


def den_fallback_case():
    """3 x 5 cells, 5-point, strong y links so d* = y; the F cell (1,1) has
    diagonal 1 and x links -0.6, -0.6 (collapse denominator 1 - 1.2 < 0) and y
    links -0.3 (to y=0) and -0.1 (to y=2).  Other rows are strictly dominant."""
    nx, ny = 3, 5
    offs = W.stencil_offsets(5, 2)           # center, (0,-1), (-1,0), (1,0), (0,1)
    key = {tuple(int(v) for v in o): e for e, o in enumerate(offs)}
    coef = np.zeros((5, 1, ny, nx))

    def link(i0, j0, i1, j1, t):
        coef[key[(i1 - i0, j1 - j0, 0)], 0, j0, i0] = -t
        coef[key[(i0 - i1, j0 - j1, 0)], 0, j1, i1] = -t

    for j in range(ny):
        for i in range(nx):
            if i + 1 < nx:
                special = j == 1 and i in (0, 1)
                link(i, j, i + 1, j, 0.6 if special else 0.1)
            if j + 1 < ny:
                t = 4.0
                if i == 1 and j == 0:
                    t = 0.3
                if i == 1 and j == 1:
                    t = 0.1
                link(i, j, i, j + 1, t)
    for j in range(ny):
        for i in range(nx):
            coef[0, 0, j, i] = 20.0
    coef[0, 0, 1, 1] = 1.0
    g = W.Geometry(2, [(nx, ny, 1)], [(0, 0, 0)])
    b = np.random.default_rng(11).uniform(-1, 1, nx * ny)
    return W.RawCase("den", g, np.zeros((1, 6), dtype=np.int32), [offs], [coef],
                     np.zeros(0, np.int64), np.zeros(0, np.int64), np.zeros(0), b)


def test_collapse_fallback_weights():
    case = den_fallback_case()
    g = case.geometry
    A, _ = assemble.assemble_raw(g.dims, case.stencils, case.coeffs, case.urow, case.ucol, case.uval)
    Ad = A.toarray()
    np.linalg.cholesky(Ad)                    # the operator is SPD
    f = 1 + 3 * 1
    den = Ad[f, f] + Ad[f, f - 1] + Ad[f, f + 1]
    assert den < 0
    h = ssamg.setup(A, g.dims, case.faces, case.stencils, 2)
    lev = h.levels[0]
    assert lev.dstar[0] == 1
    # F-box (3 x 2): cell (1,1) -> F (1,0); weights -0.3/-0.4 and -0.1/-0.4
    assert lev.wm[0][1] == pytest.approx(0.75, abs=1e-15)
    assert lev.wp[0][1] == pytest.approx(0.25, abs=1e-15)
    # other F cells keep the plain collapse (positive denominator)
    assert lev.wm[0][0] == pytest.approx(-Ad[0 + 3, 0] / (Ad[3, 3] + Ad[3, 4]), rel=1e-14)
    res = ssamg.solve(h, case.b, tol=1e-12)
    assert np.linalg.norm(res.x - np.linalg.solve(Ad, case.b)) < 1e-10 * np.linalg.norm(res.x)


# ---------------------------------------------------------------------------
# Section 3.4: weighted L1-Jacobi


@pytest.mark.parametrize("mk", [lambda: W.c3(4), lambda: W.c2(5), lambda: W.c5(5)])
def test_l1_diagonal_dominates_A(mk):
    # M_ii = sum_j |a_ij| makes M - A weakly diagonally dominant, hence
    # lambda(M^{-1} A) lies in (0, 1] on every level (the convergence property
    # the paper cites for SPD A)
    case = mk()
    A, _ = assemble.assemble_fv(case.geometry, case.stencil, case.kappa, case.aniso)
    g = case.geometry
    h = ssamg.setup(A, g.dims, g.face_kinds(), [W.stencil_offsets(case.stencil)] * g.nparts, 3,
                    relax="l1")
    for lev in h.levels:
        w = ssamg._cell_weights(lev)            # 1.5 / M_ii
        m = 1.5 / w
        Ad = lev.A.toarray()
        lam = np.linalg.eigvals(Ad / m[:, None]).real
        assert lam.max() <= 1.0 + 1e-12 and lam.min() > 0
        # M_ii is the full row (stencil and couplings) in absolute value
        assert np.allclose(m, np.abs(Ad).sum(axis=1), rtol=1e-14)


def test_l1_vcycle_spd_and_pcg():
    case = W.c3(4)
    A, _ = assemble.assemble_fv(case.geometry, 27, case.kappa, case.aniso)
    g = case.geometry
    h = ssamg.setup(A, g.dims, g.face_kinds(), [W.stencil_offsets(27)] * 8, 3, relax="l1")
    n = A.shape[0]
    B = np.column_stack([ssamg.vcycle(h, e) for e in np.eye(n)])
    assert np.max(np.abs(B - B.T)) <= 1e-12 * np.max(np.abs(B))
    assert np.linalg.eigvalsh(0.5 * (B + B.T)).min() > 0
    res = ssamg.solve(h, case.b, tol=1e-10)
    xd = np.linalg.solve(A.toarray(), case.b)
    assert np.linalg.norm(res.x - xd) <= 1e-8 * np.linalg.norm(xd)


# ---------------------------------------------------------------------------
# Section 3.4: the "skip" option


def _skip_levels(h, p=0):
    return {l for l, lev in enumerate(h.levels) if lev._cache["skip"][p]}


def test_skip_levels_from_hand_sequences():
    """Relaxation is off at level l when d*_l = d*_{l-3} (3D).  Worked by hand
    on the Algorithm 1 sequences of tests/golden: the isotropic 16^3 box,
    x y z repeating over 12 coarsening levels, skips levels 3..11; the
    (100,1,1) 64^3 box, xxxx yz xyz xyz yzyzyz, skips 3, 6, 7, 8, 9, 10, 11;
    the coarsest level never skips."""
    _, h = fv_hierarchy(W.c1(16), skip=True)
    assert _skip_levels(h) == set(range(3, 12))
    assert seq_of(h) == "xyzxyzxyzxyz"
    case = W.c2(64)
    case.geometry.dims = case.geometry.dims[:1]
    case.geometry.origins = case.geometry.origins[:1]
    case.aniso = case.aniso[:1]
    case.kappa = case.kappa[:64 ** 3]
    _, h = fv_hierarchy(case, skip=True)
    assert seq_of(h) == "xxxxyzxyzxyzyzyzyz"
    assert _skip_levels(h) == {3, 6, 7, 8, 9, 10, 11}
    _, h0 = fv_hierarchy(W.c1(16))
    assert _skip_levels(h0) == set()


def test_skip_zeroes_exactly_the_skipped_parts():
    _, h = fv_hierarchy(W.c2(8), skip=True, relax="l1")
    for l, lev in enumerate(h.levels):
        wd = ssamg._cell_weights(lev)
        for p in range(len(lev.dims)):
            seg = wd[lev.offsets[p]:lev.offsets[p + 1]]
            if lev._cache["skip"][p]:
                assert np.all(seg == 0.0), (l, p)
            else:
                assert np.all(seg > 0.0), (l, p)


@pytest.mark.parametrize("relax", ["jacobi", "l1"])
def test_skip_vcycle_spd_and_pcg(relax):
    """With relaxation off on some levels the cycle is still symmetric positive
    definite (the finest level always relaxes) and PCG reaches the dense
    solution."""
    case = W.c1(6)
    A, h = fv_hierarchy(case, skip=True, relax=relax)
    assert _skip_levels(h)
    n = A.shape[0]
    B = np.column_stack([ssamg.vcycle(h, e) for e in np.eye(n)])
    assert np.max(np.abs(B - B.T)) <= 1e-12 * np.max(np.abs(B))
    assert np.linalg.eigvalsh(0.5 * (B + B.T)).min() > 0
    x_direct = sla.solve(A.toarray(), case.b, assume_a="pos")
    res = ssamg.solve(h, case.b, tol=1e-10, max_iter=200)
    assert res.converged
    assert np.linalg.norm(res.x - x_direct) <= 1e-8 * np.linalg.norm(x_direct)
