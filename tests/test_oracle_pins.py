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


# ---------------------------------------------------------------------------
# extraction helpers: the stencil and coupling layouts the parity tests read


def _cases_small():
    g = W.Geometry(3, [(9, 7, 5), (6, 7, 5), (5, 4, 6)], [(0, 0, 0), (9, 0, 0), (9, 7, 0)])
    raw = W.random_link_case(1, g, 27, junk_outside=True)
    A, _ = assemble.assemble_raw(g.dims, raw.stencils, raw.coeffs, raw.urow, raw.ucol, raw.uval)
    hraw = ssamg.setup(A, g.dims, raw.faces, raw.stencils, 3,
                       ustruct0=assemble.u_structure(raw.urow, raw.ucol, A.shape[0]))
    out = [("raw", hraw)]
    for name, mk in (("c1", lambda: W.c1(6)), ("c2", lambda: W.c2(5)), ("c3", lambda: W.c3(4)),
                     ("c4", lambda: W.c4(5, nrhs=1)), ("c5", lambda: W.c5(5))):
        out.append((name, fv_hierarchy(mk())[1]))
    return out


def _same_part_from_stencils(lev, values):
    """Rebuild the same-part operator of a level from per-part stencil arrays."""
    rows, cols, vals = [], [], []
    for p, (nx, ny, nz) in enumerate(lev.dims):
        k, j, i = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
        i, j, k = i.reshape(-1), j.reshape(-1), k.reshape(-1)
        for e, (dx, dy, dz) in enumerate(lev.pattern[p]):
            inb = ((i + dx >= 0) & (i + dx < nx) & (j + dy >= 0) & (j + dy < ny)
                   & (k + dz >= 0) & (k + dz < nz))
            r = lev.offsets[p] + i + nx * (j + ny * k)
            c = lev.offsets[p] + (i + dx) + nx * ((j + dy) + ny * (k + dz))
            rows.append(r[inb])
            cols.append(c[inb])
            vals.append(values[p][e][inb])
            # nothing may be stored for a neighbour outside the box
            assert np.all(values[p][e][~inb] == 0.0)
    import scipy.sparse as sps
    return sps.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                          shape=lev.A.shape)


def test_stencil_extraction_rebuilds_the_operator():
    """stencil_values (entry by entry) and stencil_values_fast (vectorised)
    agree bit for bit on every level of every workload shape, and the stencils
    put back in place give exactly the same-part entries of A_l (a transposed
    offset, a wrong code or a dropped entry changes the rebuilt matrix)."""
    for name, h in _cases_small():
        for l, lev in enumerate(h.levels):
            slow = [ssamg.stencil_values(lev, p) for p in range(len(lev.dims))]
            fast = [ssamg.stencil_values_fast(lev, p) for p in range(len(lev.dims))]
            for p in range(len(lev.dims)):
                assert np.array_equal(slow[p], fast[p]), (name, l, p)
            S = _same_part_from_stencils(lev, fast)
            part = np.repeat(np.arange(len(lev.dims)), np.diff(lev.offsets))
            A = lev.A.tocoo()
            m = part[A.row] == part[A.col]
            import scipy.sparse as sps
            AS = sps.csr_matrix((A.data[m], (A.row[m], A.col[m])), shape=A.shape)
            assert abs(S - AS).max() == 0.0, (name, l)


def test_coupling_extraction_is_the_cross_part_operator():
    """coupling_csr reads exactly the cross-part entries of A_l on the symbolic
    structure: stencils + couplings rebuild A_l, every stored entry crosses
    parts, and every nonzero cross-part entry of A_l is stored."""
    import scipy.sparse as sps
    for name, h in _cases_small():
        for l, lev in enumerate(h.levels):
            rp, col, val = ssamg.coupling_csr(lev)
            n = lev.n
            rows = np.repeat(np.arange(n), np.diff(rp))
            part = np.repeat(np.arange(len(lev.dims)), np.diff(lev.offsets))
            assert np.all(part[rows] != part[col]), (name, l)
            assert np.all(np.diff(col)[np.diff(rows) == 0] > 0), (name, l)   # sorted, no duplicates
            U = sps.csr_matrix((val, (rows, col)), shape=(n, n))
            S = _same_part_from_stencils(lev, [ssamg.stencil_values_fast(lev, p)
                                               for p in range(len(lev.dims))])
            assert abs(S + U - lev.A).max() == 0.0, (name, l)
            A = lev.A.tocoo()
            cross = (part[A.row] != part[A.col]) & (A.data != 0)
            if cross.any():
                st = lev.ustruct.tocsr()
                got = np.asarray(st[A.row[cross], A.col[cross]]).ravel()
                assert np.all(got == 1.0), (name, l)


def _zero_smoother(h):
    for lev in h.levels:
        lev._cache["wd"] = np.zeros(lev.n)


def test_direct_coarsest_branch_is_the_exact_inverse():
    """coarse = "direct": with one level the cycle is A^{-1} b itself; with two
    levels and the smoother switched off it is P (P^T A P)^{-1} P^T, so B A P = P
    (the coarse correction reproduces every interpolated vector exactly)."""
    case = W.c2(4)
    _, h1 = fv_hierarchy(case, max_levels=1, coarse="direct")
    A = h1.levels[0].A.toarray()
    b = np.random.default_rng(4).uniform(-1, 1, A.shape[0])
    assert np.allclose(ssamg.vcycle(h1, b), np.linalg.inv(A) @ b, rtol=0, atol=1e-12)
    _, h2 = fv_hierarchy(case, max_levels=2, coarse="direct")
    _zero_smoother(h2)
    P = h2.levels[0].P.toarray()
    A0 = h2.levels[0].A.toarray()
    B = np.column_stack([ssamg.vcycle(h2, e) for e in np.eye(A0.shape[0])])
    Ac = h2.levels[1].A.toarray()
    assert np.allclose(B, P @ np.linalg.inv(Ac) @ P.T, rtol=0, atol=1e-12)
    assert np.allclose(B @ A0 @ P, P, rtol=0, atol=1e-10)


def test_fv_27_point_edge_corner_and_interface_conductances():
    """Hand values of the finite-volume rule: an edge link has geometric weight
    1/2, a corner link 1/4, across a part face the conductivity is the harmonic
    mean of the two sides, and a side's directional factor is the mean of its
    part's factors over the link's nonzero directions."""
    g = W.Geometry(3, [(2, 2, 2), (2, 2, 2)], [(0, 0, 0), (2, 0, 0)])
    kap = np.arange(1.0, 17.0)            # cell c has kappa c + 1
    aniso = np.array([[2.0, 1.0, 1.0], [1.0, 3.0, 1.0]])
    A, _ = assemble.assemble_fv(g, 27, kap, aniso)

    def cid(p, i, j, k):
        return 8 * p + i + 2 * (j + 2 * k)

    def H(x, y):
        return 2 * x * y / (x + y)

    i0 = cid(0, 0, 0, 0)
    # inside part 0: edge (0,1,1) -> factor (1+1)/2 = 1, corner (1,1,1) -> (2+1+1)/3
    e = cid(0, 0, 1, 1)
    assert A[i0, e] == pytest.approx(-0.5 * H(1.0 * kap[i0], 1.0 * kap[e]), rel=1e-15)
    c = cid(0, 1, 1, 1)
    assert A[i0, c] == pytest.approx(-0.25 * H(4 / 3 * kap[i0], 4 / 3 * kap[c]), rel=1e-15)
    # across the part face x = 2: cell (1,0,0) of part 0 to (0,1,0) of part 1 (edge
    # (1,1,0)): factors (2+1)/2 and (1+3)/2; corner (1,1,1): (2+1+1)/3 and (1+3+1)/3
    a = cid(0, 1, 0, 0)
    eb = cid(1, 0, 1, 0)
    assert A[a, eb] == pytest.approx(-0.5 * H(1.5 * kap[a], 2.0 * kap[eb]), rel=1e-15)
    cb = cid(1, 0, 1, 1)
    assert A[a, cb] == pytest.approx(-0.25 * H(4 / 3 * kap[a], 5 / 3 * kap[cb]), rel=1e-15)
    # face link across the interface: harmonic mean of 2 kappa_a and 1 kappa_b
    fb = cid(1, 0, 0, 0)
    assert A[a, fb] == pytest.approx(-H(2.0 * kap[a], 1.0 * kap[fb]), rel=1e-15)
    assert A[a, fb] == A[fb, a]
    # a corner cell of the domain: its row sum is its ghost links, with the
    # ghost's kappa equal to its own: 3 faces, 9 edges (3 in-domain), 7 corners
    # (1 in-domain) of the 26 links point outside for cell (0,0,0) of part 0
    k0 = kap[i0]
    fsum = (2.0 + 1.0 + 1.0) * k0            # -x, -y, -z faces
    esum = 0.0
    for s in [(dx, dy, dz) for dx in (-1, 0, 1) for dy in (-1, 0, 1) for dz in (-1, 0, 1)
              if sum(v != 0 for v in (dx, dy, dz)) == 2]:
        if min(s) < 0:   # some component points out of the domain
            f = np.mean([aniso[0][d] for d in range(3) if s[d] != 0])
            esum += 0.5 * f * k0
    csum = sum(0.25 * (4 / 3) * k0 for s in range(8) if s != 7)   # 7 of 8 corners leave
    assert float(A[i0].sum()) == pytest.approx(fsum + esum + csum, rel=1e-13)


def _pb_case(a=10.0):
    """Two parts of 4 x 3 x 3 along x, 7-point, anisotropy (a,1,1) in both: d* = x
    on level 0 and the last x cell of part 0 (odd) has its +x neighbour across
    the part face."""
    g = W.Geometry(3, [(4, 3, 3), (4, 3, 3)], [(0, 0, 0), (4, 0, 0)])
    return W.FVCase("pb", g, 7, np.ones(g.n), np.array([[a, 1.0, 1.0]] * 2),
                    np.random.default_rng(0).uniform(-1, 1, g.n))


def test_lumped_part_boundary_weight_by_hand():
    """R-pb2 next to a Dirichlet face: the F cell (3,0,1) of part 0 has links
    a (-x, same part), a (+x, across the part face), ghost 1 (-y), 1 (+y), 1, 1
    (z): diagonal 2a + 4, collapse denominator 2a + 1, so the lumped weight is
    (a + a)/(2a + 1) where the literal reading gives 1; on the zero-sum row of
    cell (3,1,1) (no Dirichlet face) both give exactly 1."""
    a = 10.0
    case = _pb_case(a)
    _, h1 = fv_hierarchy(case, pb="one")
    _, h2 = fv_hierarchy(case, pb="lump")
    assert h1.levels[0].dstar[0] == 0 and h2.levels[0].dstar[0] == 0
    fn = (2, 3, 3)                       # F-box of part 0: odd x cells 1 and 3

    def fidx(i, j, k):
        return (i - 1) // 2 + fn[0] * (j + fn[1] * k)

    assert h1.levels[0].wm[0][fidx(3, 0, 1)] == 1.0
    assert h2.levels[0].wm[0][fidx(3, 0, 1)] == pytest.approx(2 * a / (2 * a + 1), rel=1e-15)
    assert h2.levels[0].wm[0][fidx(3, 1, 1)] == pytest.approx(1.0, rel=1e-15)
    assert h1.levels[0].wm[0][fidx(3, 1, 1)] == 1.0
    # away from the part face the two readings give the same weights
    assert h1.levels[0].wm[0][fidx(1, 0, 1)] == h2.levels[0].wm[0][fidx(1, 0, 1)]


@pytest.mark.parametrize("mk", [lambda: W.c2(6), lambda: W.c3(4), lambda: W.c5(6)])
def test_lumped_part_boundary_hierarchy(mk):
    """With R-pb2 every coarse operator stays SPD, P's row sums stay in [0, 1]
    on M-matrix levels, the V-cycle is SPD and PCG reaches the dense solution."""
    case = mk()
    _, h = fv_hierarchy(case, pb="lump")
    nm = 0
    for lev in h.levels[:-1]:
        rs = np.asarray(lev.P.sum(axis=1)).ravel()
        Ac = lev.A.tocoo()
        if np.all(Ac.data[Ac.row != Ac.col] <= 0):      # M-matrix level
            nm += 1
            assert np.all(rs >= -1e-14) and np.all(rs <= 1 + 1e-14)
    assert nm >= 1
    for lev in h.levels[1:4]:
        Ad = lev.A.toarray()
        assert np.allclose(Ad, Ad.T, rtol=0, atol=1e-12 * np.abs(Ad).max())
        assert np.linalg.eigvalsh(Ad).min() > 0
    n = h.levels[0].n
    if n <= 1500:
        B = np.column_stack([ssamg.vcycle(h, e) for e in np.eye(n)])
        assert np.allclose(B, B.T, atol=1e-12 * np.abs(B).max())
        assert np.linalg.eigvalsh(0.5 * (B + B.T)).min() > 0
    ref = ssamg.solve(h, case.b, tol=1e-10)
    xd = np.linalg.solve(h.levels[0].A.toarray(), case.b)
    assert ref.converged and np.linalg.norm(ref.x - xd) <= 1e-8 * np.linalg.norm(xd)


def test_hybrid_tail_is_an_exact_solve_at_the_switch_level():
    """hybrid_level = k (Section 3.5): k + 1 levels, and the cycle equals the
    same hierarchy's cycle with an exact coarsest solve; with the smoother off
    and k = 1 it is P A_1^{-1} P^T, so B A P = P."""
    case = W.c2(6)
    _, hk = fv_hierarchy(case, hybrid_level=3)
    _, hd = fv_hierarchy(case, max_levels=4, coarse="direct")
    assert hk.nlevels == 4 and hk.coarse == "direct"
    r = np.random.default_rng(8).uniform(-1, 1, hk.levels[0].n)
    assert np.array_equal(ssamg.vcycle(hk, r), ssamg.vcycle(hd, r))
    zk = ssamg.vcycle(hk, r)
    _, hs = fv_hierarchy(case, max_levels=4)
    assert np.linalg.norm(zk - ssamg.vcycle(hs, r)) > 0     # the exact solve changes the cycle
    _, h1 = fv_hierarchy(case, hybrid_level=1)
    _zero_smoother(h1)
    A0 = h1.levels[0].A.toarray()
    P = h1.levels[0].P.toarray()
    B = np.column_stack([ssamg.vcycle(h1, e) for e in np.eye(A0.shape[0])])
    assert np.allclose(B @ A0 @ P, P, rtol=0, atol=1e-10)


# ---------------------------------------------------------------------------
# parts of several boxes and glued faces (Section 2; test cases 3 and 4)


def _topo_matrix(case):
    A, off, faces = assemble.assemble_semistructured(case.dims, case.stencils, case.coeffs, case.urow,
                                                     case.ucol, case.uval, case.boxes, case.neighbors)
    return A, off, faces


def _two_cubes(m, rotated, seed=3):
    """Two m^3 parts along x, isotropic Laplacian with a random diagonal margin,
    glued through part 0's +x face; part 1 either in the same orientation or
    turned by a quarter about z ((i, j, k) -> (m-1-j, i, k))."""
    offs = W.stencil_offsets(7)
    rng = np.random.default_rng(seed)
    marg = [rng.uniform(0, 1, (m, m, m)) for _ in range(2)]      # [k][j][i]
    co = []
    for p in range(2):
        c = np.zeros((7, m, m, m))
        c[1:] = -1.0
        c[0] = 6.0 + marg[p]
        co.append(c)
    nb = [[None] * 6 for _ in range(2)]
    if not rotated:
        nb[0][1] = {"part": 1, "at": (m, 0, 0), "nbr_at": (0, 0, 0), "map": (0, 1, 2), "dir": (1, 1, 1)}
        nb[1][0] = {"part": 0, "at": (-1, 0, 0), "nbr_at": (m - 1, 0, 0), "map": (0, 1, 2), "dir": (1, 1, 1)}
    else:
        rot = np.empty_like(co[1])
        for i in range(m):
            for j in range(m):
                rot[:, :, i, m - 1 - j] = co[1][:, :, j, i]      # rotated cell (m-1-j, i) holds cell (i, j)
        co[1] = rot
        nb[0][1] = {"part": 1, "at": (m, 0, 0), "nbr_at": (m - 1, 0, 0), "map": (1, 0, 2), "dir": (1, -1, 1)}
        nb[1][2] = {"part": 0, "at": (0, -1, 0), "nbr_at": (m - 1, m - 1, 0), "map": (1, 0, 2),
                    "dir": (-1, 1, 1)}
    return W.TopoCase("two", [(m, m, m)] * 2, [offs] * 2, co, [None, None], nb,
                      np.zeros(0, dtype=np.int64), np.zeros(0, dtype=np.int64), np.zeros(0),
                      rng.uniform(-1, 1, 2 * m ** 3))


def test_cartesian_glue_is_the_placed_operator():
    """Gluing part 0's +x face to part 1's -x face without rotation gives the
    operator of the same two cubes placed side by side (the finite-volume rule
    with kappa = 1 and no margin: -1 per link, 6 on the diagonal)."""
    m = 4
    case = _two_cubes(m, rotated=False)
    for c in case.coeffs:
        c[0] = 6.0
    A, off, faces = _topo_matrix(case)
    g = W.geometry_along_x(2, [(m, m, m)] * 2)
    B, _ = assemble.assemble_fv(g, 7, np.ones(g.n), np.ones((2, 3)))
    assert abs(A - B).max() == 0.0
    assert faces.tolist() == [[0, 1, 0, 0, 0, 0], [1, 0, 0, 0, 0, 0]]


def test_quarter_turned_part_is_a_permutation():
    """Turning part 1's index space by a quarter (and its gluing with it) gives
    the same matrix with part 1's cells renumbered: east couplings of part 0
    meet north-south couplings of part 1, as in the paper's non-Cartesian case."""
    m = 4
    A, off, _ = _topo_matrix(_two_cubes(m, rotated=False))
    R, _, faces = _topo_matrix(_two_cubes(m, rotated=True))
    assert faces.tolist() == [[0, 1, 0, 0, 0, 0], [0, 0, 1, 0, 0, 0]]
    perm = np.arange(2 * m ** 3)             # rotated numbering of each Cartesian cell
    for k in range(m):
        for j in range(m):
            for i in range(m):
                perm[m ** 3 + i + m * (j + m * k)] = m ** 3 + (m - 1 - j) + m * (i + m * k)
    P = np.zeros((2 * m ** 3, 2 * m ** 3))
    P[perm, np.arange(2 * m ** 3)] = 1.0
    assert np.array_equal(P @ A.toarray() @ P.T, R.toarray())


def test_l_shaped_part_by_brute_force():
    """A part made of two boxes (an L) inside a 6 x 6 x 3 box: the active cells'
    rows are the 7-point Laplacian of the L-shaped domain built cell by cell;
    the cells outside both boxes have identity rows and no couplings."""
    offs = W.stencil_offsets(7)
    dims = [(6, 6, 3)]
    co = np.random.default_rng(5).uniform(-3, 3, (7, 3, 6, 6))      # junk everywhere
    co[1:] = -1.0
    co[0] = 6.0
    boxes = [[((0, 0, 0), (5, 2, 2)), ((0, 3, 0), (2, 5, 2))]]
    case = W.TopoCase("L", dims, [offs], [co], boxes, [[None] * 6], np.zeros(0, dtype=np.int64),
                      np.zeros(0, dtype=np.int64), np.zeros(0), np.zeros(108))
    A, _, _ = _topo_matrix(case)
    act = lambda i, j, k: 0 <= k < 3 and ((0 <= i < 6 and 0 <= j < 3) or (0 <= i < 3 and 3 <= j < 6))
    D = A.toarray()
    for k in range(3):
        for j in range(6):
            for i in range(6):
                r = i + 6 * (j + 6 * k)
                want = np.zeros(108)
                if not act(i, j, k):
                    want[r] = 1.0
                else:
                    want[r] = 6.0
                    for dx, dy, dz in offs[1:]:
                        if act(i + dx, j + dy, k + dz):
                            want[(i + dx) + 6 * ((j + dy) + 6 * (k + dz))] = -1.0
                assert np.array_equal(D[r], want), (i, j, k)


def test_tc3_junction_invariants():
    """Three cubes glued around one edge: A is symmetric and SPD, every glued
    face contributes m^2 couplings of -1 each way, interior and glued rows sum
    to zero, and PCG with SSAMG reaches the dense solution."""
    m = 5
    case = W.tc3_junction(m)
    A, off, faces = _topo_matrix(case)
    D = A.toarray()
    assert np.array_equal(D, D.T) and np.linalg.eigvalsh(D).min() > 0
    C = assemble.cross_structure(A, off)
    assert C.nnz == 2 * 3 * m * m
    assert np.all(A[C.nonzero()] == -1.0)
    part = np.repeat(np.arange(3), m ** 3)
    h = ssamg.setup(A, case.dims, faces, case.stencils, 3, ustruct0=C)
    ref = ssamg.solve(h, case.b, tol=1e-10)
    xd = np.linalg.solve(D, case.b)
    assert ref.converged and np.linalg.norm(ref.x - xd) <= 1e-8 * np.linalg.norm(xd)
    # every part coarsens along the same directions (isotropic, equal boxes)
    assert [l.dstar[0] for l in h.levels] == [l.dstar[1] for l in h.levels] == [l.dstar[2] for l in h.levels]
    assert part.size == A.shape[0]


def test_tc4_samr_invariants():
    """SAMR: ghost rows are the identity, fine-coarse couplings are -2/3 both
    ways (four per coarse face of the patch), the patch's rows sum to zero,
    A is symmetric and SPD, and PCG with SSAMG reaches the dense solution."""
    m = 8
    case = W.tc4_samr(m)
    A, off, _ = _topo_matrix(case)
    D = A.toarray()
    assert np.array_equal(D, D.T) and np.linalg.eigvalsh(D).min() > 0
    a, b = m // 4, 3 * m // 4
    for k in range(a, b):
        for j in range(a, b):
            for i in range(a, b):
                r = i + m * (j + m * k)
                row = np.zeros(D.shape[0])
                row[r] = 1.0
                assert np.array_equal(D[r], row)
    C = assemble.cross_structure(A, off)
    assert np.allclose(A[C.nonzero()], -2.0 / 3.0, rtol=0, atol=0)
    assert C.nnz == 2 * 6 * m * m                    # every fine boundary cell face, both ways
    rs = np.asarray(A.sum(axis=1)).ravel()
    assert np.max(np.abs(rs[m ** 3:])) <= 1e-13      # the patch is interior
    h = ssamg.setup(A, case.dims, case.face_kinds(), case.stencils, 3, ustruct0=C)
    ref = ssamg.solve(h, case.b, tol=1e-10)
    xd = np.linalg.solve(D, case.b)
    assert ref.converged and np.linalg.norm(ref.x - xd) <= 1e-8 * np.linalg.norm(xd)


# ---------------------------------------------------------------------------
# non-Galerkin coarse operator for star stencils (Section 5, reading R-ng)


def _interior_stencil(lev, p=0):
    vals = ssamg.stencil_values_fast(lev, p)
    nx, ny, nz = lev.dims[p]
    c = nx // 2 + nx * (ny // 2 + ny * (nz // 2))
    return {tuple(int(a) for a in t): vals[e, c] for e, t in enumerate(lev.pattern[p])}


def test_nongalerkin_constant_laplacian_is_the_coarse_cell_discretisation():
    """On the constant 7-point Laplacian (conductance 1 per face) the
    non-Galerkin operator of a level is the finite-volume stencil of the
    coarsened cells: a face of area A between centers a distance h apart
    conducts A/h.  Level 1 (cells 2x1x1): x 1/2, y and z 2, center 9; level 2
    (2x2x1): x and y 1, z 4, center 12.  A missing half, a rerouting to one
    side of the rectangle only or a wrong diagonal all change these numbers
    (the Galerkin level 1 has +1/2 along x and -1/4 on the diagonals)."""
    _, h = fv_hierarchy(W.c1(16), coarse_op="nongalerkin")
    assert [lev.dstar[0] for lev in h.levels[:2]] == [0, 1]
    want1 = {(0, 0, 0): 9.0, (-1, 0, 0): -0.5, (1, 0, 0): -0.5, (0, -1, 0): -2.0, (0, 1, 0): -2.0,
             (0, 0, -1): -2.0, (0, 0, 1): -2.0}
    want2 = {(0, 0, 0): 12.0, (-1, 0, 0): -1.0, (1, 0, 0): -1.0, (0, -1, 0): -1.0, (0, 1, 0): -1.0,
             (0, 0, -1): -4.0, (0, 0, 1): -4.0}
    for lev, want in ((h.levels[1], want1), (h.levels[2], want2)):
        got = _interior_stencil(lev)
        assert set(got) == set(want)
        for k, v in want.items():
            assert abs(got[k] - v) < 1e-13, (k, got[k], v)
    _, hg = fv_hierarchy(W.c1(16))
    g1 = _interior_stencil(hg.levels[1])
    assert abs(g1[(1, 0, 0)] - 0.5) < 1e-13 and abs(g1[(1, 1, 0)] + 0.25) < 1e-13


def _ng_cases():
    g = W.Geometry(3, [(8, 7, 6), (6, 7, 6), (5, 4, 6)], [(0, 0, 0), (8, 0, 0), (8, 7, 0)])
    raw = W.random_link_case(11, g, 7)
    A, _ = assemble.assemble_raw(g.dims, raw.stencils, raw.coeffs, raw.urow, raw.ucol, raw.uval)
    hraw = ssamg.setup(A, g.dims, raw.faces, raw.stencils, 3, coarse_op="nongalerkin",
                       ustruct0=assemble.u_structure(raw.urow, raw.ucol, A.shape[0]))
    return [("raw", hraw), ("c5", fv_hierarchy(W.c5(8), coarse_op="nongalerkin")[1]),
            ("c2", fv_hierarchy(W.c2(6), coarse_op="nongalerkin")[1])]


@pytest.mark.parametrize("name", ["raw", "c5", "c2"])
def test_nongalerkin_invariants(name):
    """Every level of a non-Galerkin hierarchy on variable coefficients: star
    patterns only; symmetric (a rerouting to the wrong neighbour breaks this
    once coefficients vary); every row sum equal to that of the Galerkin
    product of the level above (pins the diagonal); the cross-part entries
    and the entries of parts that did not coarsen untouched; positive
    definite; and PCG converges."""
    h = dict(_ng_cases())[name]
    for l in range(1, h.nlevels):
        lev, up = h.levels[l], h.levels[l - 1]
        for p in range(len(lev.dims)):
            assert all(np.count_nonzero(t) <= 1 for t in lev.pattern[p])
        A = lev.A
        assert abs(A - A.T).max() <= 1e-13 * abs(A).max()
        G = ssamg.galerkin(up.A, up.P)
        assert np.allclose(np.asarray(A.sum(axis=1)).ravel(), np.asarray(G.sum(axis=1)).ravel(),
                           rtol=0, atol=1e-12 * abs(A).max())
        part = assemble.cell_coords(lev.dims, lev.offsets)[0]
        D = (A - G).tocoo()
        D.data[abs(D.data) <= 1e-13 * abs(A).max()] = 0
        D.eliminate_zeros()
        assert np.all(part[D.row] == part[D.col])
        moved = {p for p in range(len(lev.dims)) if up.dstar[p] >= 0}
        assert set(np.unique(part[D.row]).tolist()) <= moved
        if A.shape[0] <= 1500:
            assert np.linalg.eigvalsh(A.toarray()).min() > 0
    r = np.random.default_rng(4).uniform(-1, 1, h.levels[0].n)
    res = ssamg.solve(h, r)
    assert res.converged and res.iters <= 30


def test_nongalerkin_leaves_other_stencils_galerkin():
    """A 27-point part is not a star: the option changes nothing there."""
    case = W.c3(4)
    _, h = fv_hierarchy(case, coarse_op="nongalerkin")
    _, hg = fv_hierarchy(case)
    for a, b in zip(h.levels, hg.levels):
        assert (a.A != b.A).nnz == 0
