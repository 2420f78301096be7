"""Shared helpers of the GPU parity tests: build the same workload on both sides
(oracle on the CPU, the HIP library through its C ABI) and compare level data."""
import numpy as np

import workloads as W
from oracle import assemble, ssamg as O


def oracle_fv(case, **kw):
    A, _ = assemble.assemble_fv(case.geometry, case.stencil, case.kappa, case.aniso)
    g = case.geometry
    pat = [W.stencil_offsets(case.stencil, g.ndim)] * g.nparts
    return O.setup(A, g.dims, g.face_kinds(), pat, g.ndim, omega=kw.get("omega", case.omega),
                   max_levels=kw.get("max_levels", 64), min_coarse_size=kw.get("min_coarse_size", 0),
                   relax=kw.get("relax", case.relax), coarse=kw.get("coarse", "sweep"),
                   skip=kw.get("skip", False), pb=kw.get("pb", "one"),
                   hybrid_level=kw.get("hybrid_level", 0),
                   coarse_op=kw.get("coarse_op", "galerkin"))


def oracle_raw(case, **kw):
    g = case.geometry
    A, _ = assemble.assemble_raw(g.dims, case.stencils, case.coeffs, case.urow, case.ucol, case.uval)
    return O.setup(A, g.dims, case.faces, case.stencils, g.ndim, omega=kw.get("omega", 0.0),
                   ustruct0=assemble.u_structure(case.urow, case.ucol, A.shape[0]),
                   max_levels=kw.get("max_levels", 64), min_coarse_size=kw.get("min_coarse_size", 0),
                   pb=kw.get("pb", "one"), coarse_op=kw.get("coarse_op", "galerkin"))


def gpu_fv(case, **params):
    import torch
    from paper_2205_14273_amd.ssamg import Problem, Solver
    kappa = torch.as_tensor(case.kappa, device="cuda")
    pr = Problem.from_fv(case.geometry, case.stencil, kappa, case.aniso)
    if case.omega > 0 and "omega" not in params:
        params["omega"] = case.omega
    if "relax" not in params:
        params["relax"] = 1 if case.relax == "l1" else 0
    elif isinstance(params["relax"], str):
        params["relax"] = 1 if params["relax"] == "l1" else 0
    s = Solver(pr, **params).setup()
    return pr, s


def gpu_raw(case, **params):
    from paper_2205_14273_amd.ssamg import Problem, Solver
    pr = Problem.from_raw(case)
    s = Solver(pr, **params).setup()
    return pr, s


def row_rel_err(a, b):
    """max over rows of max_j |a_ij - b_ij| / max_j |b_ij| (rows = cells, axis 1)."""
    scale = np.max(np.abs(b), axis=0)
    scale = np.where(scale > 0, scale, 1.0)
    return float(np.max(np.max(np.abs(a - b), axis=0) / scale)) if a.size else 0.0


def compare_hierarchy(h, s, nparts, rtol=1e-12, check_values=True):
    """Integer data bit-exact; stencils, weights and couplings to rtol."""
    assert s.nlevels == h.nlevels, (s.nlevels, h.nlevels)
    for l, lev in enumerate(h.levels):
        for p in range(nparts):
            li = s.level_info(l, p)
            assert tuple(li["dims"]) == tuple(lev.dims[p]), (l, p)
            assert li["dstar"] == lev.dstar[p], (l, p, li["dstar"], lev.dstar[p])
            assert abs(li["omega"] - float(lev.omega[p])) <= 1e-15, (l, p)
            assert np.array_equal(li["pattern"], np.asarray(lev.pattern[p])), (l, p)
            if not check_values:
                continue
            want = O.stencil_values_fast(lev, p)
            got = s.copy_stencil(l, p)
            assert row_rel_err(got, want) <= rtol, (l, p, row_rel_err(got, want))
            if l < h.nlevels - 1 and lev.dstar[p] >= 0:
                wm, wp = s.copy_interp(l, p)
                assert np.max(np.abs(wm - lev.wm[p])) <= rtol, (l, p)
                assert np.max(np.abs(wp - lev.wp[p])) <= rtol, (l, p)
        # coupling structure bit-exact, values to rtol relative to the row's diagonal
        rp, col, val = s.copy_coupling(l)
        st = lev.ustruct.tocsr()
        st.sort_indices()
        assert np.array_equal(rp, st.indptr.astype(np.int64)), l
        assert np.array_equal(col, st.indices.astype(np.int64)), l
        if check_values and len(val):
            orp, ocol, oval = O.coupling_csr(lev)
            diag = np.abs(lev.A.diagonal())
            rows = np.repeat(np.arange(len(rp) - 1), np.diff(rp))
            assert np.max(np.abs(val - oval) / diag[rows]) <= rtol, l


# Element-wise tolerances of the V-cycle z = B r against the oracle: FP64 kernels
# differ from the oracle only in summation order; the FP32 cycle rounds every
# operation to FP32 (unit roundoff 6e-8) through ~20 levels of a few operations.
CYCLE_RTOL = {0: 1e-12, 1: 2e-5}


def vcycle_scale(h, r):
    """Rounding scale of each entry of the oracle's V-cycle z = B r: the same
    recursion with every operator (A_l, P_l, the smoother factors, the coarsest
    solve) replaced by its entrywise absolute value, applied to |r|.  Any
    implementation that forms the same sums in another order or precision
    changes z_i by at most a small multiple of this value, so a local error on a
    row of small magnitude cannot hide under a norm of the whole vector."""
    L = h.nlevels

    def rec(l, bl):
        lev = h.levels[l]
        wd = np.abs(O._cell_weights(lev))
        Aa = abs(lev.A)
        if l == L - 1:
            if h.coarse == "direct":
                return np.abs(np.linalg.inv(lev.A.toarray())) @ bl
            return wd * bl
        x = wd * bl
        rr = bl + Aa @ x
        xc = rec(l + 1, abs(lev.P).T @ rr)
        x = x + abs(lev.P) @ xc
        return x + wd * (bl + Aa @ x)

    return rec(0, np.abs(np.asarray(r, dtype=np.float64)))


def assert_cycle_close(z, want, scale, rtol, what=""):
    """|z_i - want_i| <= rtol * scale_i for every entry."""
    err = np.abs(np.asarray(z) - np.asarray(want))
    ratio = err / np.maximum(scale, 1e-300)
    worst = int(np.argmax(ratio))
    assert ratio[worst] <= rtol, (what, worst, float(ratio[worst]), rtol)
    return float(ratio[worst])


def oracle_topo(case, **kw):
    """Oracle hierarchy of a problem with parts of several boxes and glued faces."""
    A, off, faces = assemble.assemble_semistructured(case.dims, case.stencils, case.coeffs, case.urow,
                                                     case.ucol, case.uval, case.boxes, case.neighbors)
    return O.setup(A, case.dims, case.face_kinds(), case.stencils, case.ndim,
                   ustruct0=assemble.cross_structure(A, off), **kw)


def gpu_topo(case, **params):
    from paper_2205_14273_amd.ssamg import Problem, Solver
    pr = Problem.from_topo(case)
    s = Solver(pr, **params).setup()
    return pr, s
