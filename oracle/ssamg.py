"""Oracle: SSAMG setup, V(1,1) cycle and PCG in FP64 (test infrastructure only).

Written from the paper, step by step:

  direction_sums / grid_spacing   Section 3.1: c_d summed over the part's cells of
      minus the off-diagonal stencil coefficients with a nonzero d-component
      (sign-adjusted by the center), W_pd = sqrt(max_i c_i / c_d).
  coarsen                          Algorithm 1: per level and part, if the box
      has more than one cell, d* = argmin_d W_pd (ties to the smallest index),
      halve the box in d*, double W_pd*.
  relax_weight                     eq:relax1 / eq:alpha-beta:
      omega_p = 2 / (3 - beta_p/alpha_p).
  interpolation_weights            Section 3.2, eq:prolEx: two-point collapse of
      the row along d*; part-boundary rule (crossing weight 0, opposite 1).
  galerkin                         eq:galerkin: A_c = P^T A P (one sparse
      product; S_c and U_c are its same-part and cross-part entries).
  vcycle / pcg                     Section 3.4 and the Section 4 protocol.

Readings where the paper is silent or garbled (all are listed in the design notes):
  R-sign   eq:prolEx is printed without a minus sign; the weights used are
           -(sum of the +-1 coefficients along d*) / (sum of the 0 coefficients),
           which makes them positive for an M-matrix (1/2 for the Laplacian).
  R-tie    d* ties: W values within a relative 1e-10 are tied, smallest d wins;
           directions whose extent is 1 are not candidates.
  R-coarse even cells (index parity in the part's own index space, lower corner 0)
           are coarse; coarse index i/2; coarse extent ceil(n/2).
  R-pb     part-boundary rule: the weight that would cross a part face is absent
           and the opposite weight is set to 1.
  R-pb2    (option pb="lump") the opposite weight instead takes the dropped
           weight on top, the dropped weight being the collapse of the row's
           couplings, -(sum_j u_fj)/den over all of the row's cross-part entries
           (the only reading available on coarse levels, where entries of U
           carry no offset); on rows of zero sum it equals R-pb, next to a
           Dirichlet face it is smaller than 1.  Rows whose denominator is not
           positive keep weight 1.
  R-den    the collapse is undefined where its denominator (the sum of the
           row's coefficients with zero d* component) is not positive, which
           happens on Galerkin operators of strongly heterogeneous problems;
           there the weights are the row's -d* and +d* coefficient sums divided
           by their total (constants are interpolated), or 1/2 each when that
           total is not negative.  Rows with a positive denominator are
           untouched.
  R-omega  omega at level l uses W at level l (before that level's doubling) and
           d*_l; a part that no longer coarsens uses d* = argmin W; the sums in
           eq:alpha-beta run over d = 0 .. n_d - 1.
  R-stop   coarsen until every part is a single cell (coarsest size = n_parts)
           unless max_levels or min_coarse_size stops earlier.
  R-last   the coarsest level gets one sweep of the same relaxation from zero
           (Section 3.5, non-hybrid case), or optionally a dense direct solve.
  R-skip   the "skip" option (Section 3.4): a part does not relax at level l >= n_d
           when it coarsens there along the same direction as at level l - n_d
           (d*_l = d*_{l-n_d} >= 0); the coarsest level and parts that no
           longer coarsen always relax.  Not relaxing means a zero smoother
           factor: no pre-sweep contribution and no post-sweep change.
  R-ng     the non-Galerkin coarse operator that Section 5 plans for isotropic
           problems (option coarse_op="nongalerkin") is not specified there.
           Reading: it applies to parts whose stencil is a star (every offset
           has at most one nonzero component, e.g. 7-point), keeps the star
           pattern on the coarse level, and starts from the Galerkin product.
           Each same-part entry (I, J) whose offset (t, Q) has both a nonzero
           component across d* (t) and along d* (Q) joins the corners of the
           rectangle I, K1 = I + t, J, K2 = I + Q; it is removed and half of
           its value is added to each of the four star entries (I, K1),
           (I, K2), (K1, J), (K2, J) along the rectangle's sides, and the
           diagonals of rows K1 and K2 lose half of it, so every row sum of
           the Galerkin operator is kept.  Seen as a graph Laplacian, each
           diagonal edge is replaced by the four sides of its rectangle at
           half its weight; a symmetric operator stays symmetric.  For the
           constant-coefficient Laplacian the result is the finite-volume
           stencil of the coarsened cells.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp

from .assemble import cell_coords

TIE_RTOL = 1e-10


@dataclass
class Level:
    dims: list                  # per-part box extents at this level
    offsets: np.ndarray         # cell offsets, length nparts + 1
    A: sp.csr_matrix            # full operator at this level
    pattern: list               # per-part symbolic stencil pattern [nent][3]
    ustruct: sp.csr_matrix      # 0/1 structure of the inter-part couplings
    dstar: list = field(default_factory=list)    # -1: part not coarsened here
    omega: np.ndarray = None    # per-part relaxation weight
    wm: list = field(default_factory=list)       # per-part F-box weights (toward -d*)
    wp: list = field(default_factory=list)       # per-part F-box weights (toward +d*)
    P: sp.csr_matrix = None     # interpolation to the next level
    _cache: dict = field(default_factory=dict)

    @property
    def n(self):
        return int(self.offsets[-1])


def _offsets(dims):
    return np.concatenate([[0], np.cumsum([a * b * c for a, b, c in dims])]).astype(np.int64)


def _entries(level):
    """COO of the level operator with local coordinates of both ends (cached)."""
    if "entries" in level._cache:
        return level._cache["entries"]
    A = level.A.tocoo()
    part, ci, cj, ck = cell_coords(level.dims, level.offsets)
    r, c = A.row.astype(np.int64), A.col.astype(np.int64)
    same = part[r] == part[c]
    s = np.stack([ci[c] - ci[r], cj[c] - cj[r], ck[c] - ck[r]], axis=1)
    level._cache["entries"] = (r, c, A.data, part, same, s)
    return level._cache["entries"]


# ---------------------------------------------------------------------------
# Section 3.1: grid-spacing metric and Algorithm 1


def direction_sums(level, ndim):
    """c[p][d] of Section 3.1 from the structured part S of the level operator.

    Correctly rounded sums (math.fsum) so the value does not depend on order.
    """
    r, c, v, part, same, s = _entries(level)
    diag = level.A.diagonal()
    sgn = np.where(diag[r] < 0, -1.0, 1.0)
    off = same & (r != c)
    nparts = len(level.dims)
    cd = np.zeros((nparts, 3))
    for p in range(nparts):
        sel = off & (part[r] == p)
        for d in range(ndim):
            m = sel & (s[:, d] != 0)
            cd[p, d] = math.fsum((-sgn[m] * v[m]).tolist())
    return cd


def grid_spacing(cd, ndim):
    """W_pd = sqrt(max_i c_i / c_d); a direction with c_d <= 0 gets W = inf."""
    nparts = cd.shape[0]
    W = np.full((nparts, 3), np.inf)
    for p in range(nparts):
        cmax = max(cd[p, :ndim])
        for d in range(ndim):
            if cd[p, d] > 0 and cmax > 0:
                W[p, d] = math.sqrt(cmax / cd[p, d])
    return W


def _argmin_tied(w, cand):
    wmin = min(w[d] for d in cand)
    for d in cand:
        if w[d] <= wmin * (1.0 + TIE_RTOL) or w[d] == wmin:
            return d
    return cand[0]


def relax_weight(Wp, dstar, ndim):
    """omega_p = 2 / (3 - beta_p / alpha_p) (eq:relax1, eq:alpha-beta)."""
    inv = [0.0 if not np.isfinite(Wp[d]) else 1.0 / (Wp[d] * Wp[d]) for d in range(ndim)]
    alpha = sum(inv)
    beta = sum(inv[d] for d in range(ndim) if d != dstar)
    ratio = beta / alpha if alpha > 0 else 0.0
    return 2.0 / (3.0 - ratio)


def coarsen(W0, dims0, ndim, max_levels=64, min_coarse_size=0):
    """Algorithm 1.  Returns per-level lists: dims, dstar, omega_auto."""
    W = np.array(W0, dtype=np.float64)
    dims = [tuple(d) for d in dims0]
    all_dims, all_dstar, all_omega = [dims], [], []
    while True:
        l = len(all_dims) - 1
        total = sum(a * b * c for a, b, c in dims)
        last = (all(a * b * c == 1 for a, b, c in dims) or l >= max_levels - 1
                or (min_coarse_size > 0 and total < min_coarse_size))
        dstar, omega, nxt = [], [], []
        for p, d in enumerate(dims):
            cand = [a for a in range(ndim) if d[a] > 1]
            if last or not cand:
                ds = _argmin_tied(W[p], list(range(ndim)))
                omega.append(relax_weight(W[p], ds, ndim))
                dstar.append(-1)
                nxt.append(d)
                continue
            ds = _argmin_tied(W[p], cand)
            omega.append(relax_weight(W[p], ds, ndim))
            dstar.append(ds)
            nd = list(d)
            nd[ds] = (d[ds] + 1) // 2
            nxt.append(tuple(nd))
            W[p, ds] *= 2.0
        all_dstar.append(dstar)
        all_omega.append(np.asarray(omega))
        if last:
            break
        dims = nxt
        all_dims.append(dims)
    return all_dims, all_dstar, all_omega


# ---------------------------------------------------------------------------
# Section 3.2: interpolation


def coarse_pattern(fine_pattern, dstar):
    """Symbolic coarse stencil: component d* maps 0 -> {-1,0,1}, +-1 -> {0,+-1};
    the others are unchanged.  Sorted by (dz, dy, dx)."""
    if dstar < 0:
        out = {tuple(int(v) for v in s) for s in fine_pattern}
    else:
        out = set()
        for s in fine_pattern:
            s = [int(v) for v in s]
            opts = (-1, 0, 1) if s[dstar] == 0 else (0, s[dstar])
            for t in opts:
                u = list(s)
                u[dstar] = t
                out.add(tuple(u))
    return np.asarray(sorted(out, key=lambda t: (t[2], t[1], t[0])), dtype=np.int32)


def interpolation_weights(level, p, dstar, faces, pb="one"):
    """(wm, wp) over the F-box of part p: F cells are the odd cells along d*.

    wm multiplies the coarse neighbour at -d*, wp the one at +d* (P_W, P_E of
    eq:prolEx, with the sign reading R-sign).  A neighbour outside the box on a
    physical face is simply absent; on a part face the crossing weight is zero
    and the opposite weight is 1 (R-pb, pb="one"), or (pb="lump", reading R-pb2)
    the opposite weight plus the dropped one, taken as the collapse of the
    row's couplings: -(sum over the row's cross-part entries)/den.
    """
    nx, ny, nz = level.dims[p]
    n = [nx, ny, nz]
    r, c, v, part, same, s = _entries(level)
    sel = same & (part[r] == p)
    rl = r[sel] - level.offsets[p]
    sd = s[sel, dstar]
    vv = v[sel]
    ncell = nx * ny * nz
    den = np.bincount(rl[sd == 0], weights=vv[sd == 0], minlength=ncell)
    sm = np.bincount(rl[sd == -1], weights=vv[sd == -1], minlength=ncell)
    spl = np.bincount(rl[sd == +1], weights=vv[sd == +1], minlength=ncell)
    fdims = list(n)
    fdims[dstar] = n[dstar] // 2
    fk, fj, fi = np.meshgrid(np.arange(fdims[2]), np.arange(fdims[1]), np.arange(fdims[0]),
                             indexing="ij")
    fc = [fi.reshape(-1), fj.reshape(-1), fk.reshape(-1)]
    fc[dstar] = 2 * fc[dstar] + 1                     # fine coordinate of each F cell
    lin = fc[0] + nx * (fc[1] + ny * fc[2])
    dd = den[lin]
    sml, spll = sm[lin], spl[lin]
    good = dd > 0
    with np.errstate(divide="ignore", invalid="ignore"):
        wm = np.where(good, -sml / np.where(good, dd, 1.0), 0.0)
        wp = np.where(good, -spll / np.where(good, dd, 1.0), 0.0)
        # R-den: where the collapse denominator is not positive the row's two
        # off-plane sums alone set the weights, normalised so that constants
        # are interpolated; with no attracting off-plane coupling, 1/2 each
        ssum = sml + spll
        att = ssum < 0
        safe = np.where(att, ssum, 1.0)
        wm = np.where(good, wm, np.where(att, sml / safe, 0.5))
        wp = np.where(good, wp, np.where(att, spll / safe, 0.5))
    if not (np.all(np.isfinite(wm)) and np.all(np.isfinite(wp))):
        raise FloatingPointError("non-finite interpolation weight")
    lo_out = fc[dstar] - 1 < 0
    hi_out = fc[dstar] + 1 > n[dstar] - 1
    wm = np.where(lo_out, 0.0, wm)
    wp = np.where(hi_out, 0.0, wp)
    one_m = one_p = 1.0
    if pb == "lump":
        cross = ~same & (part[r] == p)
        usum = np.bincount(r[cross] - level.offsets[p], weights=v[cross], minlength=ncell)[lin]
        with np.errstate(divide="ignore", invalid="ignore"):
            one_m = np.where(good, -(sml + usum) / np.where(good, dd, 1.0), 1.0)
            one_p = np.where(good, -(spll + usum) / np.where(good, dd, 1.0), 1.0)
    elif pb != "one":
        raise ValueError("pb must be 'one' or 'lump'")
    if faces[p][2 * dstar + 1]:          # + face is a part boundary
        wm = np.where(hi_out & ~lo_out, one_m, wm)
    if faces[p][2 * dstar]:              # - face is a part boundary
        wp = np.where(lo_out & ~hi_out, one_p, wp)
    return wm, wp


def interpolation_matrix(level, cdims, coffsets):
    """P (N_l x N_{l+1}) from d* and the F-box weights of every part."""
    rows, cols, vals = [], [], []
    for p, (nx, ny, nz) in enumerate(level.dims):
        ds = level.dstar[p]
        cx, cy, cz = cdims[p]
        k, j, i = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
        i, j, k = i.reshape(-1), j.reshape(-1), k.reshape(-1)
        fid = level.offsets[p] + i + nx * (j + ny * k)
        if ds < 0:
            rows.append(fid)
            cols.append(coffsets[p] + i + cx * (j + cy * k))
            vals.append(np.ones(fid.size))
            continue
        f = [i, j, k]
        even = f[ds] % 2 == 0

        def cid(cc):
            return coffsets[p] + cc[0] + cx * (cc[1] + cy * cc[2])

        cc = list(f)
        cc[ds] = f[ds] // 2
        rows.append(fid[even])
        cols.append(cid(cc)[even])
        vals.append(np.ones(int(even.sum())))
        # odd cells: F-box index
        n = [nx, ny, nz]
        fdims = list(n)
        fdims[ds] = n[ds] // 2
        ff = list(f)
        ff[ds] = (f[ds] - 1) // 2
        flin = ff[0] + fdims[0] * (ff[1] + fdims[1] * ff[2])
        odd = ~even
        wm, wp = level.wm[p], level.wp[p]
        # -d* neighbour: coarse index (f-1)/2, present when f-1 >= 0
        cm = list(f)
        cm[ds] = (f[ds] - 1) // 2
        has_m = odd & (f[ds] - 1 >= 0)
        rows.append(fid[has_m])
        cols.append(cid(cm)[has_m])
        vals.append(wm[flin[has_m]])
        cpl = list(f)
        cpl[ds] = (f[ds] + 1) // 2
        has_p = odd & (f[ds] + 1 <= n[ds] - 1)
        rows.append(fid[has_p])
        cols.append(cid(cpl)[has_p])
        vals.append(wp[flin[has_p]])
    P = sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(level.n, int(coffsets[-1])))
    P.sort_indices()
    return P


def galerkin(A, P):
    """eq:galerkin: A_c = P^T A P."""
    Ac = (P.T @ A @ P).tocsr()
    Ac.sort_indices()
    return Ac


def is_star(pattern):
    """Every offset has at most one nonzero component (e.g. the 7-point stencil)."""
    return all(int(np.count_nonzero(np.asarray(t))) <= 1 for t in pattern)


def non_galerkin(Ac, cdims, coffs, p, dstar):
    """Reading R-ng for part p of a coarse operator Ac (Section 5, future work):
    every same-part entry v at (I, J) of offset (t, Q), t across d* and Q along
    d* both nonzero, is removed and v/2 is added at (I, I+t), (I, I+Q),
    (I+t, J) and (I+Q, J); the diagonals of I+t and I+Q lose v/2 each, which
    keeps every row sum."""
    A = Ac.tocoo()
    o0, o1 = int(coffs[p]), int(coffs[p + 1])
    nx, ny, nz = cdims[p]
    stride = np.array([1, nx, nx * ny])
    inp = (A.row >= o0) & (A.row < o1) & (A.col >= o0) & (A.col < o1)

    def coord(g):
        loc = g - o0
        return np.stack([loc % nx, (loc // nx) % ny, loc // (nx * ny)], axis=1)

    sel = np.nonzero(inp)[0]
    off = coord(A.col[sel]) - coord(A.row[sel])
    q = off[:, dstar]
    t = off.copy()
    t[:, dstar] = 0
    move = sel[(q != 0) & np.any(t != 0, axis=1)]
    qm = q[(q != 0) & np.any(t != 0, axis=1)]
    keep = np.ones(A.nnz, dtype=bool)
    keep[move] = False
    I, J, v = A.row[move], A.col[move], A.data[move]
    K1 = J - qm * stride[dstar]      # I + t
    K2 = I + qm * stride[dstar]      # I + Q
    for K in (K1, K2):
        assert np.all((K >= o0) & (K < o1))
    h = 0.5 * v
    rows = np.concatenate([A.row[keep], I, I, K1, K2, K1, K2])
    cols = np.concatenate([A.col[keep], K1, K2, J, J, K1, K2])
    vals = np.concatenate([A.data[keep], h, h, h, h, -h, -h])
    out = sp.coo_matrix((vals, (rows, cols)), shape=Ac.shape).tocsr()
    out.sort_indices()
    return out


def _pattern_of(P):
    Q = P.copy()
    Q.data = np.ones_like(Q.data)
    return Q


@dataclass
class Hierarchy:
    ndim: int
    levels: list
    faces: np.ndarray
    W0: np.ndarray
    cd: np.ndarray
    coarse: str = "sweep"
    relax: str = "jacobi"
    l1_factor: float = 1.5
    skip: bool = False

    @property
    def nlevels(self):
        return len(self.levels)


def setup(A0, dims, faces, pattern0, ndim, ustruct0=None, omega=0.0, max_levels=64,
          min_coarse_size=0, coarse="sweep", relax="jacobi", skip=False, pb="one", hybrid_level=0,
          coarse_op="galerkin"):
    """Full SSAMG setup.  ``pattern0[p]`` is the input stencil of part p.

    ``coarse_op="nongalerkin"``: parts with star stencils get the non-Galerkin
    coarse operator of reading R-ng (the rest stay Galerkin).

    ``hybrid_level`` = k > 0: the hybrid scheme of Section 3.5 - SSAMG builds
    levels 0 .. k-1 and the problem left at level k is solved exactly (here by
    a dense direct solve, standing in for the unstructured solver the paper
    switches to), i.e. the hierarchy ends at level k with coarse = "direct".

    ``ustruct0``: 0/1 structure of the input couplings (defaults to A0's
    cross-part entries).
    """
    if hybrid_level > 0:
        max_levels = min(max_levels, hybrid_level + 1)
        coarse = "direct"
    offsets = _offsets(dims)
    part = cell_coords(dims, offsets)[0]
    if ustruct0 is None:
        Uc = A0.tocoo()
        m = part[Uc.row] != part[Uc.col]
        ustruct0 = sp.csr_matrix((np.ones(int(m.sum())), (Uc.row[m], Uc.col[m])), shape=A0.shape)
    lev0 = Level(list(dims), offsets, A0.tocsr(), [np.asarray(q) for q in pattern0],
                 ustruct0.tocsr())
    cd = direction_sums(lev0, ndim)
    W0 = grid_spacing(cd, ndim)
    all_dims, all_dstar, all_omega = coarsen(W0, dims, ndim, max_levels, min_coarse_size)
    levels = [lev0]
    for l in range(len(all_dims)):
        lev = levels[l]
        lev.dstar = list(all_dstar[l])
        lev.omega = (np.full(len(dims), omega) if omega > 0 else all_omega[l])
        if l == len(all_dims) - 1:
            break
        cdims = all_dims[l + 1]
        coffs = _offsets(cdims)
        lev.wm, lev.wp = [], []
        for p in range(len(dims)):
            if lev.dstar[p] >= 0:
                wm, wp = interpolation_weights(lev, p, lev.dstar[p], faces, pb)
            else:
                wm, wp = np.zeros(0), np.zeros(0)
            lev.wm.append(wm)
            lev.wp.append(wp)
        lev.P = interpolation_matrix(lev, cdims, coffs)
        Ac = galerkin(lev.A, lev.P)
        pats = [coarse_pattern(lev.pattern[p], lev.dstar[p]) for p in range(len(dims))]
        if coarse_op == "nongalerkin":
            for p in range(len(dims)):
                if lev.dstar[p] >= 0 and is_star(lev.pattern[p]):
                    Ac = non_galerkin(Ac, cdims, coffs, p, lev.dstar[p])
                    pats[p] = np.asarray([t for t in pats[p] if np.count_nonzero(t) <= 1],
                                         dtype=np.int32)
        elif coarse_op != "galerkin":
            raise ValueError(f"unknown coarse_op {coarse_op!r}")
        Pb = _pattern_of(lev.P)
        ust = (Pb.T @ lev.ustruct @ Pb).tocsr()
        ust.data[:] = 1.0
        ust.sort_indices()
        levels.append(Level(list(cdims), coffs, Ac, pats, ust))
    h = Hierarchy(ndim, levels, np.asarray(faces), W0, cd, coarse, relax,
                  omega if (relax == "l1" and omega > 0) else 1.5, skip)
    for l, lev in enumerate(levels):
        lev._cache["relax"] = (relax, h.l1_factor)
        lev._cache["skip"] = skip_mask(levels, l, ndim) if skip else np.zeros(len(dims), dtype=bool)
    return h


def skip_mask(levels, l, ndim):
    """Parts that do not relax at level l under the skip option (reading R-skip)."""
    ds = levels[l].dstar
    if l < ndim:
        return np.zeros(len(ds), dtype=bool)
    prev = levels[l - ndim].dstar
    return np.array([ds[p] >= 0 and ds[p] == prev[p] for p in range(len(ds))], dtype=bool)


# ---------------------------------------------------------------------------
# level data in the layouts the solver library exposes


def stencil_values(level, p):
    """[nent][ncell] coefficients of part p in the order of level.pattern[p]."""
    r, c, v, part, same, s = _entries(level)
    sel = same & (part[r] == p)
    pat = level.pattern[p]
    key = {tuple(int(a) for a in t): e for e, t in enumerate(pat)}
    nx, ny, nz = level.dims[p]
    out = np.zeros((len(pat), nx * ny * nz))
    for rr, vv, ss in zip(r[sel] - level.offsets[p], v[sel], s[sel]):
        e = key.get(tuple(int(a) for a in ss))
        if e is None:
            raise AssertionError(f"entry {tuple(ss)} outside the symbolic pattern")
        out[e, rr] += vv
    return out


def stencil_values_fast(level, p):
    """Vectorised twin of stencil_values (same result, for large levels)."""
    r, c, v, part, same, s = _entries(level)
    sel = same & (part[r] == p)
    pat = level.pattern[p]
    code = (pat[:, 0] + 1) + 3 * (pat[:, 1] + 1) + 9 * (pat[:, 2] + 1)
    lut = -np.ones(27, dtype=np.int64)
    lut[code] = np.arange(len(pat))
    ss = s[sel]
    e = lut[(ss[:, 0] + 1) + 3 * (ss[:, 1] + 1) + 9 * (ss[:, 2] + 1)]
    if np.any(e < 0):
        raise AssertionError("entry outside the symbolic pattern")
    nx, ny, nz = level.dims[p]
    out = np.zeros((len(pat), nx * ny * nz))
    np.add.at(out, (e, r[sel] - level.offsets[p]), v[sel])
    return out


def coupling_csr(level):
    """Cross-part couplings on the symbolic structure: (rowptr, col, val)."""
    st = level.ustruct.tocsr()
    st.sort_indices()
    A = level.A.tocsr()
    coo_r = np.repeat(np.arange(st.shape[0]), np.diff(st.indptr))
    vals = np.asarray(A[coo_r, st.indices]).reshape(-1) if st.nnz else np.zeros(0)
    return st.indptr.astype(np.int64), st.indices.astype(np.int64), vals


# ---------------------------------------------------------------------------
# Section 3.4 relaxation, V(1,1) cycle, PCG


def _cell_weights(level):
    """Per-cell factor of the smoother x <- x + w (b - A x) (eq:relax0):
    weighted Jacobi w = omega_p / a_ii (eq:relax1), or weighted L1-Jacobi
    w = factor / sum_j |a_ij| over the whole row of A = S + U (Section 3.4)."""
    if "wd" not in level._cache:
        relax, factor = level._cache.get("relax", ("jacobi", 1.5))
        if relax == "l1":
            level._cache["wd"] = factor / np.asarray(abs(level.A).sum(axis=1)).ravel()
        else:
            part = np.repeat(np.arange(len(level.dims)), np.diff(level.offsets))
            level._cache["wd"] = level.omega[part] / level.A.diagonal()
        skip = level._cache.get("skip")
        if skip is not None and skip.any():
            part = np.repeat(np.arange(len(level.dims)), np.diff(level.offsets))
            level._cache["wd"] = np.where(skip[part], 0.0, level._cache["wd"])
    return level._cache["wd"]


def vcycle(h, b):
    """One V(1,1) cycle, zero initial guess: weighted Jacobi pre/post sweeps,
    restriction by P^T, interpolation by P; one sweep (or a direct solve) on
    the coarsest level."""
    L = h.nlevels

    def rec(l, bl):
        lev = h.levels[l]
        wd = _cell_weights(lev)
        if l == L - 1:
            if h.coarse == "direct":
                # dense Cholesky factor of the coarsest operator, formed once
                if "chol" not in lev._cache:
                    lev._cache["chol"] = sla.cho_factor(lev.A.toarray())
                return sla.cho_solve(lev._cache["chol"], bl)
            return wd * bl
        x = wd * bl
        r = bl - lev.A @ x
        xc = rec(l + 1, lev.P.T @ r)
        x = x + lev.P @ xc
        x = x + wd * (bl - lev.A @ x)
        return x

    return rec(0, np.asarray(b, dtype=np.float64))


@dataclass
class PCGResult:
    x: np.ndarray
    iters: int
    relres: float
    true_relres: float
    converged: bool
    history: list


def pcg(A, b, precond, tol=1e-8, max_iter=100, flexible=False):
    """Preconditioned CG, x0 = 0; stops when ||r||_2 < tol ||b||_2.
    One iteration = one product with A.  ``flexible`` uses the Polak-Ribiere
    beta = z_new^T (r_new - r_old) / (r_old^T z_old)."""
    b = np.asarray(b, dtype=np.float64)
    x = np.zeros_like(b)
    r = b.copy()
    bn = math.sqrt(float(b @ b))
    hist = [1.0 if bn > 0 else 0.0]
    if bn == 0.0:
        return PCGResult(x, 0, 0.0, 0.0, True, hist)
    z = precond(r)
    p = z.copy()
    rz = float(r @ z)
    it = 0
    conv = False
    while it < max_iter:
        q = A @ p
        pq = float(p @ q)
        if not pq > 0:
            raise FloatingPointError("PCG breakdown: p^T A p <= 0")
        alpha = rz / pq
        x += alpha * p
        r_old = r
        r = r - alpha * q
        it += 1
        rn = math.sqrt(float(r @ r))
        hist.append(rn / bn)
        if rn < tol * bn:
            conv = True
            break
        z = precond(r)
        if flexible:
            beta = float(z @ (r - r_old)) / rz
            rz = float(r @ z)
        else:
            rz_new = float(r @ z)
            beta = rz_new / rz
            rz = rz_new
        p = z + beta * p
    tr = float(np.linalg.norm(b - A @ x)) / bn
    return PCGResult(x, it, hist[-1], tr, conv, hist)


def solve(h, b, tol=1e-8, max_iter=100, flexible=False):
    return pcg(h.levels[0].A, b, lambda r: vcycle(h, r), tol, max_iter, flexible)
