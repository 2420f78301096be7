"""Oracle: assembly of the semi-structured matrix A = S + U (test infrastructure only).

Section 2 of the paper: a matrix on an SStruct grid is the sum of a structured
part S (per-part stencil coefficients, variable per cell) and an unstructured
part U (a sparse matrix holding the couplings between parts).  Cells are
numbered part-major, lexicographic with x fastest inside a part.

Dirichlet elimination (a reading; the paper's workloads are zero-Dirichlet
finite-difference problems, Section 4): a stencil coefficient whose neighbour
lies outside its part's box is dropped.  Couplings across parts live in U only.

The finite-volume rule used to generate the synthetic workloads (kappa -> A)
is a property of the inputs, not of SSAMG; it and its adjoint gradient are
implemented here from their definitions:
  t_ij = g_s * H(a_{p(i),s} kappa_i, a_{p(j),s} kappa_j),  H(x,y) = 2xy/(x+y),
  g_s = 1 / 2^(nnz(s)-1) (faces 1, edges 1/2, corners 1/4), a_{p,s} the mean of
  the part's directional factors over the nonzero components of s; a neighbour
  outside every part is a ghost with kappa_j = kappa_i (contributes to the
  diagonal only); A_ii = sum of t over the cell's links, A_ij = -t_ij.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp


def cell_coords(dims, offsets):
    """part[N], i[N], j[N], k[N] for a level with per-part box extents ``dims``."""
    parts, ii, jj, kk = [], [], [], []
    for p, (nx, ny, nz) in enumerate(dims):
        n = nx * ny * nz
        idx = np.arange(n)
        parts.append(np.full(n, p, dtype=np.int64))
        ii.append(idx % nx)
        jj.append((idx // nx) % ny)
        kk.append(idx // (nx * ny))
    return (np.concatenate(parts), np.concatenate(ii), np.concatenate(jj),
            np.concatenate(kk))


def assemble_raw(dims, stencils, coeffs, urow, ucol, uval):
    """Global CSR of A = S + U.

    dims[p] = (nx, ny, nz); stencils[p] = [nent][3] offsets; coeffs[p] =
    [nent][nz][ny][nx].  Entries pointing out of the part box are dropped.
    U must hold only inter-part couplings (an assumption of the paper's
    theorem on U_c); duplicates are summed.
    """
    offsets = np.concatenate([[0], np.cumsum([a * b * c for a, b, c in dims])]).astype(np.int64)
    N = int(offsets[-1])
    rows, cols, vals = [], [], []
    for p, (nx, ny, nz) in enumerate(dims):
        k, j, i = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
        gid = offsets[p] + (i + nx * (j + ny * k))
        for e, (dx, dy, dz) in enumerate(np.asarray(stencils[p])):
            ni, nj, nk = i + dx, j + dy, k + dz
            inb = (ni >= 0) & (ni < nx) & (nj >= 0) & (nj < ny) & (nk >= 0) & (nk < nz)
            rows.append(gid[inb])
            cols.append(offsets[p] + (ni + nx * (nj + ny * nk))[inb])
            vals.append(np.asarray(coeffs[p][e], dtype=np.float64)[inb])
    urow = np.asarray(urow, dtype=np.int64)
    ucol = np.asarray(ucol, dtype=np.int64)
    if urow.size:
        pr = np.searchsorted(offsets, urow, side="right") - 1
        pc = np.searchsorted(offsets, ucol, side="right") - 1
        if np.any(pr == pc):
            raise ValueError("U holds a coupling inside one part")
    rows.append(urow)
    cols.append(ucol)
    vals.append(np.asarray(uval, dtype=np.float64))
    A = sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(N, N))
    A.sum_duplicates()
    A.sort_indices()
    return A, offsets


def u_structure(urow, ucol, N):
    """Canonical structure of the input couplings (unique (row, col) pairs) as a
    0/1 CSR pattern; structural zeros given by the caller are kept."""
    P = sp.csr_matrix((np.ones(len(urow)), (np.asarray(urow), np.asarray(ucol))), shape=(N, N))
    P.sum_duplicates()
    P.data[:] = 1.0
    P.sort_indices()
    return P


# ---------------------------------------------------------------------------
# finite-volume workloads


def _link_factor(aniso_p, s):
    """a_{p,s}: mean of the part's directional factors over the nonzero components."""
    nz = [a for a in range(3) if s[a] != 0]
    return np.mean([aniso_p[a] for a in nz])


def _geom_weight(s):
    return 1.0 / (2.0 ** (sum(1 for a in s if a != 0) - 1))


def _global_table(geometry):
    """Dense global id table over the bounding box of all parts (+1 layer), -1 = none."""
    org = np.asarray(geometry.origins)
    dm = np.asarray(geometry.dims)
    lo = org.min(axis=0) - 1
    hi = (org + dm).max(axis=0) + 1
    shape = tuple(int(v) for v in (hi - lo))
    gid = -np.ones(shape[::-1], dtype=np.int64)
    offs = geometry.offsets
    for p in range(geometry.nparts):
        ox, oy, oz = org[p] - lo
        nx, ny, nz = dm[p]
        gid[oz:oz + nz, oy:oy + ny, ox:ox + nx] = offs[p] + np.arange(nx * ny * nz).reshape(nz, ny, nx)
    return gid, lo


def fv_links(geometry, stencil, kappa, aniso):
    """All directed links (i, j_or_-1, s, t_ij, dt_ij/dkappa_i) of the FV rule.

    Yields one record array per stencil offset s != 0.  j = -1 marks a ghost
    (Dirichlet) neighbour.
    """
    from workloads import stencil_offsets
    offs = stencil_offsets(stencil, geometry.ndim)[1:]
    gid, lo = _global_table(geometry)
    org = np.asarray(geometry.origins)
    out = []
    for s in offs:
        dx, dy, dz = (int(v) for v in s)
        g = _geom_weight(s)
        for p in range(geometry.nparts):
            nx, ny, nz = geometry.dims[p]
            ox, oy, oz = org[p] - lo
            ids = gid[oz:oz + nz, oy:oy + ny, ox:ox + nx].reshape(-1)
            nb = gid[oz + dz:oz + dz + nz, oy + dy:oy + dy + ny, ox + dx:ox + dx + nx].reshape(-1)
            ai = _link_factor(aniso[p], s)
            xi = ai * kappa[ids]
            has = nb >= 0
            # neighbour's part factor
            aj = np.empty_like(xi)
            pj = np.searchsorted(geometry.offsets, np.where(has, nb, 0), side="right") - 1
            for q in range(geometry.nparts):
                aj[pj == q] = _link_factor(aniso[q], s)
            xj = np.where(has, aj * kappa[np.where(has, nb, 0)], xi)
            t = g * 2.0 * xi * xj / (xi + xj)
            dt = g * ai * 2.0 * xj * xj / (xi + xj) ** 2
            # ghost: t = g * a_i kappa_i, dt/dkappa_i = g * a_i
            dt = np.where(has, dt, g * ai)
            out.append((ids, np.where(has, nb, -1), s, t, dt))
    return out


def assemble_fv(geometry, stencil, kappa, aniso):
    """Global CSR of the FV operator; returns (A, offsets)."""
    N = geometry.n
    diag = np.zeros(N)
    rows, cols, vals = [], [], []
    for ids, nb, s, t, dt in fv_links(geometry, stencil, kappa, aniso):
        np.add.at(diag, ids, t)
        has = nb >= 0
        rows.append(ids[has])
        cols.append(nb[has])
        vals.append(-t[has])
    rows.append(np.arange(N))
    cols.append(np.arange(N))
    vals.append(diag)
    A = sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(N, N))
    A.sum_duplicates()
    A.sort_indices()
    return A, geometry.offsets


def fv_gradient(geometry, stencil, kappa, aniso, lam, x):
    """dL/dkappa_c = -lam^T (dA/dkappa_c) x for A = A(kappa) of the FV rule.

    A = sum over links {i,j} of t_ij (e_i - e_j)(e_i - e_j)^T plus, for ghost
    links, t e_i e_i^T.  Each directed record (i, j) carries dt_ij/dkappa_i, so
    summing -dt * (lam_i - lam_j)(x_i - x_j) over the records of cell i gives the
    gradient (both directions of a link are present).
    """
    g = np.zeros(geometry.n)
    for ids, nb, s, t, dt in fv_links(geometry, stencil, kappa, aniso):
        has = nb >= 0
        jj = np.where(has, nb, 0)
        term = np.where(has, (lam[ids] - lam[jj]) * (x[ids] - x[jj]), lam[ids] * x[ids])
        np.add.at(g, ids, -dt * term)
    return g


# ---------------------------------------------------------------------------
# parts of several boxes and glued part faces (Section 2: a part is a set of
# boxes in its own index space; parts may be connected in non-Cartesian ways,
# and adaptive refinement keeps coarse cells under a patch as ghost unknowns)

FACE_ORDER = ((0, -1), (0, +1), (1, -1), (1, +1), (2, -1), (2, +1))


def neighbor_image(nb, x):
    """Index of point x (outside the part, across the glued face) in the
    neighbour part's space: y[map[d]] = nbr_at[map[d]] + dir[d] (x[d] - at[d])."""
    y = [0, 0, 0]
    for d in range(3):
        y[nb["map"][d]] = nb["nbr_at"][nb["map"][d]] + nb["dir"][d] * (x[d] - nb["at"][d])
    return y


def active_mask(dims_p, boxes_p):
    """Cells of the part's bounding box that lie in one of its boxes (all when
    the part has no box list)."""
    nx, ny, nz = dims_p
    if not boxes_p:
        return np.ones(nx * ny * nz, dtype=bool)
    m = np.zeros((nz, ny, nx), dtype=bool)
    for lo, hi in boxes_p:
        m[lo[2]:hi[2] + 1, lo[1]:hi[1] + 1, lo[0]:hi[0] + 1] = True
    return m.reshape(-1)


def assemble_semistructured(dims, stencils, coeffs, urow, ucol, uval, boxes=None, neighbors=None):
    """Global CSR of A = S + U for parts made of boxes and glued faces.

    boxes[p]: list of (lo, hi) inclusive sub-boxes of part p's bounding box
    [0, dims[p]) (None or empty: the whole box).  A cell in none of them is a
    ghost unknown: its row is the identity, and every entry pointing at it is
    dropped.  neighbors[p][f]: None, or a dict {"part", "at", "nbr_at", "map",
    "dir"} gluing face f of part p (order -x, +x, -y, +y, -z, +z) to another
    part.  A stencil entry whose neighbour c + s lies outside the box goes, in
    face order, through the first glued face it crosses whose image is an
    active cell of that face's neighbour, and becomes the coupling
    U(c, image) = a_s(c); otherwise it is dropped (Dirichlet).  Returns (A,
    offsets, faces) with faces[p][f] = 1 on glued faces.
    """
    nparts = len(dims)
    boxes = boxes or [None] * nparts
    neighbors = neighbors or [[None] * 6 for _ in range(nparts)]
    offsets = np.concatenate([[0], np.cumsum([a * b * c for a, b, c in dims])]).astype(np.int64)
    N = int(offsets[-1])
    act = [active_mask(dims[p], boxes[p]) for p in range(nparts)]
    rows, cols, vals = [], [], []
    for p, (nx, ny, nz) in enumerate(dims):
        st = np.asarray(stencils[p])
        co = np.asarray(coeffs[p], dtype=np.float64).reshape(len(st), -1)
        for c in range(nx * ny * nz):
            g = int(offsets[p]) + c
            if not act[p][c]:
                rows.append(g)
                cols.append(g)
                vals.append(1.0)
                continue
            x = (c % nx, (c // nx) % ny, c // (nx * ny))
            for e, s in enumerate(st):
                t = [x[d] + int(s[d]) for d in range(3)]
                if all(0 <= t[d] < dims[p][d] for d in range(3)):
                    tc = t[0] + nx * (t[1] + ny * t[2])
                    if act[p][tc]:
                        rows.append(g)
                        cols.append(int(offsets[p]) + tc)
                        vals.append(co[e][c])
                    continue
                for f, (ax, sg) in enumerate(FACE_ORDER):
                    nb = neighbors[p][f]
                    crossed = t[ax] < 0 if sg < 0 else t[ax] >= dims[p][ax]
                    if nb is None or not crossed:
                        continue
                    q = nb["part"]
                    y = neighbor_image(nb, t)
                    if all(0 <= y[d] < dims[q][d] for d in range(3)):
                        yc = y[0] + dims[q][0] * (y[1] + dims[q][1] * y[2])
                        if act[q][yc]:
                            rows.append(g)
                            cols.append(int(offsets[q]) + yc)
                            vals.append(co[e][c])
                            break
    urow = np.asarray(urow, dtype=np.int64)
    ucol = np.asarray(ucol, dtype=np.int64)
    if urow.size:
        pr = np.searchsorted(offsets, urow, side="right") - 1
        pc = np.searchsorted(offsets, ucol, side="right") - 1
        if np.any(pr == pc):
            raise ValueError("U holds a coupling inside one part")
        for r, c_ in zip(urow, ucol):
            for gg in (r, c_):
                q = int(np.searchsorted(offsets, gg, side="right") - 1)
                if not act[q][gg - offsets[q]]:
                    raise ValueError("U touches a ghost cell")
    A = sp.csr_matrix((np.concatenate([np.asarray(vals, dtype=np.float64), np.asarray(uval, dtype=np.float64)]),
                       (np.concatenate([np.asarray(rows, dtype=np.int64), urow]),
                        np.concatenate([np.asarray(cols, dtype=np.int64), ucol]))), shape=(N, N))
    A.sum_duplicates()
    A.sort_indices()
    faces = np.array([[1 if neighbors[p][f] is not None else 0 for f in range(6)] for p in range(nparts)])
    return A, offsets, faces


def cross_structure(A, offsets):
    """0/1 pattern of A's cross-part entries (the coupling structure U starts with)."""
    C = A.tocoo()
    part = np.searchsorted(offsets, C.row, side="right") - 1
    partc = np.searchsorted(offsets, C.col, side="right") - 1
    m = part != partc
    P = sp.csr_matrix((np.ones(int(m.sum())), (C.row[m], C.col[m])), shape=A.shape)
    P.sum_duplicates()
    P.data[:] = 1.0
    P.sort_indices()
    return P
