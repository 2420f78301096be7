"""Seeded synthetic inputs for the SSAMG solver and its CPU oracle.

This module is the only code that the HIP path's tests/bench and the oracle
share.  It lays out geometry and draws random numbers; it holds none of the
solver's arithmetic (no coarsening, interpolation, Galerkin products, smoothing
or Krylov steps) and no finite-volume assembly: each side turns the raw inputs
drawn here into a matrix with its own code.

Unknown ordering everywhere: part-major, and within a part lexicographic with x
fastest (index = i + nx*(j + ny*k)).  Every part is one box with lower corner 0
in its own index space; ``origins`` places the boxes in a shared global index
space so that neighbours across parts can be found.

Workloads (the paper's test problems are finite-difference Poisson systems on
unions of m^3 cubes, Section 4 and the seven-point stencil eq:stencilA; these
are synthetic stand-ins of the same shape):

  c1  one 16^3 part, isotropic 7-point (diag 6, off-diag -1), fixed omega 2/3
  c2  four 64^3 parts along x, 7-point, per-part anisotropy 100:1:1 with the
      strong direction x, y, z, x
  c3  eight 128^3 parts in a 2x2x2 block, 27-point, kappa log-normal (sigma 2)
      times 1e4 on a checkerboard of parts
  c4  two 96^3 parts along x, 7-point, anisotropy 10:1:1, 32 right-hand sides
  c5  three 64^3 parts along x, 7-point, kappa = exp(N(0,1)); adjoint problem

Random streams: ``numpy.random.default_rng(1000*c + role)`` with role 0 = b,
1 = kappa, 2 = perturbed kappa, 3 = cell sample.  ``m`` may be reduced for
tests; the recipe is otherwise unchanged.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Optional

import numpy as np

# face order used by every interface: -x, +x, -y, +y, -z, +z
FACES = ((0, -1), (0, +1), (1, -1), (1, +1), (2, -1), (2, +1))
FACE_PHYSICAL = 0
FACE_PART = 1


@dataclass
class Geometry:
    """One box per part, lower corner 0, placed at ``origins`` in a global index space."""
    ndim: int
    dims: list            # [(nx, ny, nz)] per part
    origins: list         # [(ox, oy, oz)] per part

    @property
    def nparts(self) -> int:
        return len(self.dims)

    def ncells(self, p: int) -> int:
        nx, ny, nz = self.dims[p]
        return nx * ny * nz

    @property
    def offsets(self) -> np.ndarray:
        """Cell offset of each part in the global vector (length nparts+1)."""
        off = [0]
        for p in range(self.nparts):
            off.append(off[-1] + self.ncells(p))
        return np.asarray(off, dtype=np.int64)

    @property
    def n(self) -> int:
        return int(self.offsets[-1])

    def part_at(self, g) -> int:
        """Part containing global coordinate g, or -1 (outside every part)."""
        for p in range(self.nparts):
            o, d = self.origins[p], self.dims[p]
            if all(o[a] <= g[a] < o[a] + d[a] for a in range(3)):
                return p
        return -1

    def face_kinds(self) -> np.ndarray:
        """[nparts][6] face kinds: PART if any cell just across the face lies in
        another part, else PHYSICAL.  Pure geometry."""
        kinds = np.zeros((self.nparts, 6), dtype=np.int32)
        for p in range(self.nparts):
            o, d = self.origins[p], self.dims[p]
            for f, (ax, sgn) in enumerate(FACES):
                if ax >= self.ndim:
                    continue
                # probe every cell of the face layer just outside the box
                rng = [range(o[a], o[a] + d[a]) for a in range(3)]
                rng[ax] = [o[ax] - 1] if sgn < 0 else [o[ax] + d[ax]]
                hit = False
                for gz in rng[2]:
                    for gy in rng[1]:
                        for gx in rng[0]:
                            q = self.part_at((gx, gy, gz))
                            if q >= 0 and q != p:
                                hit = True
                                break
                        if hit:
                            break
                    if hit:
                        break
                kinds[p, f] = FACE_PART if hit else FACE_PHYSICAL
        return kinds


def stencil_offsets(kind: int, ndim: int = 3) -> np.ndarray:
    """Stencil offsets, center first, then the rest in (dz, dy, dx) order.

    kind 7 / 27 in 3D, 5 / 9 in 2D.
    """
    offs = []
    rz = (-1, 0, 1) if ndim == 3 else (0,)
    for dz in rz:
        for dy in (-1, 0, 1):
            for dx in (-1, 0, 1):
                nnz = (dx != 0) + (dy != 0) + (dz != 0)
                if nnz == 0:
                    continue
                if kind in (7, 5) and nnz > 1:
                    continue
                offs.append((dx, dy, dz))
    if kind == 27 or kind == 9 or kind == 7 or kind == 5:
        return np.asarray([(0, 0, 0)] + offs, dtype=np.int32)
    raise ValueError(f"unsupported stencil kind {kind}")


@dataclass
class FVCase:
    """A finite-volume diffusion workload: geometry + kappa + anisotropy + rhs."""
    name: str
    geometry: Geometry
    stencil: int                      # 7 or 27
    kappa: np.ndarray                 # [N] per-cell conductivity, global order
    aniso: np.ndarray                 # [nparts][3] directional factors
    b: np.ndarray                     # [N] or [nrhs][N]
    omega: float = 0.0                # <= 0: per-part omega from the grid-spacing metric
    relax: str = "jacobi"             # "jacobi" (weighted, omega) or "l1" (weighted L1, 3/2)
    tol: float = 1e-8
    max_iter: int = 100
    extra: dict = field(default_factory=dict)

    @property
    def nrhs(self) -> int:
        return 1 if self.b.ndim == 1 else self.b.shape[0]


def _along_x(nparts: int, m: int):
    dims = [(m, m, m)] * nparts
    origins = [(m * p, 0, 0) for p in range(nparts)]
    return Geometry(3, list(dims), origins)


def c1(m: int = 16) -> FVCase:
    g = Geometry(3, [(m, m, m)], [(0, 0, 0)])
    rng = np.random.default_rng(1000 * 1 + 0)
    b = rng.uniform(-1.0, 1.0, g.n)
    return FVCase("c1", g, 7, np.ones(g.n), np.ones((1, 3)), b, omega=2.0 / 3.0)


def c2(m: int = 64) -> FVCase:
    g = _along_x(4, m)
    aniso = np.array([[100.0, 1, 1], [1, 100.0, 1], [1, 1, 100.0], [100.0, 1, 1]])
    rng = np.random.default_rng(1000 * 2 + 0)
    b = rng.uniform(-1.0, 1.0, g.n)
    return FVCase("c2", g, 7, np.ones(g.n), aniso, b)


def c3(m: int = 128) -> FVCase:
    dims, origins, jump = [], [], []
    for pz in range(2):
        for py in range(2):
            for px in range(2):
                dims.append((m, m, m))
                origins.append((m * px, m * py, m * pz))
                jump.append(1e4 if (px + py + pz) % 2 == 1 else 1.0)
    g = Geometry(3, dims, origins)
    rb = np.random.default_rng(1000 * 3 + 0)
    b = rb.uniform(-1.0, 1.0, g.n)
    rk = np.random.default_rng(1000 * 3 + 1)
    z = rk.standard_normal(g.n)
    kappa = np.exp(2.0 * z)
    off = g.offsets
    for p in range(g.nparts):
        kappa[off[p]:off[p + 1]] *= jump[p]
    # weighted Jacobi with the metric's omega_p stalls on this strongly
    # heterogeneous 27-point problem; the paper's own baseline smoother
    # (weighted L1-Jacobi, factor 3/2) is used
    return FVCase("c3", g, 27, kappa, np.ones((8, 3)), b, relax="l1")


def c4(m: int = 96, nrhs: int = 32) -> FVCase:
    g = _along_x(2, m)
    rng = np.random.default_rng(1000 * 4 + 0)
    b = rng.uniform(-1.0, 1.0, (nrhs, g.n))
    aniso = np.array([[10.0, 1, 1], [10.0, 1, 1]])
    return FVCase("c4", g, 7, np.ones(g.n), aniso, b)


def c5(m: int = 64, nsample: int = 50) -> FVCase:
    g = _along_x(3, m)
    rb = np.random.default_rng(1000 * 5 + 0)
    b = rb.uniform(-1.0, 1.0, g.n)
    rk = np.random.default_rng(1000 * 5 + 1)
    kappa = np.exp(rk.standard_normal(g.n))
    rp = np.random.default_rng(1000 * 5 + 2)
    kappa_t = kappa * np.exp(0.1 * rp.standard_normal(g.n))
    rs = np.random.default_rng(1000 * 5 + 3)
    sample = rs.choice(g.n, size=min(nsample, g.n), replace=False)
    case = FVCase("c5", g, 7, kappa, np.ones((3, 3)), b)
    case.extra = {"kappa_target": kappa_t, "sample": np.sort(sample), "fd_h": 1e-6,
                  "fd_tol": 1e-13}
    return case


CONFIGS = {"c1": c1, "c2": c2, "c3": c3, "c4": c4, "c5": c5}


@dataclass
class RawCase:
    """A semi-structured matrix given directly as stencil arrays + inter-part COO.

    ``coeffs[p]`` is [nent][nz][ny][nx] (x fastest) for the offsets ``stencils[p]``;
    ``urow/ucol/uval`` are global ids and values of the inter-part couplings.
    """
    name: str
    geometry: Geometry
    faces: np.ndarray                 # [nparts][6]
    stencils: list                    # [nent][3] per part
    coeffs: list                      # [nent][nz][ny][nx] per part
    urow: np.ndarray
    ucol: np.ndarray
    uval: np.ndarray
    b: np.ndarray


def random_link_case(seed: int, geometry: Geometry, kind: int = 7,
                     junk_outside: bool = False, diag_margin: float = 0.05) -> RawCase:
    """Random symmetric M-matrix on ``geometry``: every pair of neighbouring cells
    (same part or across parts) gets a conductance t ~ U[0.5, 1.5] scaled by a
    per-link-direction factor, off-diagonals are -t, and each diagonal is the sum
    of its row's conductances plus a small random margin (Dirichlet-like).
    With ``junk_outside`` the stencil entries that point out of their box are
    filled with random garbage, which any consumer must discard.
    """
    rng = np.random.default_rng(seed)
    g = geometry
    offs = stencil_offsets(kind, g.ndim)
    nent = len(offs)
    off = g.offsets
    coeffs = [np.zeros((nent,) + tuple(reversed(g.dims[p]))) for p in range(g.nparts)]
    # per-direction anisotropy per part, random
    an = rng.uniform(0.2, 5.0, (g.nparts, 3))
    diag = np.zeros(g.n)
    rows, cols, vals = [], [], []
    # global lookup table for neighbours
    lo = np.min(np.asarray(g.origins), axis=0) - 1
    hi = np.max(np.asarray(g.origins) + np.asarray(g.dims), axis=0) + 1
    shape = tuple(int(h - l) for h, l in zip(hi, lo))
    gid = -np.ones(shape[::-1], dtype=np.int64)          # [z][y][x]
    for p in range(g.nparts):
        ox, oy, oz = (np.asarray(g.origins[p]) - lo)
        nx, ny, nz = g.dims[p]
        ids = off[p] + np.arange(nx * ny * nz).reshape(nz, ny, nx)
        gid[oz:oz + nz, oy:oy + ny, ox:ox + nx] = ids
    # each unordered link drawn once: iterate over "positive" half of offsets
    half = [tuple(o) for o in offs[1:] if (o[2], o[1], o[0]) > (0, 0, 0)]
    for p in range(g.nparts):
        ox, oy, oz = (np.asarray(g.origins[p]) - lo)
        nx, ny, nz = g.dims[p]
        ids = gid[oz:oz + nz, oy:oy + ny, ox:ox + nx]
        for s in half:
            dx, dy, dz = s
            nb = gid[oz + dz:oz + dz + nz, oy + dy:oy + dy + ny, ox + dx:ox + dx + nx]
            w = np.mean([an[p, a] for a in range(3) if s[a] != 0])
            t = rng.uniform(0.5, 1.5, ids.shape) * w / (abs(dx) + abs(dy) + abs(dz))
            mask = nb >= 0
            i, j, tv = ids[mask], nb[mask], t[mask]
            pi = np.searchsorted(off, i, side="right") - 1
            pj = np.searchsorted(off, j, side="right") - 1
            same = pi == pj
            np.add.at(diag, i, tv)
            np.add.at(diag, j, tv)
            # same-part: write stencil entries of both ends
            ks = int(np.nonzero((offs == np.asarray(s)).all(axis=1))[0][0])
            km = int(np.nonzero((offs == -np.asarray(s)).all(axis=1))[0][0])
            for q in range(g.nparts):
                sel = same & (pi == q)
                if not sel.any():
                    continue
                li = i[sel] - off[q]
                lj = j[sel] - off[q]
                coeffs[q][ks].reshape(-1)[li] = -tv[sel]
                coeffs[q][km].reshape(-1)[lj] = -tv[sel]
            cross = ~same
            rows += [i[cross], j[cross]]
            cols += [j[cross], i[cross]]
            vals += [-tv[cross], -tv[cross]]
    diag += rng.uniform(0.0, diag_margin, g.n) * diag + 1e-3
    for p in range(g.nparts):
        coeffs[p][0].reshape(-1)[:] = diag[off[p]:off[p + 1]]
    if junk_outside:
        for p in range(g.nparts):
            nx, ny, nz = g.dims[p]
            k, j, i = np.meshgrid(np.arange(nz), np.arange(ny), np.arange(nx), indexing="ij")
            for e, (dx, dy, dz) in enumerate(offs):
                out = ((i + dx < 0) | (i + dx >= nx) | (j + dy < 0) | (j + dy >= ny)
                       | (k + dz < 0) | (k + dz >= nz))
                coeffs[p][e][out] = rng.uniform(-3.0, 3.0, int(out.sum()))
    urow = np.concatenate(rows) if rows else np.zeros(0, np.int64)
    ucol = np.concatenate(cols) if cols else np.zeros(0, np.int64)
    uval = np.concatenate(vals) if vals else np.zeros(0)
    b = np.random.default_rng(seed + 1).uniform(-1.0, 1.0, g.n)
    return RawCase(f"raw{seed}", g, g.face_kinds(), [offs.copy() for _ in range(g.nparts)],
                   coeffs, urow.astype(np.int64), ucol.astype(np.int64), uval, b)


def geometry_along_x(nparts: int, dims) -> Geometry:
    """Parts of (possibly different) sizes laid side by side along x."""
    origins, x = [], 0
    for d in dims:
        origins.append((x, 0, 0))
        x += d[0]
    return Geometry(3 if any(d[2] > 1 for d in dims) else 2, list(dims), origins)


# ---------------------------------------------------------------------------
# parts glued with rotated index spaces, and parts of several boxes
# (the shapes of the paper's test cases 3 and 4, Section 4)


@dataclass
class TopoCase:
    """A semi-structured problem given as per-part stencils plus topology: the
    boxes of each part (None: the whole box; cells in no box are ghost
    unknowns) and glued faces (neighbour maps), with user couplings U.

    ``neighbors[p][f]`` is None or {"part", "at", "nbr_at", "map", "dir"}: the
    point ``at`` just across face f of part p has index ``nbr_at`` in the
    neighbour part, and part p's axis d maps to the neighbour's axis map[d]
    with direction dir[d].
    """
    name: str
    dims: list
    stencils: list                    # [nent][3] per part
    coeffs: list                      # [nent][nz][ny][nx] per part
    boxes: list                       # per part: None or [(lo, hi), ...] inclusive
    neighbors: list                   # per part: 6 entries, None or a dict
    urow: np.ndarray
    ucol: np.ndarray
    uval: np.ndarray
    b: np.ndarray
    ndim: int = 3
    faces: Optional[list] = None      # [nparts][6] face kinds; None: glued faces are part faces

    @property
    def n(self) -> int:
        return int(sum(a * b * c for a, b, c in self.dims))

    def face_kinds(self):
        if self.faces is not None:
            return np.asarray(self.faces)
        return np.array([[0 if nb is None else 1 for nb in self.neighbors[p]] for p in range(len(self.dims))])


def _laplacian_coeffs(dims, offs, off_value, rng=None, spread=0.0):
    """Constant 7-point coefficients (off-diagonal off_value, diagonal the sum of
    their magnitudes) on every cell of a box, optionally perturbed per link
    symmetrically would need a global view, so only the diagonal is perturbed
    (a positive random margin keeps the matrix an M-matrix)."""
    nx, ny, nz = dims
    co = np.zeros((len(offs), nz, ny, nx))
    for e, s in enumerate(offs):
        if tuple(s) != (0, 0, 0):
            co[e] = off_value
    co[0] = -off_value * (len(offs) - 1)
    if rng is not None and spread > 0:
        co[0] += rng.uniform(0.0, spread, (nz, ny, nx))
    return co


def tc3_junction(m: int = 16, seed: int = 6000) -> TopoCase:
    """Three m^3 parts around a common edge along z (a three-point intersection
    in the xy-plane): the +x face of part p is glued to the +y face of part
    p+1 (mod 3) with the index space rotated by a quarter turn, so an east
    coefficient of one part couples to a north coefficient of the next.
    Isotropic 7-point Laplacian (diagonal 6, off-diagonal -1), zero Dirichlet
    on every other face, right-hand side U[-1, 1]."""
    offs = stencil_offsets(7)
    dims = [(m, m, m)] * 3
    neighbors = [[None] * 6 for _ in range(3)]
    for p in range(3):
        q = (p + 1) % 3
        # across p's +x face: (m + a, j, k) -> (j, m - 1 - a, k) in part q
        neighbors[p][1] = {"part": q, "at": (m, 0, 0), "nbr_at": (0, m - 1, 0),
                           "map": (1, 0, 2), "dir": (-1, 1, 1)}
        # across q's +y face: (i, m + a, k) -> (m - 1 - a, i, k) in part p
        neighbors[q][3] = {"part": p, "at": (0, m, 0), "nbr_at": (m - 1, 0, 0),
                           "map": (1, 0, 2), "dir": (1, -1, 1)}
    coeffs = [_laplacian_coeffs(d, offs, -1.0) for d in dims]
    rng = np.random.default_rng(seed)
    n = 3 * m ** 3
    return TopoCase("tc3", dims, [offs] * 3, coeffs, [None] * 3, neighbors,
                    np.zeros(0, dtype=np.int64), np.zeros(0, dtype=np.int64), np.zeros(0),
                    rng.uniform(-1, 1, n))


def tc4_samr(m: int = 16, seed: int = 7000, junk: bool = True) -> TopoCase:
    """One level of refinement: part 0 is the coarse m^3 grid, part 1 an m^3
    patch refined by two covering the central (m/2)^3 coarse cells, which are
    ghost unknowns of part 0 (part 0 is the union of the six slabs around
    them).  7-point finite-volume couplings scaled by the fine spacing: -1
    between fine cells, -2 between coarse cells, -2/3 between a fine cell and
    the coarse cell across the patch face (both ways, in U); diagonals are the
    sums of a row's couplings, a zero-Dirichlet ghost outside the domain
    counting as a coarse link.  With ``junk`` the ghost cells' given
    coefficients are random and must be replaced by an identity row."""
    if m % 4:
        raise ValueError("m must be a multiple of 4")
    offs = stencil_offsets(7)
    a, b = m // 4, 3 * m // 4            # hole [a, b)^3 in coarse indices
    rng = np.random.default_rng(seed)
    dims = [(m, m, m), (m, m, m)]
    # part 0: the six slabs around the hole
    boxes0 = [((0, 0, 0), (m - 1, m - 1, a - 1)), ((0, 0, b), (m - 1, m - 1, m - 1)),
              ((0, 0, a), (m - 1, a - 1, b - 1)), ((0, b, a), (m - 1, m - 1, b - 1)),
              ((0, a, a), (a - 1, b - 1, b - 1)), ((b, a, a), (m - 1, b - 1, b - 1))]

    def in_hole(i, j, k):
        return a <= i < b and a <= j < b and a <= k < b

    co0 = np.zeros((7, m, m, m))
    co1 = np.zeros((7, m, m, m))
    urow, ucol, uval = [], [], []
    off0, off1 = 0, m ** 3
    for k in range(m):
        for j in range(m):
            for i in range(m):
                # coarse cell
                if in_hole(i, j, k):
                    co0[:, k, j, i] = rng.uniform(-3, 3, 7) if junk else 0.0
                else:
                    diag = 0.0
                    for e, (dx, dy, dz) in enumerate(offs[1:], start=1):
                        t = (i + dx, j + dy, k + dz)
                        if not all(0 <= t[d] < m for d in range(3)):
                            diag += 2.0                      # Dirichlet ghost
                        elif in_hole(*t):
                            # the face of the patch: four fine cells across it
                            ax = [d for d in range(3) if (dx, dy, dz)[d] != 0][0]
                            f0 = [2 * (v - a) for v in (i, j, k)]
                            f0[ax] = 0 if (dx, dy, dz)[ax] > 0 else m - 1
                            others = [d for d in range(3) if d != ax]
                            for u in range(2):
                                for v in range(2):
                                    f = list(f0)
                                    f[others[0]] += u
                                    f[others[1]] += v
                                    fid = off1 + f[0] + m * (f[1] + m * f[2])
                                    cid = off0 + i + m * (j + m * k)
                                    urow += [cid, fid]
                                    ucol += [fid, cid]
                                    uval += [-2.0 / 3.0, -2.0 / 3.0]
                                    diag += 2.0 / 3.0
                        else:
                            co0[e, k, j, i] = -2.0
                            diag += 2.0
                    co0[0, k, j, i] = diag
                # fine cell (i, j, k) of the patch
                diag = 0.0
                for e, (dx, dy, dz) in enumerate(offs[1:], start=1):
                    t = (i + dx, j + dy, k + dz)
                    if all(0 <= t[d] < m for d in range(3)):
                        co1[e, k, j, i] = -1.0
                        diag += 1.0
                    else:
                        diag += 2.0 / 3.0                # the coupling to the coarse cell across
                co1[0, k, j, i] = diag
    n = 2 * m ** 3
    # the patch's faces all border the coarse part (couplings in U)
    return TopoCase("tc4", dims, [offs, offs], [co0, co1], [boxes0, None],
                    [[None] * 6, [None] * 6], np.asarray(urow, dtype=np.int64),
                    np.asarray(ucol, dtype=np.int64), np.asarray(uval), rng.uniform(-1, 1, n),
                    faces=[[0] * 6, [1] * 6])
