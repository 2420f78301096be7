"""Python binding of the SSAMG C ABI.

The ``ssamg_*`` functions mirror include/ssamg.h one to one (argument
marshalling only).  ``Problem`` and ``Solver`` wrap the handles; PyTorch
tensors provide device memory and ``torch.cuda.current_stream()`` the HIP
stream.  Every step of setup and solve runs in the library's HIP kernels.
"""
from __future__ import annotations

import ctypes as C

import numpy as np
import torch

from . import _lib as L
from ._lib import SSAMGError, check, lib  # noqa: F401


def _ptr(t):
    return C.c_void_p(t.data_ptr()) if t is not None else None


def _stream():
    return C.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ints(v):
    a = (C.c_int * len(v))(*[int(x) for x in v])
    return a


# The C ABI takes raw pointers and cannot see buffer sizes: a tensor of the
# wrong dtype, device or length would make the kernels read or write out of
# bounds.  Every device vector is therefore checked here before the call.


def _dev_vec(t, n, name):
    """``t`` must be a contiguous float64 tensor on the HIP device with n elements."""
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name}: expected a torch tensor, got {type(t).__name__}")
    if not t.is_cuda:
        raise TypeError(f"{name}: expected a tensor on the HIP device, got device {t.device}")
    if t.dtype != torch.float64:
        raise TypeError(f"{name}: expected float64, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name}: the tensor must be contiguous")
    if t.numel() != n:
        raise ValueError(f"{name}: expected {n} elements, got {t.numel()}")
    return t


def _host_f64(a, n, name):
    """A host float64 array of exactly n elements (numpy, or a CPU tensor)."""
    if isinstance(a, torch.Tensor):
        if a.is_cuda:
            raise TypeError(f"{name}: expected host memory")
        a = a.detach().numpy()
    a = np.ascontiguousarray(a, dtype=np.float64).reshape(-1)
    if a.size != n:
        raise ValueError(f"{name}: expected {n} elements, got {a.size}")
    return a


# ---------------------------------------------------------------- raw ABI


def ssamg_problem_create(ndim, nparts):
    h = C.c_void_p()
    check(lib().ssamg_problem_create(ndim, nparts, C.byref(h)))
    return h


def ssamg_problem_destroy(h):
    check(lib().ssamg_problem_destroy(h))


def ssamg_problem_set_box(h, part, lo, hi):
    check(lib().ssamg_problem_set_box(h, part, _ints(lo), _ints(hi)))


def ssamg_problem_set_origin(h, part, origin):
    check(lib().ssamg_problem_set_origin(h, part, _ints(origin)))


def ssamg_problem_add_box(h, part, lo, hi):
    check(lib().ssamg_problem_add_box(h, part, _ints(lo), _ints(hi)))


def ssamg_problem_set_neighbor(h, part, face, nbr_part, at, nbr_at, map_, dir_):
    check(lib().ssamg_problem_set_neighbor(h, part, face, nbr_part, _ints(at), _ints(nbr_at), _ints(map_),
                                           _ints(dir_)))


def ssamg_problem_set_face(h, part, face, kind):
    check(lib().ssamg_problem_set_face(h, part, face, kind))


def ssamg_problem_set_stencil(h, part, offsets):
    off = np.ascontiguousarray(np.asarray(offsets, dtype=np.int32).reshape(-1))
    check(lib().ssamg_problem_set_stencil(h, part, len(off) // 3, _ints(off)))


def ssamg_problem_part_size(h, part):
    nent, ncell = C.c_int(), C.c_int64()
    check(lib().ssamg_problem_part_size(h, part, C.byref(nent), C.byref(ncell)))
    return nent.value, ncell.value


def ssamg_problem_set_coeffs(h, part, vals, constant=0):
    """vals: a float64 tensor on the HIP device, or a host array (numpy / CPU
    tensor) of nent * ncell values (nent with constant = 1)."""
    nent, ncell = ssamg_problem_part_size(h, part)
    if nent == 0:
        raise ValueError(f"part {part}: set the stencil before the coefficients")
    n = nent if constant else nent * ncell
    if isinstance(vals, torch.Tensor) and vals.is_cuda:
        t = _dev_vec(vals, n, "coefficients")
        check(lib().ssamg_problem_set_coeffs(h, part, _ptr(t), L.MEM_DEVICE, constant))
    else:
        a = _host_f64(vals, n, "coefficients")
        check(lib().ssamg_problem_set_coeffs(h, part, a.ctypes.data_as(C.c_void_p), L.MEM_HOST,
                                             constant))


def ssamg_problem_set_coupling(h, rows, cols, vals):
    """COO couplings: three host arrays, or three tensors on the HIP device
    (int64 rows and columns, float64 values) of equal length."""
    dev = [isinstance(a, torch.Tensor) and a.is_cuda for a in (rows, cols, vals)]
    if any(dev):
        if not all(dev):
            raise TypeError("couplings: rows, cols and vals must all be device tensors or all host")
        for t, dt, name in ((rows, torch.int64, "rows"), (cols, torch.int64, "cols"),
                            (vals, torch.float64, "vals")):
            if t.dtype != dt or not t.is_contiguous() or t.dim() != 1:
                raise TypeError(f"couplings: {name} must be a contiguous 1-D {dt} tensor")
        if not rows.numel() == cols.numel() == vals.numel():
            raise ValueError("couplings: rows, cols and vals differ in length")
        check(lib().ssamg_problem_set_coupling(h, rows.numel(), _ptr(rows), _ptr(cols), _ptr(vals),
                                               L.MEM_DEVICE))
        return
    r = np.ascontiguousarray(rows, dtype=np.int64).reshape(-1)
    c = np.ascontiguousarray(cols, dtype=np.int64).reshape(-1)
    v = np.ascontiguousarray(vals, dtype=np.float64).reshape(-1)
    if not r.size == c.size == v.size:
        raise ValueError("couplings: rows, cols and vals differ in length")
    check(lib().ssamg_problem_set_coupling(h, len(r), r.ctypes.data_as(C.c_void_p),
                                           c.ctypes.data_as(C.c_void_p),
                                           v.ctypes.data_as(C.c_void_p), L.MEM_HOST))


def ssamg_problem_fv_assemble(h, kappa, aniso, stencil):
    n = ssamg_problem_num_cells(h)
    np_ = ssamg_problem_num_parts(h)
    _dev_vec(kappa, n, "kappa")
    a = _host_f64(aniso, 3 * np_, "aniso")
    check(lib().ssamg_problem_fv_assemble(h, _ptr(kappa), a.ctypes.data_as(L.PD), stencil, _stream()))


def ssamg_problem_fv_grad(h, lam, x, grad):
    """lam, x: [N] or [N, nrhs] float64 device tensors; grad: [N]."""
    n = ssamg_problem_num_cells(h)
    nrhs = 1 if x.dim() == 1 else int(x.shape[1])
    _dev_vec(lam, n * nrhs, "lambda")
    _dev_vec(x, n * nrhs, "x")
    _dev_vec(grad, n, "grad")
    check(lib().ssamg_problem_fv_grad(h, nrhs, _ptr(lam), _ptr(x), _ptr(grad), _stream()))


def ssamg_problem_num_cells(h):
    n = C.c_int64()
    check(lib().ssamg_problem_num_cells(h, C.byref(n)))
    return n.value


def ssamg_problem_num_parts(h):
    n = C.c_int()
    check(lib().ssamg_problem_num_parts(h, C.byref(n)))
    return n.value


def ssamg_params_default():
    p = L.ssamg_params()
    check(lib().ssamg_params_default(C.byref(p)))
    return p


def ssamg_solver_create(prob, params, stream=None):
    h = C.c_void_p()
    check(lib().ssamg_solver_create(prob, C.byref(params), stream if stream is not None else _stream(),
                                    C.byref(h)))
    return h


def ssamg_solver_destroy(h):
    check(lib().ssamg_solver_destroy(h))


def ssamg_setup_symbolic(h):
    check(lib().ssamg_setup_symbolic(h))


def ssamg_workspace_bytes(h):
    n = C.c_size_t()
    check(lib().ssamg_workspace_bytes(h, C.byref(n)))
    return n.value


def ssamg_setup_numeric(h, ws=None):
    if ws is None:
        check(lib().ssamg_setup_numeric(h, None, 0))
    else:
        if not (isinstance(ws, torch.Tensor) and ws.is_cuda and ws.is_contiguous()):
            raise TypeError("workspace: expected a contiguous tensor on the HIP device")
        check(lib().ssamg_setup_numeric(h, _ptr(ws), ws.numel() * ws.element_size()))


TUNE_FIELDS = ("strips", "cols4", "split", "strips_mv", "cols4_mv")


def ssamg_autotune(h, nrhs, cache_path=None):
    check(lib().ssamg_autotune(h, nrhs, None if cache_path is None else str(cache_path).encode()))


def ssamg_tune_get(h, level, nrhs):
    rec = (C.c_int * 6)()
    check(lib().ssamg_tune_get(h, level, nrhs, rec))
    out = dict(zip(TUNE_FIELDS, rec[:5]))
    out["stored"] = bool(rec[5])
    return out


def ssamg_tune_set(h, level, nrhs, rec):
    arr = (C.c_int * 5)(*[int(rec[k]) for k in TUNE_FIELDS])
    check(lib().ssamg_tune_set(h, level, nrhs, arr))


def ssamg_update_coeffs(h, part, vals, where, expected):
    """New values of one part of the solver's problem; ``expected`` is the
    part's nent * ncell (the solver handle does not expose its problem)."""
    if where == L.MEM_DEVICE:
        t = _dev_vec(vals, expected, "coefficients")
        check(lib().ssamg_update_coeffs(h, part, _ptr(t), where))
    else:
        arr = _host_f64(vals, expected, "coefficients")
        check(lib().ssamg_update_coeffs(h, part, arr.ctypes.data_as(C.c_void_p), where))


def ssamg_solve(h, nrhs, b, x, layout=L.LAYOUT_CELL_MAJOR):
    n = ssamg_level_cells(h, 0) * nrhs
    _dev_vec(b, n, "b")
    _dev_vec(x, n, "x")
    info = L.ssamg_info()
    st = lib().ssamg_solve(h, nrhs, _ptr(b), _ptr(x), layout, C.byref(info))
    check(st, allow_not_converged=True)
    return st, info


def ssamg_solve_noalloc(h, nrhs, b, x, layout=L.LAYOUT_CELL_MAJOR):
    """ssamg_solve without device allocation (fixed per-GPU scratch array)."""
    n = ssamg_level_cells(h, 0) * nrhs
    _dev_vec(b, n, "b")
    _dev_vec(x, n, "x")
    info = L.ssamg_info()
    st = lib().ssamg_solve_noalloc(h, nrhs, _ptr(b), _ptr(x), layout, C.byref(info))
    check(st, allow_not_converged=True)
    return st, info


def ssamg_apply_A(h, level, x, y):
    n = ssamg_level_cells(h, level)
    _dev_vec(x, n, "x")
    _dev_vec(y, n, "y")
    check(lib().ssamg_apply_A(h, level, _ptr(x), _ptr(y)))


def ssamg_apply_precond(h, r, z):
    n = ssamg_level_cells(h, 0)
    _dev_vec(r, n, "r")
    _dev_vec(z, n, "z")
    check(lib().ssamg_apply_precond(h, _ptr(r), _ptr(z)))


def ssamg_num_levels(h):
    n = C.c_int()
    check(lib().ssamg_num_levels(h, C.byref(n)))
    return n.value


def ssamg_level_cells(h, level):
    n = C.c_int64()
    check(lib().ssamg_level_cells(h, level, C.byref(n)))
    return n.value


def ssamg_level_info(h, level, part):
    d = L.ssamg_level_desc()
    check(lib().ssamg_level_info(h, level, part, C.byref(d)))
    return d


def ssamg_direction_sums(h, nparts):
    out = np.zeros(nparts * 3)
    check(lib().ssamg_direction_sums(h, out.ctypes.data_as(L.PD)))
    return out.reshape(nparts, 3)


def ssamg_copy_stencil(h, level, part, nent, ncell):
    out = np.zeros((nent, ncell))
    check(lib().ssamg_copy_stencil(h, level, part, out.ctypes.data_as(L.PD)))
    return out


def ssamg_copy_interp(h, level, part, nf):
    wm = np.zeros(max(nf, 1))
    wp = np.zeros(max(nf, 1))
    check(lib().ssamg_copy_interp(h, level, part, wm.ctypes.data_as(L.PD), wp.ctypes.data_as(L.PD)))
    return wm[:nf], wp[:nf]


def ssamg_coupling_nnz(h, level):
    n = C.c_int64()
    check(lib().ssamg_coupling_nnz(h, level, C.byref(n)))
    return n.value


def ssamg_copy_coupling(h, level, nrows):
    nnz = ssamg_coupling_nnz(h, level)
    rp = np.zeros(nrows + 1, dtype=np.int64)
    col = np.zeros(max(nnz, 1), dtype=np.int64)
    val = np.zeros(max(nnz, 1))
    check(lib().ssamg_copy_coupling(h, level, rp.ctypes.data_as(L.PI64), col.ctypes.data_as(L.PI64),
                                    val.ctypes.data_as(L.PD)))
    return rp, col[:nnz], val[:nnz]


def ssamg_probe_set(h, kind):
    check(lib().ssamg_probe_set(h, kind))


def ssamg_probe_read(h):
    n = C.c_int64()
    ms = C.c_double()
    by = C.c_double()
    check(lib().ssamg_probe_read(h, C.byref(n), C.byref(ms), C.byref(by)))
    return n.value, ms.value, by.value


# ---------------------------------------------------------------- objects


class Problem:
    """A semi-structured problem: one box per part (lower corner 0)."""

    def __init__(self, ndim, dims, origins=None):
        self.ndim = ndim
        self.dims = [tuple(int(v) for v in d) for d in dims]
        self.nparts = len(self.dims)
        self.h = ssamg_problem_create(ndim, self.nparts)
        for p, d in enumerate(self.dims):
            ssamg_problem_set_box(self.h, p, (0, 0, 0), (d[0] - 1, d[1] - 1, d[2] - 1))
            if origins is not None:
                ssamg_problem_set_origin(self.h, p, origins[p])
        self.n = ssamg_problem_num_cells(self.h)

    def __del__(self):
        h = getattr(self, "h", None)
        if h is not None and L._lib is not None:
            L._lib.ssamg_problem_destroy(h)
            self.h = None

    @classmethod
    def from_fv(cls, geometry, stencil, kappa, aniso):
        """Finite-volume problem assembled on the device from per-cell kappa."""
        pr = cls(geometry.ndim, geometry.dims, geometry.origins)
        pr.fv_assemble(kappa, aniso, stencil)
        return pr

    @classmethod
    def from_raw(cls, case):
        """Problem given as stencil arrays + inter-part couplings (host arrays)."""
        g = case.geometry
        pr = cls(g.ndim, g.dims)
        for p in range(pr.nparts):
            for f in range(6):
                ssamg_problem_set_face(pr.h, p, f, int(case.faces[p][f]))
            ssamg_problem_set_stencil(pr.h, p, case.stencils[p])
            ssamg_problem_set_coeffs(pr.h, p, np.asarray(case.coeffs[p]).reshape(-1))
        ssamg_problem_set_coupling(pr.h, case.urow, case.ucol, case.uval)
        return pr

    @classmethod
    def from_topo(cls, case):
        """Problem with parts of several boxes and glued faces: per-part stencil
        arrays, box lists, neighbour maps and couplings (host arrays)."""
        pr = cls(case.ndim, case.dims)
        faces = case.face_kinds()
        for p in range(pr.nparts):
            for f in range(6):
                ssamg_problem_set_face(pr.h, p, f, int(faces[p][f]))
            for lo, hi in (case.boxes[p] or []):
                ssamg_problem_add_box(pr.h, p, lo, hi)
        for p in range(pr.nparts):
            for f, nb in enumerate(case.neighbors[p]):
                if nb is not None:
                    ssamg_problem_set_neighbor(pr.h, p, f, nb["part"], nb["at"], nb["nbr_at"], nb["map"],
                                               nb["dir"])
        for p in range(pr.nparts):
            ssamg_problem_set_stencil(pr.h, p, case.stencils[p])
            ssamg_problem_set_coeffs(pr.h, p, np.asarray(case.coeffs[p]).reshape(-1))
        ssamg_problem_set_coupling(pr.h, case.urow, case.ucol, case.uval)
        return pr

    def fv_assemble(self, kappa, aniso, stencil):
        """kappa: float64 tensor on the HIP device, one value per cell."""
        self._kappa = kappa
        ssamg_problem_fv_assemble(self.h, kappa, aniso, stencil)

    def fv_grad(self, lam, x):
        """-sum_k lam_k^T (dA/dkappa) x_k for [N] or [N, nrhs] lam and x."""
        g = torch.empty(self.n, dtype=torch.float64, device=x.device)
        ssamg_problem_fv_grad(self.h, lam.contiguous(), x.contiguous(), g)
        return g


class Solver:
    """SSAMG-preconditioned PCG on a Problem (which must outlive the solver)."""

    def __init__(self, problem, **params):
        self.problem = problem
        self.params = ssamg_params_default()
        for k, v in params.items():
            if not hasattr(self.params, k):
                raise TypeError(f"unknown parameter {k}")
            setattr(self.params, k, v)
        # the library orders its work on the stream current at creation; calls
        # made under another stream are ordered against it both ways (_enter
        # and _leave), so inputs produced there (fv_assemble, b) are complete
        # before the solver reads them and outputs are ready when it resumes
        self.stream = torch.cuda.current_stream()
        self.h = ssamg_solver_create(problem.h, self.params)
        self.ws = None

    def _enter(self):
        cur = torch.cuda.current_stream()
        if cur != self.stream:
            self.stream.wait_stream(cur)
        return cur

    def _leave(self, cur, *outs):
        if cur != self.stream:
            for t in outs:
                t.record_stream(self.stream)
            cur.wait_stream(self.stream)

    def __del__(self):
        h = getattr(self, "h", None)
        if h is not None and L._lib is not None:
            L._lib.ssamg_solver_destroy(h)
            self.h = None

    def setup(self):
        """Symbolic + numeric setup; the workspace is a torch uint8 tensor."""
        self.setup_symbolic()
        self.setup_numeric()
        return self

    def setup_symbolic(self):
        cur = self._enter()
        ssamg_setup_symbolic(self.h)
        self._leave(cur)
        self.nlevels = ssamg_num_levels(self.h)

    def setup_numeric(self):
        nbytes = ssamg_workspace_bytes(self.h)
        if self.ws is None or self.ws.numel() < nbytes:
            self.ws = None
            with torch.cuda.stream(self.stream):
                self.ws = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
        cur = self._enter()
        ssamg_setup_numeric(self.h, self.ws)
        self._leave(cur)

    def solve(self, b, x=None, layout=L.LAYOUT_CELL_MAJOR):
        """b: float64 device tensor, [N] or [N, nrhs] (rhs fastest) in the
        default layout, [nrhs, N] with ``layout=LAYOUT_RHS_MAJOR``.
        Returns (x, status, info); x has b's shape."""
        b = b.contiguous()
        if b.dim() == 1:
            nrhs = 1
        else:
            nrhs = int(b.shape[0] if layout == L.LAYOUT_RHS_MAJOR else b.shape[1])
        if x is None:
            x = torch.empty_like(b)
        cur = self._enter()
        st, info = ssamg_solve(self.h, nrhs, b, x, layout)
        self._leave(cur, b, x)
        return x, st, info

    def update_coeffs(self, part, vals):
        """New stencil values of one part ([nent][nz][ny][nx], same pattern: a
        CUDA float64 tensor or a host array); run setup() again before solving."""
        nent, ncell = ssamg_problem_part_size(self.problem.h, part)
        cur = self._enter()
        if isinstance(vals, torch.Tensor) and vals.is_cuda:
            v = vals.contiguous().reshape(-1)
            ssamg_update_coeffs(self.h, part, v, L.MEM_DEVICE, nent * ncell)
            self._leave(cur, v)
        else:
            ssamg_update_coeffs(self.h, part, vals, L.MEM_HOST, nent * ncell)
            self._leave(cur)

    def autotune(self, nrhs, cache_path=None):
        """Time and keep the fastest launch options of the batched cycle for
        width nrhs (optionally through a JSON cache file)."""
        ssamg_autotune(self.h, nrhs, cache_path)

    def tune_get(self, level, nrhs):
        """Launch options of a level for width nrhs: strips, cols4, split,
        strips_mv, cols4_mv, and whether they are a stored record."""
        return ssamg_tune_get(self.h, level, nrhs)

    def tune_set(self, level, nrhs, **rec):
        """Store launch options (missing fields take the current values)."""
        cur = ssamg_tune_get(self.h, level, nrhs)
        cur.update(rec)
        ssamg_tune_set(self.h, level, nrhs, cur)

    def apply_A(self, level, x):
        y = torch.empty_like(x)
        x = x.contiguous()
        cur = self._enter()
        ssamg_apply_A(self.h, level, x, y)
        self._leave(cur, x, y)
        return y

    def apply_precond(self, r):
        z = torch.empty_like(r)
        r = r.contiguous()
        cur = self._enter()
        ssamg_apply_precond(self.h, r, z)
        self._leave(cur, r, z)
        return z

    def level_info(self, level, part):
        d = ssamg_level_info(self.h, level, part)
        return {"dims": tuple(d.dims), "offset": d.offset, "dstar": d.dstar, "omega": d.omega,
                "nent": d.nent, "pattern": np.array([[d.pattern[e][a] for a in range(3)]
                                                      for e in range(d.nent)], dtype=np.int32),
                "fdims": tuple(d.fdims), "skip": d.skip}

    def level_cells(self, level):
        return sum(int(np.prod(self.level_info(level, p)["dims"])) for p in range(self.problem.nparts))

    def direction_sums(self):
        return ssamg_direction_sums(self.h, self.problem.nparts)

    def copy_stencil(self, level, part):
        li = self.level_info(level, part)
        return ssamg_copy_stencil(self.h, level, part, li["nent"], int(np.prod(li["dims"])))

    def copy_interp(self, level, part):
        li = self.level_info(level, part)
        return ssamg_copy_interp(self.h, level, part, int(np.prod(li["fdims"])) if li["dstar"] >= 0 else 0)

    def copy_coupling(self, level):
        return ssamg_copy_coupling(self.h, level, self.level_cells(level))
