"""x = A(kappa)^{-1} b as a differentiable function of kappa and b.

A(kappa) is the finite-volume operator the library assembles on the device
(two-point harmonic-mean conductances, zero-Dirichlet ghosts outside every
part).  The backward pass is the adjoint method: with g = dL/dx,

    lambda = A^{-T} g = A^{-1} g          (A is symmetric)
    dL/db       = lambda
    dL/dkappa_c = -lambda^T (dA/dkappa_c) x

The adjoint solve reuses the SSAMG hierarchy built in the forward pass (same
operator, so no second setup), and the last line is one pass of the library's
``fv_grad`` kernels over the cells and the inter-part couplings.
"""
from __future__ import annotations

import torch

from .ssamg import Problem, Solver, SSAMGError


class FVSolver:
    """One geometry (boxes, origins, stencil, anisotropy) and its SSAMG solver.

    ``solve(kappa, b)`` assembles A(kappa), runs the setup when kappa changed,
    and solves; it is differentiable in kappa and b.  b is [N] or [N, nrhs]
    (right-hand side index fastest, nrhs a power of two <= max_nrhs).
    """

    def __init__(self, geometry, stencil, aniso, **params):
        self.geometry = geometry
        self.stencil = int(stencil)
        self.aniso = aniso
        self.problem = Problem(geometry.ndim, geometry.dims, geometry.origins)
        self.solver = Solver(self.problem, **params)
        self._kappa = None          # the kappa the current hierarchy was built from
        self._kappa_version = None

    def _prepare(self, kappa):
        """Assemble and set up for ``kappa`` unless the hierarchy already matches it."""
        if (self._kappa is not None and self._kappa.data_ptr() == kappa.data_ptr()
                and self._kappa_version == kappa._version and self._kappa.shape == kappa.shape):
            return
        self.problem.fv_assemble(kappa, self.aniso, self.stencil)
        self.solver.setup()
        self._kappa = kappa
        self._kappa_version = kappa._version

    def _solve(self, kappa, b):
        self._prepare(kappa)
        x, status, info = self.solver.solve(b)
        if status != 0:
            raise SSAMGError(status, f"solve did not converge (relres {info.relres[0]:.3e})")
        return x

    def solve(self, kappa, b):
        return _SSAMGSolve.apply(kappa, b, self)


class _SSAMGSolve(torch.autograd.Function):
    @staticmethod
    def forward(ctx, kappa, b, fv):
        kappa = kappa.detach().contiguous()
        x = fv._solve(kappa, b.detach().contiguous())
        ctx.fv = fv
        ctx.save_for_backward(kappa, x)
        return x

    @staticmethod
    def backward(ctx, gx):
        kappa, x = ctx.saved_tensors
        fv = ctx.fv
        lam = fv._solve(kappa, gx.contiguous())
        grad_kappa = None
        if ctx.needs_input_grad[0]:
            # one kernel pass sums the contributions of every right-hand side
            grad_kappa = fv.problem.fv_grad(lam, x)
        grad_b = lam if ctx.needs_input_grad[1] else None
        return grad_kappa, grad_b, None


def ssamg_solve(kappa, b, fv: FVSolver):
    """Functional form: x = A(kappa)^{-1} b with the solver state held by ``fv``."""
    return _SSAMGSolve.apply(kappa, b, fv)
