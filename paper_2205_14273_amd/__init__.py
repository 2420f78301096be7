"""Semi-structured algebraic multigrid (SSAMG) for AMD Instinct MI355X.

The solver is the HIP library ``libssamg.so`` (sources in ``csrc/``, C ABI in
``include/ssamg.h``); ``ssamg`` is its thin ctypes binding and ``autograd``
wraps x = A(kappa)^{-1} b as a differentiable function.
"""
from ._lib import SSAMGError  # noqa: F401


def __getattr__(name):
    if name in ("Problem", "Solver"):
        from . import ssamg
        return getattr(ssamg, name)
    raise AttributeError(name)
