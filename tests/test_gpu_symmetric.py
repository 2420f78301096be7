"""Mirrored coefficient reads (parameter symmetric = 1, the default).

For a symmetric operator the kernels read a_s(c) for a negative offset s as the
neighbour's mirrored entry a_{-s}(c + s).  Finite-volume and Galerkin
operators are symmetric only up to rounding in their stored entries, so the
mirrored operator equals the stored one to a few ulps: the level products must
agree with full reads to 1e-14 relative to |A||x|, and the solves to the
solver tolerance with the same iteration counts (+-1).
"""
import numpy as np
import pytest

import workloads as W
from tests.parity_util import gpu_fv

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _print_case(name):
    print(f"[gpu symmetric] case {name}", flush=True)


@pytest.mark.parametrize("name", ["c3_8", "c2_12", "c5_9"])
@pytest.mark.parametrize("precision", [0, 1])
def test_mirrored_reads_match_full_reads(name, precision):
    _print_case(f"{name} precision={precision}")
    case = {"c3_8": lambda: W.c3(8), "c2_12": lambda: W.c2(12), "c5_9": lambda: W.c5(9)}[name]()
    _, s1 = gpu_fv(case, cycle_precision=precision, symmetric=1)
    _, s0 = gpu_fv(case, cycle_precision=precision, symmetric=0)
    assert s1.nlevels == s0.nlevels
    rng = np.random.default_rng(3)
    for level in range(s1.nlevels):
        n = s1.level_cells(level)
        x = torch.as_tensor(rng.uniform(-1, 1, n), device="cuda")
        y1 = s1.apply_A(level, x)
        y0 = s0.apply_A(level, x)
        # scale: |A||x| of the full operator, from the product with |x| of the stored stencil
        ax = s0.apply_A(level, x.abs()).abs() + y0.abs()
        scale = float(torch.max(ax))
        assert float(torch.max(torch.abs(y1 - y0))) <= 1e-14 * scale, level
    b = torch.as_tensor(case.b if case.b.ndim == 1 else case.b[0], device="cuda")
    x1, st1, i1 = s1.solve(b)
    x0, st0, i0 = s0.solve(b)
    assert st1 == 0 and st0 == 0
    assert abs(i1.iters[0] - i0.iters[0]) <= 1
    assert i1.true_relres[0] < case.tol and i0.true_relres[0] < case.tol
    rel = float(torch.linalg.norm(x1 - x0) / torch.linalg.norm(x0))
    assert rel <= 1e-6, rel


def test_symmetric_parameter_is_checked():
    from paper_2205_14273_amd.ssamg import SSAMGError
    case = W.c1(8)
    with pytest.raises(SSAMGError):
        gpu_fv(case, symmetric=2)
