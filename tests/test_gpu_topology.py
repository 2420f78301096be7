"""Parts of several boxes and glued (rotated) part faces through the C ABI.

The library turns the topology (box lists with ghost cells, neighbour maps)
into its semi-structured operator itself; the oracle does the same from the
same description with its own code.  Integer structure must match bit for bit
(levels, d*, boxes, coupling CSR), values to a row-relative 1e-12, the cycle
entry by entry, and solves to the oracle's iterations +-1.

Workloads: three cubes around a common edge with quarter-turned index spaces
(the shape of the paper's test case 3), one level of adaptive refinement with
ghost unknowns under the patch and -2/3 fine-coarse couplings (test case 4),
an L-shaped part of two boxes, and two cubes whose second index space is
turned against the first.
"""
import numpy as np
import pytest

import workloads as W
from oracle import ssamg as O
from tests.parity_util import (CYCLE_RTOL, assert_cycle_close, compare_hierarchy, gpu_topo, oracle_topo,
                               vcycle_scale)

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _cuda(a):
    return torch.as_tensor(np.ascontiguousarray(a), device="cuda", dtype=torch.float64)


def _print_case(name):
    print(f"[gpu topology] case {name}", flush=True)


def _l_shape():
    offs = W.stencil_offsets(27)
    rng = np.random.default_rng(9)
    dims = [(12, 10, 7), (9, 10, 7)]
    # part 0: an L of two boxes; part 1 glued to part 0's +x face (Cartesian)
    co = []
    t = rng.uniform(0.5, 1.5, (13,))      # shared by both parts: couplings across the glue stay symmetric
    for p, (nx, ny, nz) in enumerate(dims):
        c = np.zeros((27, nz, ny, nx))
        for e, s in enumerate(offs[1:], start=1):
            # symmetric constant couplings: a_s = a_{-s}
            key = tuple(s) if (s[2], s[1], s[0]) > (0, 0, 0) else tuple(-np.asarray(s))
            half = [tuple(o) for o in offs[1:] if (o[2], o[1], o[0]) > (0, 0, 0)]
            c[e] = -t[half.index(key)]
        c[0] = -c[1:].sum(axis=0) + rng.uniform(0.0, 0.2, (nz, ny, nx))
        co.append(c)
    boxes = [[((0, 0, 0), (11, 4, 6)), ((0, 5, 0), (5, 9, 6))], None]
    nb = [[None] * 6 for _ in range(2)]
    nb[0][1] = {"part": 1, "at": (12, 0, 0), "nbr_at": (0, 0, 0), "map": (0, 1, 2), "dir": (1, 1, 1)}
    nb[1][0] = {"part": 0, "at": (-1, 0, 0), "nbr_at": (11, 0, 0), "map": (0, 1, 2), "dir": (1, 1, 1)}
    n = sum(a * b * c for a, b, c in dims)
    b = rng.uniform(-1, 1, n)
    return W.TopoCase("L27", dims, [offs, offs], co, boxes, nb, np.zeros(0, dtype=np.int64),
                      np.zeros(0, dtype=np.int64), np.zeros(0), b)


def _rotated_pair():
    from tests.test_oracle_pins import _two_cubes
    return _two_cubes(9, rotated=True)


CASES = {
    "tc3_8": lambda: W.tc3_junction(8),
    "tc3_13": lambda: W.tc3_junction(13),
    "tc4_8": lambda: W.tc4_samr(8),
    "tc4_16": lambda: W.tc4_samr(16),
    "L27": _l_shape,
    "rot9": _rotated_pair,
}


@pytest.mark.parametrize("name", list(CASES))
@pytest.mark.parametrize("precision", [0, 1])
def test_topology_parity(name, precision):
    _print_case(f"{name} precision={precision}")
    case = CASES[name]()
    h = oracle_topo(case)
    pr, s = gpu_topo(case, cycle_precision=precision)
    compare_hierarchy(h, s, len(case.dims))
    r = np.random.default_rng(71).uniform(-1, 1, h.levels[0].n)
    z = s.apply_precond(_cuda(r)).cpu().numpy()
    assert_cycle_close(z, O.vcycle(h, r), vcycle_scale(h, r), CYCLE_RTOL[precision], name)
    ref = O.solve(h, case.b, tol=1e-8, flexible=(precision == 1))
    x, st, info = s.solve(_cuda(case.b))
    assert st == 0 and abs(info.iters[0] - ref.iters) <= 1, (info.iters[0], ref.iters)
    assert info.true_relres[0] < 1e-8
    assert np.linalg.norm(x.cpu().numpy() - ref.x) <= 1e-6 * np.linalg.norm(ref.x)


def test_ghost_cells_keep_their_right_hand_side():
    """A ghost unknown's row is the identity, so x = b there; with b = 0 on the
    ghost cells their solution is zero up to the solver's tolerance (the
    preconditioned directions do touch them; the residual there does not)."""
    case = W.tc4_samr(8)
    m, a, b_ = 8, 2, 6
    ghost = np.zeros(case.n, dtype=bool)
    for k in range(a, b_):
        for j in range(a, b_):
            for i in range(a, b_):
                ghost[i + m * (j + m * k)] = True
    bb = case.b.copy()
    bb[ghost] = 0.0
    pr, s = gpu_topo(case)
    x, st, info = s.solve(_cuda(bb))
    xg = x.cpu().numpy()
    assert st == 0 and np.max(np.abs(xg[ghost])) <= 1e-8 * np.max(np.abs(xg))


def test_topology_argument_errors():
    from paper_2205_14273_amd import ssamg as B
    from paper_2205_14273_amd._lib import SSAMGError
    pr = B.Problem(3, [(4, 4, 4), (4, 4, 4)])
    with pytest.raises(SSAMGError):      # not a point across the face
        B.ssamg_problem_set_neighbor(pr.h, 0, 1, 1, (3, 0, 0), (0, 0, 0), (0, 1, 2), (1, 1, 1))
    with pytest.raises(SSAMGError):      # not a permutation
        B.ssamg_problem_set_neighbor(pr.h, 0, 1, 1, (4, 0, 0), (0, 0, 0), (0, 0, 2), (1, 1, 1))
    with pytest.raises(SSAMGError):      # glued to itself
        B.ssamg_problem_set_neighbor(pr.h, 0, 1, 0, (4, 0, 0), (0, 0, 0), (0, 1, 2), (1, 1, 1))
    with pytest.raises(SSAMGError):      # box outside the part
        B.ssamg_problem_add_box(pr.h, 0, (0, 0, 0), (4, 3, 3))
    # a coupling on a ghost cell
    B.ssamg_problem_add_box(pr.h, 0, (0, 0, 0), (1, 3, 3))
    with pytest.raises(SSAMGError) as e:
        B.ssamg_problem_set_coupling(pr.h, [3, 64], [64, 3], [-1.0, -1.0])     # cell 3 of part 0 is a ghost
    assert e.value.status == -1
    # fv_assemble does not place parts with topology
    with pytest.raises(SSAMGError) as e:
        B.ssamg_problem_fv_assemble(pr.h, torch.ones(128, dtype=torch.float64, device="cuda"),
                                    np.ones((2, 3)), 7)
    assert e.value.status == -3
