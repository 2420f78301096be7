"""Launch options of the batched V-cycle and the autotuner that picks them.

The options only change how the kernels cover a level (four columns per thread
or one, the z-plane strip order of the four-column sweeps, the first sweep
split from the residual or fused with it, the same for the FP64 product of
PCG), never what they compute, so every option must give bit-identical
solutions and iteration counts.  The workload is the 2 x 24^3, 32 right-hand
side version of the batched benchmark problem: at that width the z-planes of
levels 0 and 1 split into whole blocks and the eight XCD ranges hold whole
planes, so the strip orders really permute the blocks (with strips that do and
do not divide a plane's block count).
"""
import json

import numpy as np
import pytest

import workloads as W
from tests.parity_util import gpu_fv

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

FP64, FP32 = 0, 1
NRHS = 32
DEFAULT = {"strips": 1, "cols4": -1, "split": -1, "strips_mv": 1, "cols4_mv": -1}


def _print_case(name):
    print(f"[gpu autotune] case {name}", flush=True)


def _setup(precision, **params):
    case = W.c4(24, nrhs=NRHS)
    B = torch.as_tensor(np.ascontiguousarray(case.b.T), device="cuda")
    _, s = gpu_fv(case, max_nrhs=NRHS, cycle_precision=precision, **params)
    return case, B, s


def _solve(s, B):
    x, st, info = s.solve(B)
    assert st == 0
    return x, [info.iters[k] for k in range(NRHS)]


VARIANTS = [
    {"cols4": 0},
    {"cols4": 1, "strips": 2},
    {"cols4": 1, "strips": 4},          # 18 blocks per plane at level 0: strips of 5, 5, 5, 3
    {"cols4": 1, "strips": 6},
    {"split": 0},
    {"split": 1},
    {"cols4": 0, "split": 1},
]
VARIANTS_MV = [{"cols4_mv": 0}, {"cols4_mv": 1, "strips_mv": 3}, {"cols4_mv": 1, "strips_mv": 8}]


@pytest.mark.parametrize("precision", [FP64, FP32])
def test_every_launch_option_is_bit_identical(precision):
    _print_case(f"c4_24 x {NRHS} options precision={precision}")
    _, B, s = _setup(precision)
    x0, it0 = _solve(s, B)
    variants = VARIANTS + (VARIANTS_MV if precision == FP32 else [])
    for level in (0, 1):
        for v in variants:
            if level > 0 and "cols4_mv" in v:
                continue
            s.tune_set(level, NRHS, **{**DEFAULT, **v})
            x, it = _solve(s, B)
            assert it == it0, (level, v)
            assert torch.equal(x, x0), (level, v)
            s.tune_set(level, NRHS, **DEFAULT)


def test_tune_set_rejects_bad_records():
    _print_case("c4_24 bad records")
    from paper_2205_14273_amd.ssamg import SSAMGError
    _, _, s = _setup(FP32)
    for bad in ({"strips": 0}, {"strips": 65}, {"split": 2}, {"cols4": -2}, {"cols4_mv": 3}):
        with pytest.raises(SSAMGError):
            s.tune_set(0, NRHS, **{**DEFAULT, **bad})
    with pytest.raises(SSAMGError):
        s.tune_set(0, 1, **{**DEFAULT, "cols4": 1})       # one column per solve: no four-column sweep
    with pytest.raises(SSAMGError):
        s.tune_set(0, 3, **DEFAULT)                        # not a power of two


def test_autotune_keeps_results_and_round_trips_its_cache(tmp_path):
    _print_case("c4_24 autotune + cache")
    _, B, s = _setup(FP32)
    x0, it0 = _solve(s, B)
    cache = tmp_path / "tune.json"
    s.autotune(NRHS, cache)
    eligible = [l for l in range(s.nlevels) if s.level_cells(l) * NRHS >= 1 << 16]
    assert 0 in eligible and 1 in eligible
    recs = {l: s.tune_get(l, NRHS) for l in eligible}
    for l in eligible:
        assert recs[l]["stored"], l
    x, it = _solve(s, B)
    assert it == it0 and torch.equal(x, x0)
    data = json.loads(cache.read_text())
    assert data["format"] == "ssamg-autotune-1"
    assert len(data["records"]) >= len(eligible)
    for r in data["records"]:
        assert set(r) == {"key", "strips", "cols4", "split", "strips_mv", "cols4_mv"}
        assert "|lg5" in r["key"]
    # a new solver of the same shapes takes the records from the file
    _, _, s2 = _setup(FP32)
    s2.autotune(NRHS, cache)
    for l in eligible:
        assert s2.tune_get(l, NRHS) == recs[l], l
    x2, it2 = _solve(s2, B)
    assert it2 == it0 and torch.equal(x2, x0)


def test_autotune_parameter_tunes_on_first_solve():
    _print_case("c4_24 autotune=1")
    _, B, s0 = _setup(FP32)
    x0, it0 = _solve(s0, B)
    _, _, s = _setup(FP32, autotune=1)
    assert not s.tune_get(0, NRHS)["stored"]
    x, it = _solve(s, B)
    assert s.tune_get(0, NRHS)["stored"]
    assert it == it0 and torch.equal(x, x0)
    # the records survive a new setup of the same shapes
    s.setup()
    assert s.tune_get(0, NRHS)["stored"]
    x, it = _solve(s, B)
    assert it == it0 and torch.equal(x, x0)
