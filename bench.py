#!/usr/bin/env python3
"""SSAMG benchmark on one MI355X: seconds of setup + solve to a 1e-8 relative
residual, FP32 V-cycle inside FP64 PCG (the timed step) next to the FP64 cycle,
the roofline of the dominant kernel, and the CPU oracle as baseline.

A step is one pass of the whole hot path over one synthetic input already
resident in HBM: finite-volume assembly from kappa, symbolic + numeric setup
(metric, Algorithm 1, interpolation, Galerkin products, FP32 copies) and the
preconditioned CG solve.  Prints exactly one JSON line on stdout; progress goes
to stderr.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--config c3]

The default workload is the largest single-GPU configuration: 8 parts of 128^3
(16.8M cells), 27-point heterogeneous diffusion.  The main roofline is that of
its dominant kernel, the FP64 product q = A p of PCG; the finest-level
post-smoothing sweep of the cycle is reported beside it.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "SSAMG setup+solve sec to 1e-8 rel residual (FP64 vs FP32 V-cycle); HBM GB/s"
HBM_PEAK_GBS = 8000.0

DESCR = {
    "c1": "1 part 16^3, 7-point Laplacian, fixed omega 2/3",
    "c2": "4 parts of 64^3 along x, 7-point diffusion, anisotropy 100:1:1 strong x,y,z,x",
    "c3": "8 parts of 128^3 in 2x2x2, 27-point, log-normal kappa (sigma 2), 1e4 part jumps",
    "c4": "2 parts of 96^3 along x, 7-point, anisotropy 10:1:1, 32 right-hand sides",
    "c5": "3 parts of 64^3 along x, 7-point, kappa = exp(N(0,1)), adjoint gradient",
}

# finest-level kernel kinds the library can time with HIP events, and the
# kernel names rocprofv3 reports for them in a mixed-precision cycle
PROBES = {
    "matvec": (0, "k_stencil<double, 3, double, double, 1, {n}>"),      # product that also forms p.q
    "resid0": (2, "k_smooth_resid<float, double, 1, {n}>"),
    "restrict0": (3, "k_restrict<float>"),
    "interp0": (4, "k_interp_add<float>"),
    "jacobi0": (5, "k_stencil<float, 2, double, double, 1, {n}>"),
}
# batched solves: the post-sweep also forms r.z and z.q (mode 4)
PROBES_BATCHED = {"jacobi0": "k_stencil<float, 4, double, double, 1, {n}>"}


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def kernel_source_hash():
    """Hash of the source file that defines the probed cycle kernels."""
    h = hashlib.sha256()
    with open(os.path.join(ROOT, "paper_2205_14273_amd", "csrc", "kernels_vcycle.hip"), "rb") as fh:
        h.update(fh.read())
    return h.hexdigest()[:16]


def stencil_entries(case):
    return 7 if case.stencil in (5, 7) else (9 if case.stencil == 9 else 27)


def stored_traffic(config, probe):
    """HBM bytes per launch measured with rocprofv3 --pmc for this kernel, if the
    stored measurement was taken on the current kernel sources."""
    path = os.path.join(ROOT, "profiles", f"traffic_{config}_{probe}.txt")
    if not os.path.exists(path):
        return None
    vals = {}
    with open(path) as fh:
        for line in fh:
            if ":" in line and not line.startswith("#"):
                k, v = line.split(":", 1)
                vals[k.strip()] = v.strip()
    if vals.get("kernel_source_hash") != kernel_source_hash():
        return None
    try:
        return float(vals["hbm_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--config", default="c3", choices=sorted(DESCR))
    ap.add_argument("--m", type=int, default=None, help="box size override (smaller runs)")
    ap.add_argument("--probe", default="matvec", choices=sorted(PROBES),
                    help="kernel of the main roofline (timed with HIP events in the timed run)")
    ap.add_argument("--probe2", default="jacobi0", choices=sorted(PROBES) + ["none"],
                    help="kernel of the second roofline (a short extra run of the FP32 cycle)")
    ap.add_argument("--hybrid-level", type=int, default=0, metavar="K",
                    help="hybrid coarse tail: end the hierarchy at level K and solve it exactly "
                         "(0: off)")
    ap.add_argument("--coarse-op", default="galerkin", choices=["galerkin", "nongalerkin"],
                    help="coarse stencils of 7-point parts: Galerkin (default) or the non-Galerkin "
                         "option for isotropic problems")
    ap.add_argument("--skip", action="store_true",
                    help="the skip option of Section 3.4 (no relaxation where a part coarsens along the "
                         "same direction as ndim levels above)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--no-autotune", action="store_true",
                    help="batched configurations: keep the default launch options")
    ap.add_argument("--autotune-cache", default=None, metavar="PATH",
                    help="batched configurations: read the launch options of tuned levels from "
                         "this JSON file (levels not in it are timed) and write them back")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="only run 5 device-to-device copies of MIB MiB (the reference kernel "
                         "that scales rocprofv3 FETCH_SIZE/WRITE_SIZE readings) and exit")
    args = ap.parse_args()

    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path; use --gpus 1",
              file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import workloads as W
    from paper_2205_14273_amd import ssamg as B

    if not torch.cuda.is_available():
        print("bench.py needs a HIP device", file=sys.stderr)
        sys.exit(1)
    dev = torch.device("cuda:0")

    if args.calibrate_copy:
        nbytes = args.calibrate_copy << 20
        src = torch.ones(nbytes // 4, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        for _ in range(5):
            dst.copy_(src)
        torch.cuda.synchronize()
        print(json.dumps({"calibrate_copy_bytes": nbytes, "copies": 5}))
        return

    mk = W.CONFIGS[args.config]
    case = mk(args.m) if args.m else mk()
    g = case.geometry
    N = g.n
    nrhs = case.nrhs
    log(f"config {args.config} N={N} nrhs={nrhs}")
    kappa = torch.as_tensor(case.kappa, device=dev)
    if nrhs == 1:
        b = torch.as_tensor(case.b, device=dev)
    else:
        b = torch.as_tensor(np.ascontiguousarray(case.b.T), device=dev)   # [N][nrhs]
    aniso = case.aniso

    def make_solver(precision):
        pr = B.Problem(g.ndim, g.dims, g.origins)
        params = dict(cycle_precision=precision, max_nrhs=nrhs, tol=case.tol,
                      max_iter=case.max_iter,
                      relax=B.L.RELAX_L1_JACOBI if case.relax == "l1" else B.L.RELAX_JACOBI)
        if case.omega > 0:
            params["omega"] = case.omega
        if args.hybrid_level > 0:
            params["hybrid_level"] = args.hybrid_level
        if args.coarse_op == "nongalerkin":
            params["coarse_op"] = B.L.COARSE_OP_NONGALERKIN
        if args.skip:
            params["skip"] = 1
        pr.fv_assemble(kappa, aniso, case.stencil)
        s = B.Solver(pr, **params)
        return pr, s

    def step(pr, s, x):
        t0 = time.perf_counter()
        pr.fv_assemble(kappa, aniso, case.stencil)
        t1 = time.perf_counter()
        s.setup_symbolic()
        ts = time.perf_counter()
        s.setup_numeric()
        t2 = time.perf_counter()
        x, st, info = s.solve(b, x)
        t3 = time.perf_counter()
        if st != 0:
            raise RuntimeError(f"solve did not converge: status {st}")
        return x, info, (t1 - t0, t2 - t1, t3 - t2, ts - t1, t2 - ts)

    tune_s = {}

    def run(precision, steps, warmup, probe_kind=None):
        pr, s = make_solver(precision)
        x = torch.empty_like(b)
        if nrhs >= 4 and not args.no_autotune:
            # launch options of the batched cycle: timed once on this hierarchy,
            # kept by the solver across the setups of the timed steps
            s.setup()
            t0 = time.perf_counter()
            s.autotune(nrhs, args.autotune_cache)
            tune_s[precision] = time.perf_counter() - t0
            log(f"  autotune ({'fp32' if precision else 'fp64'} cycle): {tune_s[precision]*1e3:.1f} ms")
            for lev in range(s.nlevels):
                rec = s.tune_get(lev, nrhs)
                if rec.pop("stored"):
                    log(f"    level {lev}: {rec}")
        for _ in range(warmup):
            x, info, _ = step(pr, s, x)
        if probe_kind is not None:
            B.ssamg_probe_set(s.h, probe_kind)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        phases = []
        for k in range(steps):
            x, info, ph = step(pr, s, x)
            phases.append(ph)
            log(f"  {'fp32' if precision else 'fp64'} cycle step {k}: assemble {ph[0]*1e3:.2f} ms, "
                f"setup {ph[1]*1e3:.2f} ms (symbolic {ph[3]*1e3:.2f}, numeric {ph[4]*1e3:.2f}), "
                f"solve {ph[2]*1e3:.2f} ms, iters {info.iters[0]}")
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        probe = B.ssamg_probe_read(s.h) if probe_kind is not None else None
        ph = np.median(np.asarray(phases), axis=0)
        its = [info.iters[k] for k in range(nrhs)]
        res = {"ms_per_step": (t1 - t0) / steps * 1e3, "assemble_s": ph[0], "setup_s": ph[1],
               "solve_s": ph[2], "symbolic_s": ph[3], "numeric_s": ph[4],
               "iters": its if nrhs > 1 else its[0],
               "true_relres": max(info.true_relres[k] for k in range(nrhs)), "levels": s.nlevels}
        return res, x, probe, s

    nent = stencil_entries(case)

    def probe_name_of(probe):
        kind, name = PROBES[probe]
        if nrhs >= 4 and probe in PROBES_BATCHED:
            name = PROBES_BATCHED[probe]
        name = name.format(n=nent)
        if probe == "matvec" and nent > 7:
            name = name[:-1] + ", true>"       # mirrored reads of a symmetric stencil
        p2 = os.environ.get("SSAMG_PRODUCT2", "1")
        if (probe == "matvec" and nrhs == 1 and nent == 27 and p2 != "0"
                and all(dd[0] % 2 == 0 for dd in g.dims)):
            # two cells per thread (full 27-point, even rows); 2: the row
            # neighbours come from the adjacent lanes
            name = "k_product2s<true>" if p2 == "2" else "k_product2<true>"
        if nrhs >= 4 and not (name.startswith("k_stencil<double") and nent == 27):
            # four right-hand-side columns per thread on batched levels
            name = name.replace("k_stencil<", "k_stencil4<")
        return kind, name

    def roofline(probe, meas):
        """Achieved bandwidth of one kernel: algorithmic bytes per launch over
        its average duration (HIP events recorded by the kernel's own dispatch,
        on the solver's stream, over every launch of the timed steps)."""
        if not meas or meas[0] <= 0:
            return None
        launches, ms, by = meas
        avg_s = ms / launches * 1e-3
        streamed = by / launches                     # what the kernel must stream
        alg = streamed
        if probe == "matvec":
            # the product's algorithmic bytes as the survey counts them: every
            # stencil entry, x and y, (s + 2) * 8 bytes per cell and column
            alg = float(N) * (nent + 2 * nrhs) * 8
        achieved = alg / avg_s / 1e9
        out = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
               "frac": round(achieved / HBM_PEAK_GBS, 4),
               "traffic": stored_traffic(args.config, probe),
               "kernel": probe_name_of(probe)[1], "launches": launches,
               "avg_launch_us": round(avg_s * 1e6, 2), "alg_bytes_per_launch": alg}
        if streamed != alg:
            # mirrored reads: only the center and the positive half of the
            # symmetric stencil are streamed
            out["streamed_bytes_per_launch"] = streamed
            out["achieved_streamed"] = round(streamed / avg_s / 1e9, 1)
            out["frac_streamed"] = round(streamed / avg_s / 1e9 / HBM_PEAK_GBS, 4)
        return out

    log("timed run: FP32 V-cycle inside FP64 PCG")
    mixed, x32, probe, s32 = run(B.L.FP32, args.steps, args.warmup, probe_name_of(args.probe)[0])
    fp64 = None
    x64 = None
    if not args.no_fp64:
        log("comparison run: FP64 V-cycle (same steps)")
        fp64, x64, _, _ = run(B.L.FP64, args.steps, args.warmup)
    per_rhs = None
    if nrhs > 1:
        # the same right-hand sides solved one at a time on the same hierarchy
        # (solve only: setup is shared), against the batched solve per column
        log(f"sequential run: the {nrhs} right-hand sides one by one (FP32 cycle)")
        cols = [b[:, k].contiguous() for k in range(nrhs)]
        xs = torch.empty_like(cols[0])
        s32.solve(cols[0], xs)                      # captures the one-column graph
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        its = []
        for col in cols:
            _, st1, inf1 = s32.solve(col, xs)
            its.append(inf1.iters[0])
        torch.cuda.synchronize()
        seq = (time.perf_counter() - t0) * 1e3
        per_rhs = {"batched_solve_ms_per_rhs": round(mixed["solve_s"] * 1e3 / nrhs, 4),
                   "sequential_solve_ms_per_rhs": round(seq / nrhs, 4),
                   "sequential_iters_min_max": [min(its), max(its)]}
        log(f"  sequential: {seq:.1f} ms for {nrhs} solves ({seq / nrhs:.2f} ms each), iters {min(its)}-{max(its)}")
    roof = roofline(args.probe, probe)
    roof2 = None
    if args.probe2 != "none" and args.probe2 != args.probe:
        log(f"second roofline: {args.probe2}, two more FP32-cycle steps")
        _, _, probe2, _ = run(B.L.FP32, 2, 0, probe_name_of(args.probe2)[0])
        roof2 = roofline(args.probe2, probe2)

    cpu = None
    err = {}
    if not args.no_cpu_baseline:
        log("cpu baseline: oracle on the host cores")
        from oracle import assemble, ssamg as O
        scale = 1.0
        iter_scale = 1.0
        if args.config in ("c3",) and not args.m:
            sample_case = W.c3(64)
            scale = N / sample_case.geometry.n
            sample = (f"c3 recipe at 8 parts of 64^3 ({sample_case.geometry.n:,} cells; the full "
                      f"workload does not fit the oracle's time bound): assembly and setup scaled by "
                      f"the cell ratio {scale:g}, the solve by the cell ratio times the ratio of the "
                      f"GPU's iterations at full size to the oracle's on the sample")
        elif args.config == "c4":
            sample_case = case
            sample = "full c4 problem with its first right-hand side, time scaled by 32"
            scale = float(nrhs)
        else:
            sample_case = case
            sample = f"full {args.config} workload, one step (FV assembly + setup + PCG to 1e-8), FP64"
        sg = sample_case.geometry
        t0 = time.perf_counter()
        A, _ = assemble.assemble_fv(sg, sample_case.stencil, sample_case.kappa, sample_case.aniso)
        h = O.setup(A, sg.dims, sg.face_kinds(), [W.stencil_offsets(sample_case.stencil, sg.ndim)]
                    * sg.nparts, sg.ndim, omega=sample_case.omega, relax=sample_case.relax,
                    hybrid_level=args.hybrid_level, coarse_op=args.coarse_op, skip=args.skip)
        ts = time.perf_counter()
        bb = sample_case.b if sample_case.b.ndim == 1 else sample_case.b[0]
        ref = O.solve(h, bb, tol=sample_case.tol, max_iter=sample_case.max_iter)
        t1 = time.perf_counter()
        gpu_iters = mixed["iters"] if nrhs == 1 else mixed["iters"][0]
        if sample_case is not case and args.config == "c3":
            iter_scale = gpu_iters / max(ref.iters, 1)
        value = ((ts - t0) + (t1 - ts) * iter_scale) * scale
        cpu = {"value": round(value, 3), "unit": "s", "cores": 1, "kind": "oracle",
               "sample": sample, "iters": ref.iters, "measured_s": round(t1 - t0, 3),
               "measured_setup_s": round(ts - t0, 3), "measured_solve_s": round(t1 - ts, 3),
               "cell_ratio": scale, "iter_ratio": round(iter_scale, 4)}
        log(f"  oracle: {t1 - t0:.2f} s (assembly + setup {ts - t0:.2f}, solve {t1 - ts:.2f}), "
            f"iters {ref.iters}")
        if sample_case is case:
            xo = ref.x
            for name, xg in (("fp32_cycle", x32), ("fp64_cycle", x64)):
                if xg is None:
                    continue
                xv = xg.cpu().numpy()
                if nrhs > 1:
                    xv = xv[:, 0]
                err[name] = float(np.linalg.norm(xv - xo) / np.linalg.norm(xo))
            cpu["iters_vs_gpu"] = {"oracle": ref.iters,
                                   "gpu_fp32_cycle": mixed["iters"] if nrhs == 1 else mixed["iters"][0]}

    if x64 is not None:
        # the FP32 cycle's solution against the FP64 cycle's at full size (the
        # oracle's own solution is compared at the sizes it reaches, in tests)
        err["fp32_vs_fp64_cycle"] = float(torch.linalg.norm(x32 - x64) / torch.linalg.norm(x64))
    ms = mixed["ms_per_step"]
    line = {
        "metric": METRIC,
        "value": round(ms / 1e3, 6),
        "unit": "s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms, 4),
        "higher_is_better": False,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64+f32",
        "data": "synthetic",
        "config": {"workload": f"{args.config}: {DESCR[args.config]}; FP32 V(1,1) cycle in FP64 PCG, "
                               f"tol {case.tol}"
                               + (f"; hybrid tail at level {args.hybrid_level}" if args.hybrid_level else "")
                               + ("; non-Galerkin coarse stencils" if args.coarse_op == "nongalerkin" else "")
                               + ("; skip option" if args.skip else ""),
                   "cells": N, "nrhs": nrhs,
                   "levels": mixed["levels"], "iters": mixed["iters"],
                   "assemble_s": round(mixed["assemble_s"], 6), "setup_s": round(mixed["setup_s"], 6),
                   "setup_symbolic_s": round(mixed["symbolic_s"], 6),
                   "setup_numeric_s": round(mixed["numeric_s"], 6),
                   "solve_s": round(mixed["solve_s"], 6), "true_relres": mixed["true_relres"],
                   "autotune_s": round(tune_s[1], 4) if 1 in tune_s else None},
        "roofline_cycle_sweep": roof2,
        "per_rhs": per_rhs,
        "fp64_cycle": None if fp64 is None else {
            "ms_per_step": round(fp64["ms_per_step"], 4), "setup_s": round(fp64["setup_s"], 6),
            "solve_s": round(fp64["solve_s"], 6), "iters": fp64["iters"],
            "true_relres": fp64["true_relres"]},
        "err_vs_oracle": err or None,
        "roofline": roof,
        "cpu_baseline": cpu,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
