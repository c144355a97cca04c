#!/usr/bin/env python3
"""Benchmark of the AMG-DD solve phase on one MI355X.

Workload (default): 3D 7-point Laplacian on 128^3 (2,097,152 unknowns),
4x4x4 = 64 subdomains of 32^3, padding 1, 2 AlgFAC V(1,1) cycles per AMG-DD
iteration, FP64, b ~ U[-1, 1] (seed 0), x0 = 0.  One step = one AMG-DD solve
to 1e-8 relative residual (fine residual, restriction chain, composite
right-hand sides, batched AlgFAC on all 64 composite grids, patch), with all
inputs resident in HBM.  value = DOF*cycles/s = N_0 * outer iterations /
solve time.  The V(1,1) cycle on the same hierarchy and the mixed-precision
form are timed beside it and reported as extra fields.

Prints one JSON line.  --gpus must be 1 (this build runs on one GPU).
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def build_problem(name):
    from synth import config
    return config(name)


def timed_solves(torch, fn, b, steps, rtol, maxit):
    """K solves from x = 0, bracketed by device synchronisation."""
    iters = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        x = torch.zeros_like(b)
        x, info, st = fn(b, x, rtol=rtol, maxit=maxit)
        iters.append(info.iters)
    torch.cuda.synchronize()
    return time.perf_counter() - t0, iters, x


def roofline(prof):
    """Dominant launch site of one iteration: algorithmic bytes per launch over
    the average launch duration (HIP events on the launch stream)."""
    dom = max(prof, key=lambda r: r["ms"])
    per_launch_ms = dom["ms"] / dom["launches"]
    per_launch_bytes = dom["bytes"] / dom["launches"]
    achieved = per_launch_bytes / (per_launch_ms * 1e-3) / 1e9
    return dom, {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                 "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": None,
                 "kernel": f"{dom['name']} (level {dom['level']})", "bytes_per_launch": per_launch_bytes,
                 "ms_per_launch": per_launch_ms}


def cpu_baseline(seconds=12.0):
    """The oracle (plain serial FP64 NumPy/SciPy) timed on the host: AMG-DD
    iterations on a 64^3 Laplacian with 2^3 subdomains of 32^3 (cfg2's
    subdomain size, padding and cycle count at 1/8 of its subdomains), BLAS
    limited to one thread; DOF*cycles/s = N_0 * iterations / time."""
    from threadpoolctl import threadpool_limits

    from oracle import amg, composite, cycles
    from synth import make_problem
    p = make_problem((64, 64, 64), (2, 2, 2), eta=1, n_fac=2)
    H = amg.setup(p.A)
    comps = composite.build_all(H, p.part, p.nparts, p.eta)
    co = cycles.CoarseSolver(H.A[H.L])
    with threadpool_limits(1):
        x = np.zeros(p.n)
        it = 0
        t0 = time.perf_counter()
        while time.perf_counter() - t0 < seconds or it < 3:
            x = cycles.amgdd_iteration(H, comps, p.b, x, 2, co)
            it += 1
        dt = time.perf_counter() - t0
    return {"value": round(p.n * it / dt, 1), "unit": "DOF*cycles/s", "cores": 1, "kind": "oracle",
            "sample": f"64^3 Laplacian, 2^3 subdomains of 32^3, padding 1, 2 AlgFAC cycles: {it} AMG-DD "
                      f"iterations in {dt:.1f} s (setup excluded)"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--config", default="cfg2")
    ap.add_argument("--rtol", type=float, default=1e-8)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: this build runs on one GPU; --gpus {args.gpus} is not supported", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1906_10575_amd import amgdd

    p = build_problem(args.config)
    log(f"{args.config}: n={p.n} nnz={p.A.nnz} parts={p.nparts} eta={p.eta} n_fac={p.n_fac}")
    t0 = time.perf_counter()
    s = amgdd.Solver(p.A, p.part, p.nparts, padding=p.eta, n_fac=p.n_fac)
    setup_s = time.perf_counter() - t0
    st = s.stats()
    log(f"setup {setup_s:.1f} s, grids {st['n_grids']}, levels {st['max_levels']}, overhead "
        f"{st['composite_overhead']:.3f}, device {st['device_bytes'] / 2**30:.2f} GiB")
    b = torch.as_tensor(p.b, device="cuda:0")

    for _ in range(args.warmup):
        s.solve(b, torch.zeros_like(b), rtol=args.rtol, maxit=200)
    log("warmup done")
    dt, iters, x = timed_solves(torch, s.solve, b, args.steps, args.rtol, 200)
    its = int(np.median(iters))
    ms_per_step = dt / args.steps * 1e3
    value = p.n * sum(iters) / dt
    r = p.b - p.A @ x.cpu().numpy()
    relres = float(np.linalg.norm(r) / np.linalg.norm(p.b))
    log(f"AMG-DD: {its} iterations, {ms_per_step:.2f} ms per solve, {value:.3e} DOF*cycles/s, relres {relres:.2e}")

    prof = s.profile(kind=0, reps=3)
    dom, roof = roofline(prof)
    iter_ms = sum(r_["ms"] for r_ in prof)
    log(f"dominant launch {roof['kernel']}: {roof['ms_per_launch']:.4f} ms, {roof['achieved']:.0f} GB/s "
        f"({100 * roof['frac']:.1f}% of HBM peak); kernel time per iteration {iter_ms:.3f} ms")

    out = {
        "metric": "DOF*cycles/s and time to 1e-8 rel. residual, FP64 vs mixed; % of HBM roofline",
        "value": round(value, 1),
        "unit": "DOF*cycles/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"{args.config}: 3D 7-point Laplacian 128^3 (2,097,152 DOF), 4x4x4 subdomains of "
                               "32^3, padding 1, 2 AlgFAC V(1,1) cycles per AMG-DD iteration, RS theta 0.25 + direct "
                               "interpolation to <= 16 points, l1-Jacobi, AMG-DD solve to 1e-8 from x0 = 0",
                   "dof": p.n, "subdomains": p.nparts, "padding": p.eta, "n_fac": p.n_fac, "rtol": args.rtol},
        "amgdd_iters": its,
        "time_to_tol_ms": round(ms_per_step, 4),
        "final_relres_fp64": relres,
        "roofline": roof,
        "kernel_ms_per_iteration": round(iter_ms, 4),
        "profile_top": sorted(({k: (round(v, 5) if isinstance(v, float) else v) for k, v in r_.items()}
                               for r_ in prof), key=lambda r_: -r_["ms"])[:8],
        "setup_s": round(setup_s, 2),
        "composite_overhead": round(st["composite_overhead"], 4),
    }
    if not args.no_extras:
        dtv, itv, xv = timed_solves(torch, s.vsolve, b, max(3, args.steps // 2), args.rtol, 400)
        kv = max(3, args.steps // 2)
        out["vcycle"] = {"iters": int(np.median(itv)), "time_to_tol_ms": round(dtv / kv * 1e3, 4),
                         "dof_cycles_per_s": round(p.n * sum(itv) / dtv, 1)}
        log(f"V(1,1): {out['vcycle']}")
        sm = amgdd.Solver(p.A, p.part, p.nparts, padding=p.eta, n_fac=p.n_fac, precision="mixed")
        sm.solve(b, torch.zeros_like(b), rtol=args.rtol, maxit=200)
        dtm, itm, xm = timed_solves(torch, sm.solve, b, max(3, args.steps // 2), args.rtol, 200)
        km = max(3, args.steps // 2)
        rm = p.b - p.A @ xm.cpu().numpy()
        out["mixed"] = {"iters": int(np.median(itm)), "time_to_tol_ms": round(dtm / km * 1e3, 4),
                        "dof_cycles_per_s": round(p.n * sum(itm) / dtm, 1),
                        "final_relres_fp64": float(np.linalg.norm(rm) / np.linalg.norm(p.b))}
        log(f"mixed: {out['mixed']}")
        del sm
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline()
        log(f"cpu baseline: {out['cpu_baseline']}")
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
