#!/usr/bin/env python3
"""Benchmark of the AMG-DD solve phase on one MI355X.

Workload (default): 3D 7-point variable-coefficient diffusion on 192^3
(7,077,888 unknowns), k = exp(g) with g a seeded Gaussian random field
(sigma 1, correlation length 8 cells), harmonic-mean faces; 8x8x8 = 512
subdomains of 24^3, padding 2, 2 AlgFAC V(1,1) cycles per AMG-DD iteration,
FP64, b ~ U[-1, 1] (seed 0), x0 = 0.  One step = one AMG-DD solve to 1e-8
relative residual (fine residual, restriction chain, composite right-hand
sides, batched AlgFAC on all 512 composite grids, patch), with all inputs
resident in HBM.  value = DOF*cycles/s = N_0 * outer iterations / solve time.
Beside it: the mixed-precision form (its time to 1e-8 and its distance from
the FP64 iterates, iteration by iteration), the V(1,1) cycle on the same
hierarchy, the hybrid AMG-DD V-cycle (Algorithm 3), and the oracle on the
host's cores on a bounded sample of the same workload.

Prints one JSON line.  --gpus must be 1 (the solver runs on one device).
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


WORKLOADS = {
    "cfg2": "3D 7-point Laplacian 128^3 (2,097,152 DOF), 4x4x4 subdomains of 32^3, padding 1, 2 AlgFAC V(1,1) "
            "cycles per AMG-DD iteration, FP64, AMG-DD solve to 1e-8 from x0 = 0",
    "cfg3": "3D 7-point diffusion 192^3 (7,077,888 DOF), k = exp(GRF sigma 1, l 8), harmonic faces, 8x8x8 "
            "subdomains of 24^3, padding 2, 2 AlgFAC V(1,1) cycles per AMG-DD iteration, AMG-DD solve to 1e-8 "
            "from x0 = 0",
    "cfg4": "3D 7-point diffusion 96^3 (884,736 DOF), k = exp(GRF sigma 0.5), 3x3x3 subdomains of 32^3, padding 1, "
            "forward AMG-DD to 1e-10 plus adjoint AMG-DD to 1e-10 and face gradient",
    "cfg5": "256 independent 2D 5-point diffusion problems, sides U{64..512}, k log-normal sigma 1, Px,Py U{2..8}, "
            "padding U{1..3}; one batched handle; forward AMG-DD to 1e-8 plus adjoint AMG-DD to 1e-8",
    "p2": "2D rotated anisotropic diffusion (theta 3pi/16, eps 1e-3), bilinear elements, 1024^2 interior nodes "
          "(1,048,576 DOF), 4x4 subdomains of 256^2, padding 1, 2 AlgFAC cycles, FP64, AMG-DD solve to 1e-8",
}


def build_problem(name):
    from synth import batch_config, config
    if name == "cfg5":
        return batch_config()
    return config(name)


def measured_traffic(dom):
    """HBM bytes per launch of the dominant site from the committed rocprofv3
    --pmc record in profiles/, or None when no record matches this launch site
    or the kernel source changed since the counters were taken."""
    import glob
    import hashlib
    sha = hashlib.sha256(open(os.path.join(ROOT, "paper_1906_10575_amd", "csrc", "kernels.hpp"), "rb").read()).hexdigest()
    for path in glob.glob(os.path.join(ROOT, "profiles", "traffic_*.json")):
        rec = json.load(open(path))
        if (rec.get("kernels_sha256") == sha and rec.get("site") == dom["name"] and rec.get("level") == dom["level"]
                and rec.get("workgroups") == dom.get("workgroups")):
            return rec["traffic_bytes"]
    return None


def roofline(prof):
    """Dominant launch site of one iteration: algorithmic bytes per launch over
    the average launch duration (HIP events on the launch stream)."""
    dom = max(prof, key=lambda r: r["ms"])
    per_launch_ms = dom["ms"] / dom["launches"]
    per_launch_bytes = dom["bytes"] / dom["launches"]
    achieved = per_launch_bytes / (per_launch_ms * 1e-3) / 1e9
    return dom, {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                 "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": measured_traffic(dom),
                 "kernel": f"{dom['name']} (level {dom['level']})", "workgroups": dom.get("workgroups"),
                 "block": dom.get("block"), "bytes_per_launch": per_launch_bytes, "ms_per_launch": per_launch_ms}


def host_cores():
    """CPU threads this process may use (the box's share: at most 16) and a
    description of the host."""
    aff = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
    share = min(aff, 16)
    model = ""
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return share, {"nproc": os.cpu_count(), "affinity": aff, "model": model}


def cpu_baseline(seconds=10.0):
    """The oracle timed on the host (see _cpu_baseline_run), in a child
    process of its own: the worker processes it forks then never inherit a
    process that holds a GPU context or BLAS thread pools in use."""
    import subprocess
    r = subprocess.run([sys.executable, os.path.abspath(__file__), "--cpu-baseline-only", "--cpu-seconds",
                        str(seconds)], capture_output=True, text=True, timeout=3600)
    if r.returncode != 0:
        raise RuntimeError(f"CPU baseline run failed (exit {r.returncode}): {r.stderr[-2000:]}")
    return json.loads(r.stdout.strip().splitlines()[-1])


def _cpu_baseline_run(seconds=10.0):
    """The oracle (plain FP64 NumPy/SciPy, written from the paper) timed on the
    host on a bounded sample of the 192^3 workload: the 72^3 corner of the
    same coefficient field (GRF sigma 1, l 8, seed 1; harmonic faces;
    Dirichlet at the cut), 3^3 of its 24^3 subdomains, padding 2, 2 AlgFAC
    cycles, b ~ U[-1, 1] (seed 0).  Setup (hierarchy, composite grids) is
    not timed.  Two runs: one core (BLAS limited to one thread, subdomains in
    turn) and all of the host's cores (the AlgFAC phase of every iteration
    spread over worker processes, one subdomain per task; residual,
    restriction and patch stay serial).  DOF*cycles/s = N_0 * iterations /
    time."""
    from threadpoolctl import threadpool_limits

    from oracle import amg, composite, cycles
    from oracle.parallel import SubdomainPool
    from synth import grf, make_problem
    t0 = time.perf_counter()
    k = np.exp(grf((192,) * 3, 1.0, 8.0, 1))[:72, :72, :72]
    p = make_problem((72,) * 3, (3,) * 3, eta=2, n_fac=2, k=k)
    H = amg.setup(p.A)
    comps = composite.build_all(H, p.part, p.nparts, p.eta)
    co = cycles.CoarseSolver(H.A[H.L])
    setup_s = time.perf_counter() - t0
    share, host = host_cores()

    def timed(step):
        x = np.zeros(p.n)
        it = 0
        t1 = time.perf_counter()
        while time.perf_counter() - t1 < seconds or it < 3:
            x = step(x)
            it += 1
        return it, time.perf_counter() - t1

    with threadpool_limits(1):
        it1, dt1 = timed(lambda x: cycles.amgdd_iteration(H, comps, p.b, x, 2, co))
        workers = min(share, p.nparts)
        with SubdomainPool(H, comps, 2, workers, coarse=co) as pool:
            itn, dtn = timed(lambda x: pool.iteration(p.b, x))
    sample = (f"72^3 corner of the 192^3 workload's coefficient field, 3^3 subdomains of 24^3, padding 2, "
              f"2 AlgFAC cycles ({p.n} DOF); solve phase only (setup {setup_s:.0f} s untimed)")
    return {"value": round(p.n * itn / dtn, 1), "unit": "DOF*cycles/s", "cores": workers, "kind": "oracle",
            "sample": sample + f": {itn} AMG-DD iterations in {dtn:.1f} s on {workers} worker processes",
            "one_core": {"value": round(p.n * it1 / dt1, 1), "cores": 1,
                         "run": f"{it1} AMG-DD iterations in {dt1:.1f} s"},
            "host": host}


PRIMARY = {"cfg2": "fp64", "cfg3": "fp64", "cfg4": "fp64", "cfg5": "mixed", "p2": "fp64"}
HYBRID_LEVELS = {"cfg2": "1,2,3", "cfg3": "2,3", "p2": "1,2,3"}
RTOL = {"cfg2": 1e-8, "cfg3": 1e-8, "cfg4": 1e-10, "cfg5": 1e-8, "p2": 1e-8}


AMG_OPTS = {}  # relax / coarsen / interp from the command line


def make_solver(amgdd, p, precision, sched=(-2, 0), hybrid_level=0):
    if isinstance(p, list):
        return amgdd.Solver([q.A for q in p], [q.part for q in p], [q.nparts for q in p],
                            padding=[q.eta for q in p], n_fac=2, precision=precision, tail_level=sched[0],
                            tail_block=sched[1], hybrid_level=hybrid_level, **AMG_OPTS)
    return amgdd.Solver(p.A, p.part, p.nparts, padding=p.eta, n_fac=p.n_fac, precision=precision,
                        tail_level=sched[0], tail_block=sched[1], hybrid_level=hybrid_level, **AMG_OPTS)


def summarize_rocpd(db):
    """Per-kernel and per-(kernel, workgroups) duration statistics of a
    rocprofv3 --kernel-trace database (rocpd SQLite), as text."""
    import sqlite3
    con = sqlite3.connect(db)
    rows = con.execute("select name, grid_x, workgroup_x, duration from kernels").fetchall()
    agg, aggk = {}, {}
    for name, gx, wx, dur in rows:
        short = name.split("(")[0].replace("void ", "").replace("amgdd::dev::", "")
        key = (short, int(gx) // max(int(wx), 1), int(wx))
        agg.setdefault(key, []).append(dur)
        aggk.setdefault(short, []).append(dur)
    lines = ["kernel                                   calls   total_us    avg_us", "-" * 70]
    for k, v in sorted(aggk.items(), key=lambda kv: -sum(kv[1])):
        lines.append(f"{k[:40]:40s} {len(v):6d} {sum(v) / 1e3:10.1f} {sum(v) / len(v) / 1e3:9.3f}")
    lines += ["", "kernel                          workgroups x size   calls    avg_us", "-" * 70]
    for k, v in sorted(agg.items(), key=lambda kv: -sum(kv[1]))[:40]:
        lines.append(f"{k[0][:32]:32s} {k[1]:10d} x {k[2]:4d} {len(v):6d} {sum(v) / len(v) / 1e3:9.3f}")
    return "\n".join(lines)


def _pmc_means(path):
    """{(kernel, workgroups, workgroup size, counter): [values per dispatch]}
    from rocprofv3 --pmc CSV output (counter_collection.csv)."""
    import csv
    agg = {}
    with open(path) as fh:
        for row in csv.DictReader(fh):
            name = row.get("Kernel_Name", "")
            short = name.split("(")[0].replace("void ", "").replace("amgdd::dev::", "")
            grid = int(float(row.get("Grid_Size", 0) or 0))
            wg = int(float(row.get("Workgroup_Size", 1) or 1))
            key = (short, grid // max(wg, 1), wg, row.get("Counter_Name", ""))
            agg.setdefault(key, []).append(float(row.get("Counter_Value", 0) or 0))
    return agg


# launch sites of amgdd_profile -> kernel names in the counter output (a site
# runs one of these kernels, depending on the layout)
SITE_KERNEL = {"relax_pre": ("k_relax",), "relax_post": ("k_relax",), "relax_f": ("k_relax",),
               "relax_post_f": ("k_relax",), "relax_post_c": ("k_relax",), "w": ("k_w",),
               "down": ("k_down", "k_down_real"), "interp": ("k_interp", "k_interp_rows"), "restrict": ("k_spmv",),
               "restrict_s": ("k_restrict_rows",), "resid": ("k_resid",), "gather": ("k_gather",),
               "patch": ("k_patch",), "relax0": ("k_relax_zero",)}
KERNEL_REGEX = "k_w|k_relax|k_down|k_interp|k_restrict|k_spmv|k_resid|k_gather|k_patch|elementwise"
# third pass: L1->L2 read latency, addresser and wave activity
EXTRA_COUNTERS = ("GRBM_GUI_ACTIVE", "TA_TA_BUSY", "TA_ADDR_STALLED_BY_TC_CYCLES", "TCP_TCC_READ_REQ",
                  "TCP_TCC_READ_REQ_LATENCY", "SQ_WAVES", "SQ_WAVE_CYCLES", "SQ_WAIT_INST_ANY")
N_CU, N_XCD = 256, 8


def traffic_records(fetch_csv, write_csv, sites_log, workload, top=3, levels=None, names=None, extra_csv=None):
    """HBM traffic records of launch sites of one iteration: the `top` longest
    ones, or every site named in `names` on the composite levels in `levels`.
    FETCH_SIZE and WRITE_SIZE (KiB per dispatch, one rocprofv3 --pmc pass
    each, run with --calibrate-copy) are scaled by the same counters on the
    calibration kernel (y = x + 1 over 2^25 doubles: 256 MiB read, 256 MiB
    written) and matched to the sites of a `bench.py --sites` log by kernel and
    workgroup count.  With `extra_csv` (a third pass over EXTRA_COUNTERS) the
    record also gives the mean L1->L2 read latency, the addresser's busy and
    stalled fractions and the waves' waiting fraction.  Returns the records."""
    import hashlib
    f = _pmc_means(fetch_csv)
    w = _pmc_means(write_csv)
    x = _pmc_means(extra_csv) if extra_csv else {}

    def mean(agg, kerns, wgs, ctr):
        vals = [v for (k, g, _, c), vs in agg.items()
                if any(k.startswith(kn + "<") for kn in kerns) and g == wgs and c == ctr for v in vs]
        return sum(vals) / len(vals) if vals else None

    def calib(agg, ctr):
        # the y = x + 1 kernel only (fills of the same size run beside it)
        vals = [v for (k, g, _, c), vs in agg.items()
                if "elementwise" in k and "_add" in k and g == 32768 and c == ctr for v in vs]
        return sum(vals) / len(vals) if vals else None
    cf, cw = calib(f, "FETCH_SIZE"), calib(w, "WRITE_SIZE")
    if not cf or not cw:
        raise SystemExit("no calibration kernel in the counter output (run the passes with --calibrate-copy)")
    exp = 256.0 * 1024  # KiB
    sites = []
    for line in open(sites_log):
        parts = line.split()
        if len(parts) == 8 and parts[0] == "[bench]" and parts[1] in SITE_KERNEL and parts[2].isdigit():
            name, lvl, n, ms, mb, _, wg = parts[1], int(parts[2]), int(parts[3]), float(parts[4]), float(parts[5]), \
                parts[6], int(parts[7])
            sites.append(dict(name=name, level=lvl, launches=n, ms=ms, mb=mb, workgroups=wg))
    sha = hashlib.sha256(open(os.path.join(ROOT, "paper_1906_10575_amd", "csrc", "kernels.hpp"), "rb").read()).hexdigest()
    recs = []
    if levels is not None:
        chosen = [st for st in sites if st["level"] in levels and (names is None or st["name"] in names)]
    else:
        chosen = sorted(sites, key=lambda r: -r["ms"])[:top]
    for st in chosen:
        kern = SITE_KERNEL[st["name"]]
        fk, wk = mean(f, kern, st["workgroups"], "FETCH_SIZE"), mean(w, kern, st["workgroups"], "WRITE_SIZE")
        if fk is None or wk is None:
            continue
        traffic = (fk / (cf / exp) + wk / (cw / exp)) * 1024
        extra = None
        if x:
            c = {k: mean(x, kern, st["workgroups"], k) for k in EXTRA_COUNTERS}
            if all(v is not None for v in c.values()) and c["GRBM_GUI_ACTIVE"] > 0:
                cyc = c["GRBM_GUI_ACTIVE"] / N_XCD  # kernel cycles (per XCD)
                extra = {"counters": {k: round(v, 1) for k, v in c.items()},
                         "l2_read_latency_cycles": round(c["TCP_TCC_READ_REQ_LATENCY"] / max(c["TCP_TCC_READ_REQ"], 1), 1),
                         "ta_busy_frac": round(c["TA_TA_BUSY"] / N_CU / cyc, 3),
                         "ta_stalled_by_l1_frac": round(c["TA_ADDR_STALLED_BY_TC_CYCLES"] / N_CU / cyc, 3),
                         "wave_wait_frac": round(c["SQ_WAIT_INST_ANY"] / max(c["SQ_WAVE_CYCLES"], 1), 3),
                         "l2_read_requests_per_alg_kib": round(c["TCP_TCC_READ_REQ"] /
                                                               (st["mb"] * 1e6 / st["launches"] / 1024), 2)}
        recs.append({
            "what": f"HBM traffic per launch of the {st['name']} site on composite level {st['level']} of the "
                    f"{workload} AMG-DD iteration, from two rocprofv3 --pmc passes, scaled by the same counters on "
                    f"a known-size elementwise kernel (y = x + 1 over 2^25 doubles: 256 MiB read + 256 MiB written)",
            "kernels_sha256": sha, "site": st["name"], "level": st["level"], "kernel": " | ".join(k + "<...>" for k in kern),
            "workgroups": st["workgroups"], "fetch_size_kib": round(fk, 1), "write_size_kib": round(wk, 1),
            "calibration": {"fetch_size_kib": round(cf, 1), "write_size_kib": round(cw, 1), "expected_kib": exp,
                            "fetch_factor": round(cf / exp, 5), "write_factor": round(cw / exp, 5)},
            "traffic_bytes": int(round(traffic)), "algorithmic_bytes": st["mb"] * 1e6 / st["launches"],
            "traffic_over_algorithmic": round(traffic / (st["mb"] * 1e6 / st["launches"]), 3),
            "commands": [f"rocprofv3 --pmc FETCH_SIZE --kernel-include-regex '{KERNEL_REGEX}' -f csv -d <dir> -o run "
                         f"-- python3 bench.py --config {workload} --precision fp64 --steps 1 --warmup 1 "
                         f"--no-cpu-baseline --no-extras --calibrate-copy --sites",
                         "rocprofv3 --pmc WRITE_SIZE (same options)"] +
                        ([f"rocprofv3 --pmc {' '.join(EXTRA_COUNTERS)} (same options)"] if x else []) +
                        ["python3 bench.py --traffic-records <fetch csv> <write csv> <sites log> --config "
                         f"{workload}" + (" --traffic-extra <third csv>" if x else "") +
                         (f" --traffic-levels {','.join(map(str, sorted(levels)))}" if levels is not None else "") +
                         (f" --traffic-sites {','.join(sorted(names))}" if names else "")]})
        if extra:
            recs[-1]["l1_l2_path"] = extra
    return recs


def summarize_pmc(path):
    """Mean counter value per (kernel, workgroups) from rocprofv3 --pmc CSV
    output (counter_collection.csv), as text."""
    agg = _pmc_means(path)
    lines = ["kernel                           workgroups x size  counter        dispatches   mean_value", "-" * 88]
    for k, v in sorted(agg.items(), key=lambda kv: (kv[0][3], -sum(kv[1]))):
        lines.append(f"{k[0][:32]:32s} {k[1]:10d} x {k[2]:4d}  {k[3]:14s} {len(v):6d} {sum(v) / len(v):14.1f}")
    return "\n".join(lines)


def residual_rel(p, x):
    if isinstance(p, list):
        off = np.cumsum([0] + [q.n for q in p])
        return max(float(np.linalg.norm(q.b - q.A @ x[off[i]:off[i + 1]]) / np.linalg.norm(q.b))
                   for i, q in enumerate(p))
    return float(np.linalg.norm(p.b - p.A @ x) / np.linalg.norm(p.b))


def run_steps(torch, s, b, steps, rtol, adjoint, per_step=None):
    """K steps from x = 0; a step is one AMG-DD solve (plus, for the adjoint
    workloads, one adjoint AMG-DD solve with right-hand side u), bracketed by
    device synchronisation (every solve returns with its stream drained, so
    per-step host times are exact).  Returns (seconds, iterations per step, x)
    and appends each step's seconds to per_step."""
    iters = []
    zeros = [torch.zeros_like(b) for _ in range(2 * steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(steps):
        ts = time.perf_counter()
        x, info, st = s.solve(b, zeros[2 * k], rtol=rtol, maxit=300)
        it = info.iters
        if adjoint:
            lam, info2, st2 = s.solve_adjoint(x, zeros[2 * k + 1], rtol=rtol, maxit=300)
            it += info2.iters
        iters.append(it)
        if per_step is not None:
            per_step.append(time.perf_counter() - ts)
    torch.cuda.synchronize()
    return time.perf_counter() - t0, iters, x


def mixed_vs_fp64(torch, s64, smx, b, iters, rtol):
    """Distance of the mixed-precision iterates from the FP64 ones, iteration
    by iteration from x0 = 0 (||x_mixed - x_fp64|| / ||x_fp64||), and of the
    two solutions at the tolerance."""
    x64 = torch.zeros_like(b)
    xm = torch.zeros_like(b)
    per_iter = []
    for _ in range(iters):
        x64, _, _ = s64.solve(b, x64, rtol=0, maxit=1)
        xm, _, _ = smx.solve(b, xm, rtol=0, maxit=1)
        per_iter.append(float(torch.linalg.norm(xm - x64) / torch.linalg.norm(x64)))
    x64, _, _ = s64.solve(b, torch.zeros_like(b), rtol=rtol, maxit=300)
    xm, _, _ = smx.solve(b, torch.zeros_like(b), rtol=rtol, maxit=300)
    return per_iter, float(torch.linalg.norm(xm - x64) / torch.linalg.norm(x64))


def sweep(torch, amgdd, cfg, args):
    """The paper's parameter study (Section 6.1) at one-GPU scale: padding
    eta x AlgFAC cycles per iteration x relaxation order (natural / CF
    l1-Jacobi), each solved to the workload's tolerance from x0 = 0 in FP64.
    Per configuration: iterations, asymptotic factor, time to tolerance,
    composite overhead, and the paper's nnz cost proxy per iteration
    (composite overhead x AlgFAC cycles, in units of the hierarchy's nnz)."""
    import dataclasses
    p0 = build_problem(cfg)
    if isinstance(p0, list):
        raise SystemExit("bench.py --sweep: single-problem workloads only")
    rtol = RTOL[cfg]
    b = torch.as_tensor(p0.b, device="cuda:0")
    rows = []

    def timed(fn, reps=3):
        fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(reps):
            x, info, st = fn()
        torch.cuda.synchronize()
        return (time.perf_counter() - t0) / reps, x, info, st

    for relax in ("l1", "cf"):
        for eta in [int(v) for v in args.sweep_eta.split(",")]:
            p = dataclasses.replace(p0, eta=eta)
            for nfac in [int(v) for v in args.sweep_nfac.split(",")]:
                t0 = time.perf_counter()
                s = amgdd.Solver(p.A, p.part, p.nparts, padding=eta, n_fac=nfac, relax=relax,
                                 coarsen=AMG_OPTS["coarsen"], interp=AMG_OPTS["interp"])
                setup_s = time.perf_counter() - t0
                ov = s.stats()["composite_overhead"]
                dt, x, info, st = timed(lambda: s.solve(b, torch.zeros_like(b), rtol=rtol, maxit=300))
                rec = {"solver": "amgdd", "relax": relax, "eta": eta, "n_fac": nfac, "iters": info.iters,
                       "rho": round(info.rho_asym, 4), "time_to_tol_ms": round(dt * 1e3, 3),
                       "ms_per_iter": round(dt * 1e3 / max(info.iters, 1), 4), "composite_overhead": round(ov, 4),
                       "nnz_cost_per_iter": round(ov * nfac, 3), "status": st, "setup_s": round(setup_s, 2),
                       "relres_fp64": residual_rel(p, x.cpu().numpy())}
                rows.append(rec)
                log(f"sweep {rec}")
                s.close()
            if eta == 1:
                s = amgdd.Solver(p.A, p.part, p.nparts, padding=eta, n_fac=1, relax=relax,
                                 coarsen=AMG_OPTS["coarsen"], interp=AMG_OPTS["interp"])
                dt, x, info, st = timed(lambda: s.vsolve(b, torch.zeros_like(b), rtol=rtol, maxit=400))
                rec = {"solver": "vcycle", "relax": relax, "iters": info.iters, "rho": round(info.rho_asym, 4),
                       "time_to_tol_ms": round(dt * 1e3, 3), "ms_per_iter": round(dt * 1e3 / max(info.iters, 1), 4),
                       "status": st, "relres_fp64": residual_rel(p, x.cpu().numpy())}
                rows.append(rec)
                log(f"sweep {rec}")
                s.close()
            torch.cuda.empty_cache()
    print(json.dumps({"sweep": cfg, "workload": WORKLOADS[cfg], "rtol": rtol, "precision": "fp64", "rows": rows}),
          flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--config", default="cfg3", choices=sorted(WORKLOADS))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true")
    ap.add_argument("--tail-level", type=int, default=-2, help="fixed AlgFAC schedule cut level (-2: autotune)")
    ap.add_argument("--tail-block", type=int, default=0, help="fixed persistent workgroup size (0: autotune)")
    ap.add_argument("--hybrid-levels", default=None,
                    help="transition levels of the hybrid AMG-DD cycles timed beside the primary solve")
    ap.add_argument("--summarize-rocpd", metavar="DB", help="print a summary of a rocprofv3 kernel-trace database")
    ap.add_argument("--summarize-pmc", metavar="CSV", help="print a summary of rocprofv3 --pmc CSV output")
    ap.add_argument("--traffic-records", nargs=3, metavar=("FETCH_CSV", "WRITE_CSV", "SITES_LOG"),
                    help="write profiles/traffic_<site>_l<level>_<config>.json for the longest launch sites from "
                         "FETCH_SIZE / WRITE_SIZE --pmc output and a --sites log (host only)")
    ap.add_argument("--traffic-extra", metavar="CSV", help="third --pmc pass (EXTRA_COUNTERS) for --traffic-records")
    ap.add_argument("--traffic-levels", default=None,
                    help="comma-separated composite levels: records for every site there instead of the longest")
    ap.add_argument("--traffic-sites", default=None, help="comma-separated site names for --traffic-levels")
    ap.add_argument("--relax", default="l1", choices=["l1", "cf"], help="l1-Jacobi order (natural / CF)")
    ap.add_argument("--coarsen", default="rs", choices=["rs", "hmis"])
    ap.add_argument("--interp", default="direct", choices=["direct", "ext+i"])
    ap.add_argument("--sweep", action="store_true",
                    help="parameter sweep on the workload instead of the benchmark line: padding x AlgFAC cycles x "
                         "relaxation order, plus the V-cycle in both orders (one JSON line)")
    ap.add_argument("--sweep-eta", default="1,2,3")
    ap.add_argument("--sweep-nfac", default="1,2,4,10")
    ap.add_argument("--sites", action="store_true",
                    help="also print every launch site of one iteration (device time, algorithmic bytes, rate)")
    ap.add_argument("--precision", choices=["fp64", "mixed"], default=None,
                    help="override the workload's primary precision (the JSON line then reports that one)")
    ap.add_argument("--calibrate-copy", action="store_true",
                    help="also run 3 elementwise copies of 256 MiB (known HBM traffic, to scale PMC counters)")
    ap.add_argument("--cpu-seconds", type=float, default=10.0, help="seconds per CPU-baseline run")
    ap.add_argument("--cpu-baseline-only", action="store_true",
                    help="only time the oracle on the host (one JSON line; no GPU is touched)")
    args = ap.parse_args()
    if args.cpu_baseline_only:
        print(json.dumps(_cpu_baseline_run(args.cpu_seconds)), flush=True)
        return
    if args.summarize_rocpd:
        print(summarize_rocpd(args.summarize_rocpd))
        return
    if args.summarize_pmc:
        print(summarize_pmc(args.summarize_pmc))
        return
    if args.traffic_records:
        lv = None if args.traffic_levels is None else {int(v) for v in args.traffic_levels.split(",")}
        nm = None if args.traffic_sites is None else set(args.traffic_sites.split(","))
        for rec in traffic_records(*args.traffic_records, workload=args.config, levels=lv, names=nm,
                                   extra_csv=args.traffic_extra):
            path = os.path.join(ROOT, "profiles", f"traffic_{rec['site']}_l{rec['level']}_{args.config}.json")
            with open(path, "w") as fh:
                json.dump(rec, fh, indent=1)
            ex = rec.get("l1_l2_path")
            print(f"{path}: {rec['traffic_bytes'] / 1e6:.1f} MB traffic, {rec['algorithmic_bytes'] / 1e6:.1f} MB "
                  f"algorithmic per launch" + (f"; L2 latency {ex['l2_read_latency_cycles']} cycles, TA busy "
                                               f"{ex['ta_busy_frac']}, waves waiting {ex['wave_wait_frac']}"
                                               if ex else ""))
        return
    if args.gpus != 1:
        print(f"bench.py: the solver runs on one GPU (the multi-GPU exchange is a design only); --gpus {args.gpus} "
              f"is not supported", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_1906_10575_amd import amgdd

    cfg = args.config
    AMG_OPTS.update(relax=args.relax, coarsen=args.coarsen, interp=args.interp)
    if args.sweep:
        return sweep(torch, amgdd, cfg, args)
    prec = args.precision or PRIMARY[cfg]
    rtol = RTOL[cfg]
    adjoint = cfg in ("cfg4", "cfg5")
    p = build_problem(cfg)
    n = sum(q.n for q in p) if isinstance(p, list) else p.n
    log(f"{cfg}: n={n}, primary precision {prec}, rtol {rtol}, adjoint {adjoint}")
    t0 = time.perf_counter()
    s = make_solver(amgdd, p, prec, (args.tail_level, args.tail_block))
    setup_s = time.perf_counter() - t0
    st = s.stats()
    log(f"setup {setup_s:.1f} s, grids {st['n_grids']}, levels {st['max_levels']}, overhead "
        f"{st['composite_overhead']:.3f}, device {st['device_bytes'] / 2**30:.2f} GiB")
    bh = np.concatenate([q.b for q in p]) if isinstance(p, list) else p.b
    b = torch.as_tensor(bh, device="cuda:0")

    run_steps(torch, s, b, args.warmup, rtol, adjoint)
    st = s.stats()
    log(f"warmup done; schedule: cut level {st['tail_level']}, workgroup {st['tail_block']}, 512-thread levels "
        f"{[l for l in range(32) if (st['wide_levels'] >> l) & 1]}, LDS-band levels "
        f"{[l for l in range(32) if (st['lds_levels'] >> l) & 1]} / restriction "
        f"{[l for l in range(32) if (st['restrict_lds_levels'] >> l) & 1]} (autotune {st['autotune_s']:.2f} s)")
    per_step = []
    dt, iters, x = run_steps(torch, s, b, args.steps, rtol, adjoint, per_step)
    its = int(np.median(iters))
    ms_per_step = dt / args.steps * 1e3
    value = n * sum(iters) / dt
    relres = residual_rel(p, x.cpu().numpy())
    step_ms = {"mean": round(ms_per_step, 4), "median": round(float(np.median(per_step)) * 1e3, 4),
               "min": round(float(np.min(per_step)) * 1e3, 4), "max": round(float(np.max(per_step)) * 1e3, 4)}
    log(f"AMG-DD: {its} iterations per step, {ms_per_step:.2f} ms per step (median {step_ms['median']:.2f}, "
        f"min {step_ms['min']:.2f}), {value:.3e} DOF*cycles/s, final relres (FP64, host) {relres:.2e}")

    if args.calibrate_copy:
        # y = x + 1 over 2^25 doubles: 256 MiB read, 256 MiB written per launch
        xc = torch.ones(1 << 25, dtype=torch.float64, device="cuda:0")
        yc = torch.empty_like(xc)
        for _ in range(3):
            torch.add(xc, 1.0, out=yc)
        torch.cuda.synchronize()
        del xc, yc
        log("calibration copies done (3 x 256 MiB read + 256 MiB write)")

    prof = s.profile(kind=0, reps=3)
    dom, roof = roofline(prof)
    iter_ms = sum(r_["ms"] for r_ in prof)
    if args.sites:
        log(f"{'site':14s} {'lvl':>3s} {'n':>2s} {'ms/iter':>8s} {'MB/iter':>9s} {'GB/s':>7s} {'wg':>6s}")
        for r_ in sorted(prof, key=lambda r_: (r_["level"], r_["name"])):
            gbs = r_["bytes"] / (r_["ms"] * 1e-3) / 1e9 if r_["ms"] > 0 else 0.0
            log(f"{r_['name']:14s} {r_['level']:3d} {r_['launches']:2d} {r_['ms']:8.4f} {r_['bytes'] / 1e6:9.1f} "
                f"{gbs:7.0f} {r_['workgroups']:6d}")
    log(f"dominant launch {roof['kernel']}: {roof['ms_per_launch']:.4f} ms, {roof['achieved']:.0f} GB/s "
        f"({100 * roof['frac']:.1f}% of HBM peak); kernel time per iteration {iter_ms:.3f} ms")
    iter_bytes = sum(r_["bytes"] for r_ in prof)

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
        "dtype": "f64" if prec == "fp64" else "f32 inner / f64 outer",
        "data": "synthetic",
        "config": {"workload": f"{cfg}: {WORKLOADS[cfg]}", "dof": n, "grids": st["n_grids"],
                   "precision": prec, "rtol": rtol, "relax": args.relax, "coarsen": args.coarsen,
                   "interp": args.interp},
        "iters_per_step": its,
        "time_to_tol_ms": round(ms_per_step, 4),
        "step_ms": step_ms,
        "final_relres_fp64": relres,
        "roofline": roof,
        "kernel_ms_per_iteration": round(iter_ms, 4),
        "iteration_alg_gbs": round(iter_bytes / (iter_ms * 1e-3) / 1e9, 1),
        "profile_top": sorted(({k: (round(v, 5) if isinstance(v, float) else v) for k, v in r_.items()}
                               for r_ in prof), key=lambda r_: -r_["ms"])[:8],
        "schedule": {"tail_level": st["tail_level"], "tail_block": st["tail_block"],
                     "wide_levels": [l for l in range(32) if (st["wide_levels"] >> l) & 1],
                     "lds_levels": [l for l in range(32) if (st["lds_levels"] >> l) & 1],
                     "restrict_lds_levels": [l for l in range(32) if (st["restrict_lds_levels"] >> l) & 1],
                     "autotune_s": round(st["autotune_s"], 3), "cached": bool(st["schedule_cached"])},
        "setup_s": round(setup_s, 2),
        "composite_overhead": round(st["composite_overhead"], 4),
    }
    if not args.no_extras:
        k = max(3, args.steps // 2)
        if not isinstance(p, list) and not adjoint:
            s.vsolve(b, torch.zeros_like(b), rtol=rtol, maxit=400)
            vstep = []
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            itv = []
            for _ in range(k):
                ts = time.perf_counter()
                xv, infov, _ = s.vsolve(b, torch.zeros_like(b), rtol=rtol, maxit=400)
                vstep.append(time.perf_counter() - ts)
                itv.append(infov.iters)
            torch.cuda.synchronize()
            dtv = time.perf_counter() - t0
            out["vcycle"] = {"iters": int(np.median(itv)), "time_to_tol_ms": round(dtv / k * 1e3, 4),
                             "step_ms_median": round(float(np.median(vstep)) * 1e3, 4),
                             "step_ms_min": round(float(np.min(vstep)) * 1e3, 4),
                             "dof_cycles_per_s": round(n * sum(itv) / dtv, 1)}
            log(f"V(1,1): {out['vcycle']}")
        other = "mixed" if prec == "fp64" else "fp64"
        so = make_solver(amgdd, p, other)
        run_steps(torch, so, b, 1, rtol, adjoint)
        ostep = []
        dto, ito, xo = run_steps(torch, so, b, k, rtol, adjoint, ostep)
        out[other] = {"iters_per_step": int(np.median(ito)), "time_to_tol_ms": round(dto / k * 1e3, 4),
                      "step_ms_median": round(float(np.median(ostep)) * 1e3, 4),
                      "step_ms_min": round(float(np.min(ostep)) * 1e3, 4),
                      "dof_cycles_per_s": round(n * sum(ito) / dto, 1),
                      "final_relres_fp64": residual_rel(p, xo.cpu().numpy())}
        if not adjoint:
            # error of the reduced-precision iterates against the FP64 ones
            s64, smx = (s, so) if prec == "fp64" else (so, s)
            per_iter, at_tol = mixed_vs_fp64(torch, s64, smx, b, its, rtol)
            out["mixed_error"] = {"what": "||x_mixed - x_fp64|| / ||x_fp64|| after each iteration from x0 = 0, "
                                          "and of the two solutions at the tolerance",
                                  "per_iter": [float(f"{e:.3e}") for e in per_iter],
                                  "at_tol": float(f"{at_tol:.3e}")}
            log(f"mixed vs FP64: {out['mixed_error']}")
        log(f"{other}: {out[other]}")
        del so
        del s
        torch.cuda.empty_cache()
        hl = args.hybrid_levels if args.hybrid_levels is not None else HYBRID_LEVELS.get(cfg, "")
        if not isinstance(p, list) and not adjoint and hl:
            # hybrid AMG-DD V-cycles (Algorithm 3), same precision and tolerance
            out["hybrid"] = []
            for lt in [int(v) for v in hl.split(",") if v.strip()]:
                t0 = time.perf_counter()
                sh = make_solver(amgdd, p, prec, hybrid_level=lt)
                hsetup = time.perf_counter() - t0
                run_steps(torch, sh, b, 1, rtol, False)
                hstep = []
                dth, ith, xh = run_steps(torch, sh, b, k, rtol, False, hstep)
                sth = sh.stats()
                rec = {"level": lt, "iters": int(np.median(ith)), "time_to_tol_ms": round(dth / k * 1e3, 4),
                       "step_ms_median": round(float(np.median(hstep)) * 1e3, 4),
                       "dof_cycles_per_s": round(n * sum(ith) / dth, 1), "grids": sth["n_grids"],
                       "composite_overhead": round(sth["composite_overhead"], 4), "setup_s": round(hsetup, 2),
                       "device_gib": round(sth["device_bytes"] / 2**30, 3),
                       "final_relres_fp64": residual_rel(p, xh.cpu().numpy()),
                       "schedule": {"tail_level": sth["tail_level"], "tail_block": sth["tail_block"],
                                    **{k: [l for l in range(32) if (sth[k] >> l) & 1]
                                       for k in ("wide_levels", "lds_levels", "restrict_lds_levels")}}}
                out["hybrid"].append(rec)
                log(f"hybrid L~={lt}: {rec}")
                del sh
                torch.cuda.empty_cache()
    if not args.no_cpu_baseline and cfg == "cfg3":
        out["cpu_baseline"] = cpu_baseline(args.cpu_seconds)
        log(f"cpu baseline: {out['cpu_baseline']}")
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
