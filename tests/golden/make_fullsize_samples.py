"""Write full-size sampled oracle values for a benchmark workload, from the
oracle alone (tests/golden/<config>_samples.json).

Stored:
* the first two AMG-DD iterates and V(1,1) iterates at 2000 seeded sample
  points, with the residual norms ||b - A x_k||;
* the FP64 AMG-DD residual history to 1e-8 and, for the mixed-precision form,
  the oracle's float32 emulation (composite data and FAC cycle in float32,
  residual, patch and coarsest solve in float64) run beside it: per iteration
  ||x_f32 - x_f64|| / ||x_f64|| and its residual history.

The AMG-DD iteration is the oracle's with its subdomain loop spread over
worker processes (oracle.parallel.SubdomainPool; every subdomain's AlgFAC
cycles are independent, Section 3), checked against cycles.amgdd_iteration
bitwise on a small problem before it runs.  Runs for tens of minutes at 192^3.

    python tests/golden/make_fullsize_samples.py --config cfg3 [--workers 8]
    python tests/golden/make_fullsize_samples.py --config cfg2 --mixed-only
"""

import argparse
import json
import multiprocessing as mp
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import amg, composite, cycles  # noqa: E402
from oracle.parallel import SubdomainPool  # noqa: E402
from synth import config, make_problem  # noqa: E402

# state shared with forked workers
_G = {}


def _build(q):
    return composite.build_composite(_G["H"], _G["part"], q, _G["eta"])


def build_all(H, part, nparts, eta, workers):
    _G.update(H=H, part=part, eta=eta)
    with mp.get_context("fork").Pool(workers) as pool:
        return pool.map(_build, range(nparts), chunksize=1)


def self_check(workers):
    p = make_problem((24, 20, 18), (2, 2, 2), eta=2, n_fac=2)
    H = amg.setup(p.A)
    comps = composite.build_all(H, p.part, p.nparts, p.eta)
    cp = build_all(H, p.part, p.nparts, p.eta, workers)
    co = cycles.CoarseSolver(H.A[H.L])
    with SubdomainPool(H, cp, p.n_fac, workers, coarse=co) as pool:
        for dtype in (np.float64, np.float32):
            x1 = cycles.amgdd_iteration(H, comps, p.b, np.zeros(p.n), p.n_fac, co, dtype=dtype)
            x2 = pool.iteration(p.b, np.zeros(p.n), dtype=dtype)
            assert np.array_equal(x1, x2), "parallel driver differs from cycles.amgdd_iteration"


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--config", default="cfg3")
    ap.add_argument("--workers", type=int, default=8)
    ap.add_argument("--mixed-only", action="store_true")
    ap.add_argument("--rtol", type=float, default=1e-8)
    args = ap.parse_args()
    t0 = time.time()
    self_check(args.workers)
    print(f"self-check passed {time.time() - t0:.0f} s", flush=True)
    p = config(args.config)
    H = amg.setup(p.A)
    print(f"hierarchy {[A.shape[0] for A in H.A]} {time.time() - t0:.0f} s", flush=True)
    comps = build_all(H, p.part, p.nparts, p.eta, args.workers)
    print(f"{len(comps)} composite grids {time.time() - t0:.0f} s", flush=True)
    co = cycles.CoarseSolver(H.A[H.L])
    pool = SubdomainPool(H, comps, p.n_fac, args.workers, coarse=co)
    rng = np.random.default_rng(123)
    idx = np.sort(rng.choice(p.n, 2000, replace=False))
    out = {"what": f"oracle samples of the {args.config} workload (tests/golden/make_fullsize_samples.py)",
           "workload": f"{args.config}: n {p.n}, {p.nparts} subdomains, padding {p.eta}, {p.n_fac} AlgFAC cycles",
           "levels": [int(A.shape[0]) for A in H.A], "nnz": [int(A.nnz) for A in H.A], "idx": idx.tolist(),
           "omissions": int(sum(lev.omissions for cg in comps for lev in cg.levels))}
    bn = float(np.linalg.norm(p.b))
    # FP64 and float32-emulated AMG-DD side by side, to rtol
    x = np.zeros(p.n)
    xf = np.zeros(p.n)
    hist, histf, err = [bn], [bn], []
    for k in range(60):
        if hist[-1] <= args.rtol * bn and histf[-1] <= args.rtol * bn:
            break
        x = pool.iteration(p.b, x)
        xf = pool.iteration(p.b, xf, dtype=np.float32)
        hist.append(float(np.linalg.norm(p.b - p.A @ x)))
        histf.append(float(np.linalg.norm(p.b - p.A @ xf)))
        err.append(float(np.linalg.norm(xf - x) / np.linalg.norm(x)))
        if k < 2 and not args.mixed_only:
            out[f"amgdd_x{k + 1}"] = x[idx].tolist()
        print(f"iteration {k + 1}: relres {hist[-1] / bn:.3e} / f32 {histf[-1] / bn:.3e}, "
              f"f32 vs f64 {err[-1]:.3e}  {time.time() - t0:.0f} s", flush=True)
    pool.close()
    out["amgdd_hist"] = hist
    out["mixed_emulation"] = {"hist": histf, "err_vs_fp64": err,
                              "what": "float32 emulation of the mixed form (M1-M4): per iteration "
                                      "||x_f32 - x_f64|| / ||x_f64|| and ||b - A x_f32||"}
    if not args.mixed_only:
        x = np.zeros(p.n)
        vh = [bn]
        for k in range(2):
            x = cycles.vcycle(H, x, p.b, coarse=co)
            vh.append(float(np.linalg.norm(p.b - p.A @ x)))
            out[f"vcycle_x{k + 1}"] = x[idx].tolist()
        out["vcycle_hist"] = vh
    name = f"{args.config}_mixed_error.json" if args.mixed_only else f"{args.config}_samples.json"
    with open(os.path.join(HERE, name), "w") as fh:
        json.dump(out, fh, indent=0)
    print(f"wrote {name} {time.time() - t0:.0f} s", flush=True)


if __name__ == "__main__":
    main()
