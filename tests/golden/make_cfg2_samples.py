"""Write tests/golden/cfg2_samples.json from the oracle alone.

Workload: 3D 7-point Laplacian 128^3, 4x4x4 subdomains of 32^3, padding 1,
2 AlgFAC cycles per AMG-DD iteration, b ~ U[-1, 1] (seed 0), x0 = 0.
Stored: the residual norms ||b - A x_k|| for k = 0..2 of AMG-DD and of
V(1,1), and the iterates x_1, x_2 of both at 2000 seeded sample points.
With --hybrid L, the same for the hybrid AMG-DD V-cycle with transition
level L (Algorithm 3) into cfg2_hybrid_samples.json.
Runs for several minutes (the oracle's RS setup at 2M unknowns is slow).

    python tests/golden/make_cfg2_samples.py [--hybrid 2]
"""

import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import amg, composite, cycles  # noqa: E402
from synth import config  # noqa: E402


def hybrid(p, H, lt, t0):
    lt, Hs, comps = cycles.hybrid_setup(H, p.part, p.nparts, p.eta, lt)
    print(f"level-{lt} composite grids {time.time() - t0:.0f} s", flush=True)
    co = cycles.CoarseSolver(Hs.A[Hs.L])
    rng = np.random.default_rng(123)
    idx = np.sort(rng.choice(p.n, 2000, replace=False))
    out = {"what": "hybrid AMG-DD V-cycle samples", "workload": "cfg2 128^3 4x4x4 eta 1 n_fac 2 seed 0",
           "hybrid_level": lt, "levels": [int(A.shape[0]) for A in H.A], "idx": idx.tolist()}
    x = np.zeros(p.n)
    hist = [float(np.linalg.norm(p.b))]
    for k in range(2):
        r = p.b - p.A @ x
        x = x + cycles.hybrid_vcycle(H, Hs, comps, np.zeros(p.n), r, lt, p.n_fac, co)
        hist.append(float(np.linalg.norm(p.b - p.A @ x)))
        out[f"hybrid_x{k + 1}"] = x[idx].tolist()
    out["hybrid_hist"] = hist
    with open(os.path.join(HERE, "cfg2_hybrid_samples.json"), "w") as fh:
        json.dump(out, fh, indent=0)
    print(f"done {time.time() - t0:.0f} s", flush=True)


def main():
    t0 = time.time()
    p = config("cfg2")
    H = amg.setup(p.A)
    print(f"hierarchy {time.time() - t0:.0f} s", flush=True)
    if "--hybrid" in sys.argv:
        return hybrid(p, H, int(sys.argv[sys.argv.index("--hybrid") + 1]), t0)
    comps = composite.build_all(H, p.part, p.nparts, p.eta)
    print(f"composite grids {time.time() - t0:.0f} s", flush=True)
    co = cycles.CoarseSolver(H.A[H.L])
    rng = np.random.default_rng(123)
    idx = np.sort(rng.choice(p.n, 2000, replace=False))
    out = {"what": __doc__.strip().splitlines()[0], "workload": "cfg2 128^3 4x4x4 eta 1 n_fac 2 seed 0",
           "levels": [int(A.shape[0]) for A in H.A], "nnz": [int(A.nnz) for A in H.A], "idx": idx.tolist()}
    x = np.zeros(p.n)
    hist = [float(np.linalg.norm(p.b))]
    for k in range(2):
        x = cycles.amgdd_iteration(H, comps, p.b, x, p.n_fac, co)
        hist.append(float(np.linalg.norm(p.b - p.A @ x)))
        out[f"amgdd_x{k + 1}"] = x[idx].tolist()
    out["amgdd_hist"] = hist
    x = np.zeros(p.n)
    hist = [float(np.linalg.norm(p.b))]
    for k in range(2):
        x = cycles.vcycle(H, x, p.b, coarse=co)
        hist.append(float(np.linalg.norm(p.b - p.A @ x)))
        out[f"vcycle_x{k + 1}"] = x[idx].tolist()
    out["vcycle_hist"] = hist
    with open(os.path.join(HERE, "cfg2_samples.json"), "w") as fh:
        json.dump(out, fh, indent=0)
    print(f"done {time.time() - t0:.0f} s", flush=True)


if __name__ == "__main__":
    main()
