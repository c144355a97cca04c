"""Oracle: the AMG-DD iteration with its loop over subdomains spread over
worker processes, plain FP64 (or the float32 emulation).

TEST INFRASTRUCTURE ONLY (see oracle/amg.py).

Algorithm 2 runs the AlgFAC cycles of every subdomain independently of every
other subdomain (Section 3: the local cycles need no communication), so the
loop over subdomains may run in any order or all at once.  SubdomainPool runs
cycles.algfac for every subdomain in forked worker processes, then patches
the owned corrections exactly as cycles.amgdd_iteration does: same operands,
same per-subdomain arithmetic, so the result is bitwise the same (pinned in
tests/test_oracle_parallel.py).  The fine residual, the restriction chain and
the patch stay in the calling process."""

from __future__ import annotations

import multiprocessing as mp
from typing import Optional, Sequence

import numpy as np

from . import cycles
from .amg import Hierarchy
from .composite import CompositeGrid

# state of the forked workers (inherited at fork time, never pickled)
_STATE = {}


def _job(args):
    q, f, dtype = args
    cg = _STATE["comps"][q]
    cls = _STATE["cls"][q]
    u, _ = cycles.algfac(cg, f, _STATE["n_fac"], _STATE["coarse"], dtype=dtype, cls=cls, relax=_STATE["relax"])
    return u[0][cg.owned_local].astype(np.float64)


class SubdomainPool:
    """Forked worker processes holding the composite grids of one problem."""

    def __init__(self, H: Hierarchy, comps: Sequence[CompositeGrid], n_fac: int, workers: int,
                 coarse: Optional[cycles.CoarseSolver] = None, relax: str = "l1"):
        self.H = H
        self.comps = list(comps)
        self.workers = max(1, int(workers))
        cls = [[H.cf[l][lev.gid[: lev.n_real]] for l, lev in enumerate(cg.levels[:-1])] for cg in self.comps]
        _STATE.update(comps=self.comps, cls=cls, n_fac=int(n_fac), relax=relax,
                      coarse=coarse or cycles.CoarseSolver(H.A[H.L]))
        self.pool = mp.get_context("fork").Pool(self.workers)

    def iteration(self, b: np.ndarray, x: np.ndarray, dtype=np.float64) -> np.ndarray:
        """One AMG-DD iteration, the same result as cycles.amgdd_iteration."""
        H = self.H
        r = b - H.A[0] @ x
        rs = cycles.restrict_all(H, r, dtype)
        jobs = [(q, [rs[l][lev.gid[: lev.n_real]] for l, lev in enumerate(cg.levels)], dtype)
                for q, cg in enumerate(self.comps)]
        us = self.pool.map(_job, jobs, chunksize=1)
        xn = np.array(x, dtype=np.float64)
        for cg, u in zip(self.comps, us):
            xn[cg.owned_gid] += u
        return xn

    def close(self):
        if self.pool is not None:
            self.pool.close()
            self.pool.join()
            self.pool = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()
