"""The oracle's subdomain-parallel AMG-DD iteration (used for full-size sample
values and the all-cores CPU baseline) is bitwise the serial one."""

import numpy as np
import pytest

from oracle import amg, composite, cycles
from oracle.parallel import SubdomainPool
from synth import grf, make_problem


@pytest.mark.parametrize("relax", ["l1", "cf"])
def test_parallel_iteration_is_bitwise_serial(relax):
    dims = (20, 18, 16)
    p = make_problem(dims, (2, 2, 2), eta=2, n_fac=2, k=np.exp(grf(dims, 1.0, 8.0, 1)))
    H = amg.setup(p.A)
    comps = composite.build_all(H, p.part, p.nparts, p.eta)
    co = cycles.CoarseSolver(H.A[H.L])
    with SubdomainPool(H, comps, p.n_fac, workers=3, coarse=co, relax=relax) as pool:
        for dtype in (np.float64, np.float32):
            x = np.zeros(p.n)
            xs = np.zeros(p.n)
            for _ in range(2):
                x = pool.iteration(p.b, x, dtype=dtype)
                xs = cycles.amgdd_iteration(H, comps, p.b, xs, p.n_fac, co, dtype=dtype, relax=relax)
                assert np.array_equal(x, xs)
