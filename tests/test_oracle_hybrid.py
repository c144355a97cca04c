"""Pins for the oracle's hybrid AMG-DD cycle (Algorithm 3)."""

import numpy as np
import pytest
import scipy.linalg as sla

from oracle import amg, composite, cycles
from synth import grf, make_problem


def _hybrid(p, lt, eta=1):
    H = amg.setup(p.A)
    part = cycles.inherited_partition(H, p.part, lt)
    Hs = cycles.sub_hierarchy(H, lt)
    comps = composite.build_all(Hs, part, p.nparts, eta)
    return H, Hs, comps


def test_inherited_partition_follows_c_points():
    p = make_problem((20, 20), (2, 2))
    H = amg.setup(p.A)
    part1 = cycles.inherited_partition(H, p.part, 1)
    c = np.nonzero(H.cf[0] == 1)[0]
    assert np.array_equal(part1, p.part[c])
    assert part1.size == H.A[1].shape[0]


def test_hybrid_at_level_zero_is_amgdd():
    # lt = 0: no V-cycle levels, the cycle is one AMG-DD cycle on A_0 from zero
    p = make_problem((24, 20), (2, 2), k=np.exp(grf((24, 20), 1.0, 4.0, 1)))
    H, Hs, comps = _hybrid(p, 0)
    x = np.random.default_rng(0).standard_normal(p.n)
    r = p.b - p.A @ x
    e = cycles.hybrid_vcycle(H, Hs, comps, np.zeros(p.n), r, 0, 2)
    ref = cycles.amgdd_iteration(H, composite.build_all(H, p.part, p.nparts, 1), p.b, x, 2) - x
    np.testing.assert_allclose(e, ref, rtol=0, atol=1e-13 * np.abs(ref).max())


@pytest.mark.parametrize("lt", [1, 2])
def test_one_subdomain_hybrid_is_vcycle(lt):
    # one subdomain: the level-lt AMG-DD with one AlgFAC cycle is a V-cycle on
    # the sub-hierarchy, so the hybrid cycle is the plain V(1,1) cycle
    p = make_problem((24, 24), (1, 1))
    H, Hs, comps = _hybrid(p, lt)
    x = np.random.default_rng(1).standard_normal(p.n)
    xh = x + cycles.hybrid_vcycle(H, Hs, comps, np.zeros(p.n), p.b - p.A @ x, lt, 1)
    xv = cycles.vcycle(H, x, p.b)
    np.testing.assert_allclose(xh, xv, rtol=0, atol=1e-13 * np.abs(xv).max())


@pytest.mark.parametrize("dims,parts,lt", [((32, 32), (2, 2), 1), ((12, 12, 12), (2, 2, 2), 2)])
def test_hybrid_converges_to_dense_solution(dims, parts, lt):
    p = make_problem(dims, parts)
    H, Hs, comps = _hybrid(p, lt)
    xs = sla.solve(p.A.toarray(), p.b)
    x = np.zeros(p.n)
    r0 = np.linalg.norm(p.b)
    for _ in range(200):
        x = x + cycles.hybrid_vcycle(H, Hs, comps, np.zeros(p.n), p.b - p.A @ x, lt, 2)
        if np.linalg.norm(p.b - p.A @ x) <= 1e-13 * r0:
            break
    assert np.linalg.norm(x - xs) <= 1e-10 * np.linalg.norm(xs)


def test_sub_hierarchy_is_the_hierarchy_of_the_coarse_matrix():
    # classical coarsening depends on the matrix alone: setting up A_lt from
    # scratch reproduces levels lt.. of the fine hierarchy exactly
    p = make_problem((28, 24), (2, 2), k=np.exp(grf((28, 24), 1.0, 4.0, 3)))
    H = amg.setup(p.A)
    for lt in (1, 2):
        Hs = cycles.sub_hierarchy(H, lt)
        H2 = amg.setup(H.A[lt])
        assert H2.L == Hs.L
        for a, b in zip(H2.A, Hs.A):
            assert (a != b).nnz == 0
        for a, b in zip(H2.cf, Hs.cf):
            assert np.array_equal(a, b)


def test_hybrid_at_coarsest_level_is_vcycle():
    # lt = L: the level-L AMG-DD problem has one level, its composite grids
    # hold all of it and AlgFAC is the direct solve, for any subdomain count
    p = make_problem((24, 24), (3, 2))
    H = amg.setup(p.A)
    lt, Hs, comps = cycles.hybrid_setup(H, p.part, p.nparts, 1, 99)
    assert lt == H.L
    x = np.random.default_rng(2).standard_normal(p.n)
    xh = x + cycles.hybrid_vcycle(H, Hs, comps, np.zeros(p.n), p.b - p.A @ x, lt, 2)
    xv = cycles.vcycle(H, x, p.b)
    np.testing.assert_allclose(xh, xv, rtol=0, atol=1e-12 * np.abs(xv).max())


def test_empty_subdomains_contribute_nothing():
    # 64 subdomains of 2x2 points leave half of them without points on level
    # 2; their composite grids patch nothing, so dropping them leaves the
    # cycle unchanged
    p = make_problem((16, 16), (8, 8))
    H = amg.setup(p.A)
    lt = 2
    assert H.L > lt
    part = cycles.inherited_partition(H, p.part, lt)
    Hs = cycles.sub_hierarchy(H, lt)
    comps = composite.build_all(Hs, part, p.nparts, 1)
    empty = [q for q in range(p.nparts) if not np.any(part == q)]
    assert empty
    kept = [c for q, c in enumerate(comps) if q not in empty]
    r = p.b - p.A @ np.random.default_rng(3).standard_normal(p.n)
    e1 = cycles.hybrid_vcycle(H, Hs, comps, np.zeros(p.n), r, lt, 2)
    e2 = cycles.hybrid_vcycle(H, Hs, kept, np.zeros(p.n), r, lt, 2)
    assert np.array_equal(e1, e2)


def test_hybrid_solve_history():
    p = make_problem((32, 32), (2, 2))
    H = amg.setup(p.A)
    lt, Hs, comps = cycles.hybrid_setup(H, p.part, p.nparts, 1, 1)
    x, hist = cycles.hybrid_solve(H, Hs, comps, lt, p.b, np.zeros(p.n), 2, rtol=1e-9, maxit=60)
    assert hist[-1] <= 1e-9 * hist[0]
    assert np.linalg.norm(p.b - p.A @ x) == pytest.approx(hist[-1], rel=1e-12)
