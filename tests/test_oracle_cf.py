"""Pins for the oracle's CF-ordered l1-Jacobi relaxation (relax="cf"):
closed-form error propagation of one sweep, symmetry of the V-cycle as an
operator (the upsweep order must be the reverse of the downsweep's), the
equivalence principle of AlgFAC under CF relaxation, and the one-subdomain
and hybrid reductions."""

import numpy as np
import pytest
import scipy.linalg as sla

from oracle import amg, composite, cycles
from oracle.amg import C_PT, F_PT
from synth import grf, make_problem


def _setup(dims, parts, eta=1, k_seed=None):
    k = None if k_seed is None else np.exp(grf(dims, 1.0, 4.0, k_seed))
    p = make_problem(dims, parts, eta=eta, k=k)
    H = amg.setup(p.A)
    return p, H


@pytest.mark.parametrize("order", [cycles.C_FIRST, cycles.F_FIRST])
def test_cf_sweep_error_propagation(order):
    # error after one sweep = (I - S_2 D^-1 A)(I - S_1 D^-1 A) e, with S_k the
    # diagonal selector of the k-th class of the order: dense matrix algebra,
    # independent of the sweep's code
    p, H = _setup((14, 12), (1, 1), k_seed=4)
    A = H.A[0].toarray()
    d = np.abs(A).sum(axis=1)
    cls = H.cf[0]
    xs = sla.solve(A, p.b)
    u = np.random.default_rng(1).standard_normal(p.n)
    un = cycles.smooth(H.A[0], d, u, p.b, cls=cls, order=order)
    E = np.eye(p.n)
    for c in order:
        E = (np.eye(p.n) - np.diag((cls == c) / d) @ A) @ E
    np.testing.assert_allclose(xs - un, E @ (xs - u), rtol=0, atol=1e-12 * np.abs(xs - u).max())
    assert set(np.unique(cls)) == {C_PT, F_PT}


@pytest.mark.parametrize("relax", ["l1", "cf"])
def test_vcycle_is_a_symmetric_operator(relax):
    # for symmetric A the V(1,1) cycle from zero, f -> u, is a symmetric
    # matrix exactly when the post-smoother is the adjoint of the
    # pre-smoother: CF order down, FC order up
    p, H = _setup((11, 10), (1, 1), k_seed=2)
    B = np.column_stack([cycles.vcycle(H, np.zeros(p.n), e, relax=relax) for e in np.eye(p.n)])
    assert np.abs(B - B.T).max() <= 1e-12 * np.abs(B).max()
    if relax == "cf":
        # the helper reproduces the cycle, and a wrong upsweep order (C first
        # on both sweeps) breaks the symmetry
        Bc = np.column_stack([_vcycle_orders(H, e, cycles.C_FIRST, cycles.F_FIRST) for e in np.eye(p.n)])
        assert np.abs(Bc - B).max() <= 1e-13 * np.abs(B).max()
        Bw = np.column_stack([_vcycle_orders(H, e, cycles.C_FIRST, cycles.C_FIRST) for e in np.eye(p.n)])
        assert np.abs(Bw - Bw.T).max() > 1e-6 * np.abs(Bw).max()


def _vcycle_orders(H, f0, down, up):
    """V(1,1) from zero with explicit sweep orders (test helper)."""
    L = H.L
    co = cycles.CoarseSolver(H.A[L])
    d = [H.l1_diag(l) for l in range(L)]
    u = [None] * (L + 1)
    f = [None] * (L + 1)
    u[0] = np.zeros(H.A[0].shape[0])
    f[0] = f0
    for l in range(L):
        u[l] = cycles.smooth(H.A[l], d[l], u[l], f[l], cls=H.cf[l], order=down)
        f[l + 1] = H.R[l] @ (f[l] - H.A[l] @ u[l])
        u[l + 1] = np.zeros(H.A[l + 1].shape[0])
    u[L] = co(f[L])
    for l in range(L - 1, -1, -1):
        u[l] = u[l] + H.P[l] @ u[l + 1]
        u[l] = cycles.smooth(H.A[l], d[l], u[l], f[l], cls=H.cf[l], order=up)
    return u[0]


@pytest.mark.parametrize("dims,parts,eta,k_seed,n_fac", [((32, 32), (2, 2), 1, None, 1), ((30, 26), (3, 2), 2, 5, 3),
                                                         ((10, 10, 10), (2, 2, 2), 1, 7, 2)])
def test_cf_algfac_equals_masked_global_cycle(dims, parts, eta, k_seed, n_fac):
    # guiding principle of Section 4 under CF relaxation: both half-sweeps
    # act on real points only and see correct values at every neighbour
    p, H = _setup(dims, parts, eta, k_seed)
    comps = composite.build_all(H, p.part, p.nparts, eta)
    r0 = np.random.default_rng(11).standard_normal(p.n)
    rs = cycles.restrict_all(H, r0)
    coarse = cycles.CoarseSolver(H.A[H.L])
    for q, cg in enumerate(comps):
        D, _ = composite.composite_sets(H, p.part, q, eta)
        f = [rs[l][lv.gid[: lv.n_real]] for l, lv in enumerate(cg.levels)]
        cls = [H.cf[l][lv.gid[: lv.n_real]] for l, lv in enumerate(cg.levels[:-1])]
        u_fac, _ = cycles.algfac(cg, f, n_fac, coarse, cls=cls, relax="cf")
        u_mask = cycles.masked_vcycle(H, D, np.zeros(p.n), r0, n_fac, coarse, relax="cf")
        u_nat = cycles.masked_vcycle(H, D, np.zeros(p.n), r0, n_fac, coarse)
        assert np.abs(u_mask[0] - u_nat[0]).max() > 1e-6 * np.abs(u_nat[0]).max()
        for l, lv in enumerate(cg.levels):
            scale = np.abs(u_mask[l]).max()
            np.testing.assert_allclose(u_fac[l], u_mask[l][lv.gid], rtol=0, atol=1e-13 * scale)


@pytest.mark.parametrize("n_fac", [1, 2])
def test_cf_one_subdomain_is_vcycles(n_fac):
    p, H = _setup((20, 20), (1, 1), k_seed=2)
    comps = composite.build_all(H, p.part, 1, 1)
    x = np.random.default_rng(0).standard_normal(p.n)
    xdd = cycles.amgdd_iteration(H, comps, p.b, x, n_fac, relax="cf")
    r = p.b - p.A @ x
    e = np.zeros(p.n)
    for _ in range(n_fac):
        e = cycles.vcycle(H, e, r, relax="cf")
    np.testing.assert_allclose(xdd, x + e, rtol=0, atol=1e-13 * np.abs(x + e).max())


def test_cf_hybrid_reductions_and_convergence():
    p, H = _setup((24, 24), (1, 1))
    lt, Hs, comps = cycles.hybrid_setup(H, p.part, p.nparts, 1, 2)
    x = np.random.default_rng(1).standard_normal(p.n)
    xh = x + cycles.hybrid_vcycle(H, Hs, comps, np.zeros(p.n), p.b - p.A @ x, lt, 1, relax="cf")
    xv = cycles.vcycle(H, x, p.b, relax="cf")
    np.testing.assert_allclose(xh, xv, rtol=0, atol=1e-13 * np.abs(xv).max())
    p, H = _setup((12, 12, 12), (2, 2, 2), k_seed=3)
    comps = composite.build_all(H, p.part, p.nparts, 1)
    xs = sla.solve(p.A.toarray(), p.b)
    for fn in (lambda: cycles.amgdd_solve(H, comps, p.b, np.zeros(p.n), 2, rtol=1e-13, maxit=100, relax="cf"),
               lambda: cycles.vcycle_solve(H, p.b, np.zeros(p.n), rtol=1e-13, maxit=200, relax="cf")):
        x, hist = fn()
        assert hist[-1] <= 1e-13 * hist[0]
        assert np.linalg.norm(x - xs) <= 1e-10 * np.linalg.norm(xs)
