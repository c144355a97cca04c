"""Pins of the oracle's adjoint AMG-DD for a non-symmetric operator: AMG-DD
(Algorithm 2) on the forward hierarchy transposed (oracle.adjoint.
transposed_hierarchy).  Test operator: diffusion plus first-order upwind
convection, a non-symmetric M-matrix with the symmetric 5/7-point pattern.

What fixes the result independently of the code under test:
* Section 2's Galerkin relation A_{l+1} = R_l A_l P_l with R_l = P_l^T gives
  A_{l+1}^T = R_l A_l^T P_l: the Galerkin product of the transposed level
  operator, formed by the oracle's own Galerkin routine, must equal the
  transpose of the forward coarse operator (up to summation order);
* l1-Jacobi on A_l^T divides by column sums of |A_l| (dense computation);
* composite sets depend only on the undirected graph of A_l (Section 3), so
  the transposed hierarchy's sets equal the forward ones bit for bit;
* the converged adjoint equals the dense solve of A^T lambda = g;
* special case: one subdomain makes an AMG-DD iteration n_fac V(1,1) cycles
  on the transposed hierarchy (Section 4 guiding principle);
* AlgFAC equals the masked full-grid cycle on the transposed hierarchy."""

import numpy as np
import pytest

from oracle import adjoint, amg, composite, cycles
from synth import convection_diffusion_problem, grf


def _prob(dims=(18, 16), parts=(2, 2), vel=(1.0, 0.5), eta=1, k_seed=None):
    k = None if k_seed is None else np.exp(grf(dims, 0.5, 4.0, k_seed))
    return convection_diffusion_problem(dims, parts, velocity=vel, eta=eta, n_fac=2, k=k)


CASES = [((18, 16), (2, 2), (1.0, 0.5), None), ((9, 8, 7), (2, 2, 1), (0.7, -0.4, 0.3), 3),
         ((24, 20), (3, 2), (-1.5, 0.8), 5)]


@pytest.mark.parametrize("dims,parts,vel,k_seed", CASES)
def test_transposed_levels_are_the_galerkin_hierarchy_of_AT(dims, parts, vel, k_seed):
    p = _prob(dims, parts, vel, k_seed=k_seed)
    assert abs(p.A - p.A.T).max() > 0.1  # genuinely non-symmetric
    H = amg.setup(p.A)
    HT = adjoint.transposed_hierarchy(H)
    assert H.L >= 2
    for l in range(H.L):
        G = amg.galerkin(HT.A[l], H.P[l]).toarray()
        ref = H.A[l + 1].toarray().T
        assert np.abs(G - ref).max() <= 1e-14 * np.abs(ref).max(), f"level {l + 1}"
        assert np.array_equal(HT.A[l + 1].toarray(), ref)


@pytest.mark.parametrize("dims,parts,vel,k_seed", CASES)
def test_transposed_l1_diagonal_is_column_sums(dims, parts, vel, k_seed):
    p = _prob(dims, parts, vel, k_seed=k_seed)
    H = amg.setup(p.A)
    HT = adjoint.transposed_hierarchy(H)
    for l in range(H.L + 1):
        col = np.abs(H.A[l].toarray()).sum(axis=0)
        np.testing.assert_allclose(HT.l1_diag(l), col, rtol=1e-15, atol=0)
        assert np.abs(HT.l1_diag(l) - H.l1_diag(l)).max() > 0 or l == H.L


@pytest.mark.parametrize("dims,parts,vel,k_seed", CASES)
def test_transposed_composite_sets_are_the_forward_ones(dims, parts, vel, k_seed):
    p = _prob(dims, parts, vel, k_seed=k_seed)
    H = amg.setup(p.A)
    HT = adjoint.transposed_hierarchy(H)
    for q in range(p.nparts):
        D, Db = composite.composite_sets(H, p.part, q, p.eta)
        DT, DbT = composite.composite_sets(HT, p.part, q, p.eta)
        for l in range(H.L + 1):
            assert np.array_equal(D[l], DT[l]) and np.array_equal(Db[l], DbT[l])


@pytest.mark.parametrize("dims,parts,vel,k_seed", CASES)
def test_adjoint_amgdd_converges_to_the_dense_adjoint(dims, parts, vel, k_seed):
    p = _prob(dims, parts, vel, k_seed=k_seed)
    H = amg.setup(p.A)
    HT = adjoint.transposed_hierarchy(H)
    comps = composite.build_all(HT, p.part, p.nparts, p.eta)
    g = np.random.default_rng(7).uniform(-1, 1, p.n)
    lam, hist = cycles.amgdd_solve(HT, comps, g, np.zeros(p.n), n_fac=2, rtol=1e-13, maxit=200)
    ref = adjoint.dense_adjoint(p.A, g)
    assert np.linalg.norm(lam - ref) <= 1e-10 * np.linalg.norm(ref)
    # the forward solve on the same hierarchy does not give the adjoint
    comps_f = composite.build_all(H, p.part, p.nparts, p.eta)
    x, _ = cycles.amgdd_solve(H, comps_f, g, np.zeros(p.n), n_fac=2, rtol=1e-13, maxit=200)
    assert np.linalg.norm(x - ref) > 1e-3 * np.linalg.norm(ref)


@pytest.mark.parametrize("n_fac", [1, 2])
def test_adjoint_one_subdomain_is_transposed_vcycles(n_fac):
    p = convection_diffusion_problem((20, 18), (1, 1), velocity=(1.2, -0.6), eta=1)
    H = amg.setup(p.A)
    HT = adjoint.transposed_hierarchy(H)
    comps = composite.build_all(HT, p.part, 1, 1)
    rng = np.random.default_rng(2)
    lam = rng.standard_normal(p.n)
    g = rng.standard_normal(p.n)
    ldd = cycles.amgdd_iteration(HT, comps, g, lam, n_fac)
    r = g - p.A.T @ lam
    e = np.zeros(p.n)
    for _ in range(n_fac):
        e = cycles.vcycle(HT, e, r)
    np.testing.assert_allclose(ldd, lam + e, rtol=0, atol=1e-13 * np.abs(lam + e).max())


def test_transposed_algfac_equals_masked_global_cycle():
    p = _prob((26, 22), (2, 2), (1.0, 0.7), eta=2, k_seed=4)
    H = amg.setup(p.A)
    HT = adjoint.transposed_hierarchy(H)
    comps = composite.build_all(HT, p.part, p.nparts, p.eta)
    rng = np.random.default_rng(5)
    r0 = rng.standard_normal(p.n)
    rs = cycles.restrict_all(HT, r0)
    coarse = cycles.CoarseSolver(HT.A[HT.L])
    for q, cg in enumerate(comps):
        D, _ = composite.composite_sets(HT, p.part, q, p.eta)
        assert all(lv.omissions == 0 for lv in cg.levels[:-1])
        f = [rs[l][lv.gid[: lv.n_real]] for l, lv in enumerate(cg.levels)]
        u_fac, _ = cycles.algfac(cg, f, 2, coarse)
        u_mask = cycles.masked_vcycle(HT, D, np.zeros(p.n), r0, 2, coarse)
        for l, lv in enumerate(cg.levels):
            scale = np.abs(u_mask[l]).max()
            np.testing.assert_allclose(u_fac[l], u_mask[l][lv.gid], rtol=0, atol=1e-13 * scale)
