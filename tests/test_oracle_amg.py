"""Pins for the oracle's AMG setup (strength, RS, direct interpolation,
Galerkin) against hand-worked examples, brute force and invariants."""

import json
import os

import numpy as np
import pytest
from scipy import sparse

from oracle import amg
from synth import make_problem

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _gold(name):
    with open(os.path.join(GOLD, name)) as fh:
        return json.load(fh)


def test_golden_direct_interp_worked_example():
    g = _gold("direct_interp_5pt.json")
    A = sparse.csr_matrix(np.array(g["A"]))
    S = amg.strength(A, 0.25)
    rows = [sorted(S.indices[S.indptr[i]:S.indptr[i + 1]].tolist()) for i in range(5)]
    assert rows == g["S"]
    cf = amg.rs_first_pass(S)
    assert cf.tolist() == g["cf"]
    P = amg.direct_interpolation(A, S, cf).toarray()
    expect = np.array(g["P_num"], dtype=float) / np.array(g["P_den"], dtype=float)
    np.testing.assert_allclose(P, expect, rtol=1e-15, atol=0)


def test_golden_laplace1d_two_level():
    g = _gold("laplace1d_two_level.json")
    n = g["n"]
    A = sparse.diags([-np.ones(n - 1), 2 * np.ones(n), -np.ones(n - 1)], [-1, 0, 1]).tocsr()
    S = amg.strength(A)
    cf = amg.rs_first_pass(S)
    assert cf.tolist() == g["cf"]
    P = amg.direct_interpolation(A, S, cf)
    np.testing.assert_allclose(P.toarray(), np.array(g["P"]), rtol=0, atol=1e-15)
    A1 = amg.galerkin(A, P)
    np.testing.assert_allclose(A1.toarray(), np.array(g["A1"]), rtol=0, atol=1e-15)


def _brute_rs(S):
    """RS first pass with the measure recomputed from its definition at every
    step: lambda_i = |S^T_i cap U| + 2 |S^T_i cap F|, argmax with the smallest
    index on ties (O(n^2), tiny graphs only)."""
    S = S.toarray() != 0
    n = S.shape[0]
    ST = S.T
    st = np.zeros(n, dtype=int)
    iso = ~S.any(1) & ~S.any(0)
    st[iso] = -1
    while (st == 0).any():
        U = st == 0
        F = st == -1
        # S^T_i = {j : i in S_j} = row i of S^T = column i of S
        lam = (S[:, :] & U[:, None]).sum(0) + 2 * (S & F[:, None]).sum(0)
        lam = np.where(U, lam, -1)
        i = int(np.argmax(lam))
        if lam[i] == 0:
            for u in np.nonzero(U)[0]:
                st[u] = -1 if (S[u] & (st == 1)).any() else 1
            break
        st[i] = 1
        for j in np.nonzero(S[:, i] & (st == 0))[0]:
            st[j] = -1
    return st


@pytest.mark.parametrize("dims,k_seed", [((7, 6), None), ((9, 9), 3), ((5, 4, 4), None), ((5, 5, 5), 11)])
def test_rs_matches_bruteforce(dims, k_seed):
    from synth import grf
    k = None if k_seed is None else np.exp(grf(dims, 1.0, 2.0, k_seed))
    p = make_problem(dims, [1] * len(dims), k=k)
    H = amg.setup(p.A, max_coarse=4)
    for l in range(H.L):
        S = amg.strength(H.A[l])
        assert amg.rs_first_pass(S).tolist() == _brute_rs(S).tolist(), f"level {l}"


def test_laplacian_level0_all_neighbours_strong():
    p = make_problem((8, 8, 8), (1, 1, 1))
    S = amg.strength(p.A)
    off = p.A.copy()
    off.setdiag(0)
    off.eliminate_zeros()
    assert (S != (off != 0)).nnz == 0


@pytest.mark.parametrize("dims,k_seed", [((32, 32), None), ((24, 24), 5), ((12, 12, 12), None), ((10, 10, 10), 7)])
def test_hierarchy_invariants(dims, k_seed):
    from synth import grf
    k = None if k_seed is None else np.exp(grf(dims, 1.0, 4.0, k_seed))
    p = make_problem(dims, [1] * len(dims), k=k)
    H = amg.setup(p.A)
    assert H.A[-1].shape[0] <= 16
    for l in range(H.L):
        A, P, cf = H.A[l], H.P[l], H.cf[l]
        S = amg.strength(A)
        # every F-point with a strong connection has a strong C-neighbour
        for i in np.nonzero(cf == amg.F_PT)[0]:
            si = S.indices[S.indptr[i]:S.indptr[i + 1]]
            if si.size:
                assert (cf[si] == amg.C_PT).any()
        # injection at C-points
        Pd = P.tocsr()
        ci = np.nonzero(cf == amg.C_PT)[0]
        assert np.all(np.diff(Pd.indptr)[ci] == 1)
        assert np.all(Pd.data[Pd.indptr[ci]] == 1.0)
        # zero-row-sum F rows interpolate constants exactly
        rs = np.asarray(A.sum(1)).ravel()
        fi = np.nonzero((cf == amg.F_PT) & (np.abs(rs) < 1e-12 * A.diagonal()) & (np.diff(Pd.indptr) > 0))[0]
        ws = np.asarray(Pd.sum(1)).ravel()[fi]
        np.testing.assert_allclose(ws, 1.0, rtol=1e-13)
        # Galerkin values against a dense product, pattern contains the support
        Ac = H.A[l + 1]
        dense = P.toarray().T @ A.toarray() @ P.toarray()
        np.testing.assert_allclose(Ac.toarray(), dense, rtol=0, atol=1e-12 * np.abs(dense).max())
        pat = np.zeros(dense.shape, dtype=bool)
        pat[np.repeat(np.arange(Ac.shape[0]), np.diff(Ac.indptr)), Ac.indices] = True
        assert not np.any((np.abs(dense) > 1e-14 * np.abs(dense).max()) & ~pat)
        # symmetric, positive definite
        Ad = Ac.toarray()
        np.testing.assert_allclose(Ad, Ad.T, rtol=0, atol=1e-13 * np.abs(Ad).max())
        np.linalg.cholesky(Ad)


def test_galerkin_keeps_symbolic_zero():
    # A P has an exact cancellation that a numerical product would drop
    A = sparse.csr_matrix(np.array([[2.0, -1.0, -1.0], [-1.0, 2.0, 0.0], [-1.0, 0.0, 2.0]]))
    P = sparse.csr_matrix(np.array([[1.0, 1.0], [1.0, 0.0], [0.0, 1.0]]))
    G = amg.galerkin(A, P)
    assert G.nnz == 4
    np.testing.assert_allclose(G.toarray(), P.toarray().T @ A.toarray() @ P.toarray(), atol=1e-15)


def test_seq_row_sum_order():
    # 1 + 1e-16 + 1e-16 sequentially is 1 (each add rounds away); pairwise would give 1 + 2e-16
    indptr = np.array([0, 3])
    vals = np.array([1.0, 1e-16, 1e-16])
    assert amg.seq_row_sum(indptr, vals)[0] == 1.0
