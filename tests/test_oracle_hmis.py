"""Pins for the oracle's "best practices" AMG components: SplitMix64 (the
published reference outputs), PMIS on a hand-worked chain, HMIS reducing to
the RS first pass on one subdomain, extended+i interpolation on a hand-worked
1D case (exact linear interpolation across an F-F pair) and preserving
constants on every zero-row-sum row, and whole hierarchies that solve."""

import numpy as np
import pytest
import scipy.linalg as sla
from scipy import sparse

from oracle import amg, composite, cycles
from oracle.amg import C_PT, F_PT
from synth import config, grf, make_problem


def test_splitmix64_reference_outputs():
    # the generator's published outputs: state 0, and the first three draws
    # from state 1234567 (the state advances by the golden gamma per draw)
    assert amg.splitmix64(0) == 0xE220A8397B1DCDAF
    g = 0x9E3779B97F4A7C15
    outs = [amg.splitmix64((1234567 + k * g) % 2**64) for k in range(3)]
    assert outs == [6457827717110365317, 3203168211198807973, 9817491932198370423]
    r = amg.pmis_random(3, 1000)
    assert r.min() >= 0.0 and r.max() < 1.0 and len(np.unique(r)) == 1000


def _lap1d(n):
    return sparse.diags([-np.ones(n - 1), 2 * np.ones(n), -np.ones(n - 1)], [-1, 0, 1]).tocsr()


def test_pmis_hand_worked_chain():
    # 1D Laplacian on 5 points: every neighbour is strong, |S^T| = [1,2,2,2,1];
    # with r = [.1,.5,.3,.9,.2] the measures are [1.1,2.5,2.3,2.9,1.2]: points
    # 1 and 3 beat all their neighbours, become C, and 0, 2, 4 depend on them
    S = amg.strength(_lap1d(5))
    cf = amg.pmis(S, np.array([0.1, 0.5, 0.3, 0.9, 0.2]))
    assert cf.tolist() == [F_PT, C_PT, F_PT, C_PT, F_PT]
    # a point that influences nobody is F from the start
    S2 = sparse.csr_matrix(np.array([[0, 1, 0], [0, 0, 0], [0, 1, 0]], dtype=float))
    cf2 = amg.pmis(S2, np.array([0.5, 0.1, 0.9]))
    assert cf2.tolist() == [F_PT, C_PT, F_PT]


@pytest.mark.parametrize("dims,parts", [((24, 24), (3, 2)), ((10, 10, 10), (2, 2, 2))])
def test_pmis_and_hmis_invariants(dims, parts):
    p = make_problem(dims, parts, k=np.exp(grf(dims, 1.0, 4.0, 5)))
    S = amg.strength(p.A)
    ST = sparse.csr_matrix(S.T)
    cnt = np.diff(ST.indptr)
    r = amg.pmis_random(0, p.n)
    for cf in (amg.pmis(S, r), amg.hmis(S, p.part, r)):
        assert set(np.unique(cf)) <= {C_PT, F_PT}
        # every F-point influencing some point strongly depends on a C-point
        for i in np.nonzero(cf == F_PT)[0]:
            if cnt[i] > 0:
                assert (cf[S.indices[S.indptr[i]:S.indptr[i + 1]]] == C_PT).any(), i
    # plain PMIS: the point of largest measure wins the first round
    assert amg.pmis(S, r)[int(np.argmax(cnt + r))] == C_PT


def test_hmis_one_subdomain_is_rs_first_pass():
    # with one subdomain every RS C-point is interior; when every RS F-point
    # strongly depends on an RS C-point, PMIS has nothing left to decide
    p = make_problem((30, 28), (1, 1), k=np.exp(grf((30, 28), 1.0, 4.0, 2)))
    S = amg.strength(p.A)
    rs = amg.rs_first_pass(S)
    for i in np.nonzero(rs == F_PT)[0]:
        assert (rs[S.indices[S.indptr[i]:S.indptr[i + 1]]] == C_PT).any()
    assert np.array_equal(amg.hmis(S, p.part, amg.pmis_random(0, p.n)), rs)


def test_ext_i_hand_worked_1d():
    # A = tridiag(-1, 2, -1), C F F C: point 1 reaches C-point 3 through its
    # strong F-neighbour 2 (d_2 = a_21 + a_23 = -2):
    #   num_10 = -1, num_13 = (-1)(-1)/(-2) = -1/2, at_11 = 2 - 1/2 = 3/2
    #   -> w_10 = 2/3, w_13 = 1/3: linear interpolation, exact in 1D
    A = _lap1d(4)
    S = amg.strength(A)
    P = amg.ext_i_interpolation(A, S, np.array([C_PT, F_PT, F_PT, C_PT], dtype=np.int8)).toarray()
    np.testing.assert_allclose(P, [[1, 0], [2 / 3, 1 / 3], [1 / 3, 2 / 3], [0, 1]], rtol=1e-15)


@pytest.mark.parametrize("name", ["lap3d", "var2d", "aniso"])
def test_ext_i_preserves_constants_on_zero_row_sums(name):
    if name == "lap3d":
        A, part = make_problem((12, 12, 12), (2, 2, 2)).A, None
    elif name == "var2d":
        A = make_problem((30, 30), (2, 2), k=np.exp(grf((30, 30), 1.0, 4.0, 7))).A
    else:
        A = config("p2", scale=30).A
    S = amg.strength(A)
    cf = amg.pmis(S, amg.pmis_random(0, A.shape[0]))
    P = amg.ext_i_interpolation(A, S, cf)
    rowsum_A = np.asarray(A.sum(axis=1)).ravel()
    scale = np.abs(A).sum(axis=1).A.ravel()
    zero = np.abs(rowsum_A) <= 1e-14 * scale
    nz = np.diff(P.indptr) > 0
    ones = np.asarray(P.sum(axis=1)).ravel()
    sel = zero & nz
    assert sel.sum() > 0.3 * A.shape[0]
    np.testing.assert_allclose(ones[sel], 1.0, rtol=0, atol=1e-12)
    # C rows inject
    assert np.all(np.diff(P.indptr)[cf == C_PT] == 1)


def test_ext_i_without_f_neighbours_is_direct():
    # F-points whose strong neighbours are all C and that have no weak
    # neighbours: w_ij = -a_ij / a_ii, the direct weights with alpha = 1
    A = _lap1d(5)
    S = amg.strength(A)
    cf = np.array([C_PT, F_PT, C_PT, F_PT, C_PT], dtype=np.int8)
    Pe = amg.ext_i_interpolation(A, S, cf).toarray()
    Pd = amg.direct_interpolation(A, S, cf).toarray()
    np.testing.assert_array_equal(Pe, Pd)


@pytest.mark.parametrize("coarsen,interp", [("hmis", "ext+i"), ("hmis", "direct"), ("rs", "ext+i")])
def test_best_practice_hierarchies_solve(coarsen, interp):
    p = make_problem((10, 10, 10), (2, 2, 2), eta=1)
    H = amg.setup(p.A, coarsen=coarsen, interp=interp, part=p.part)
    assert H.L >= 2
    comps = composite.build_all(H, p.part, p.nparts, 1)
    xs = sla.solve(p.A.toarray(), p.b)
    x, hist = cycles.amgdd_solve(H, comps, p.b, np.zeros(p.n), 2, rtol=1e-12, maxit=100)
    assert np.linalg.norm(x - xs) <= 1e-9 * np.linalg.norm(xs)
    # Galerkin coarse operators of ext+i / HMIS hierarchies stay symmetric
    for A in H.A:
        assert abs(A - A.T).max() <= 1e-12 * abs(A).max()


def test_truncation_keeps_largest_and_row_sum():
    # |w| order 0.4 (7), 0.3 (9), 0.2 (11), 0.1 (3) kept; the dropped -0.05
    # and 0.05 cancel, so the kept sum already equals the row sum 1
    cols, vals = amg.truncate_row([3, 5, 7, 9, 11, 13], [0.1, -0.05, 0.4, 0.3, 0.2, 0.05], 4)
    assert cols == [3, 7, 9, 11]
    np.testing.assert_allclose(vals, [0.1, 0.4, 0.3, 0.2], rtol=1e-14)
    # dropping 0.2 of a row summing to 1: kept entries scale by 1 / 0.8
    c1, v1 = amg.truncate_row([0, 1, 2], [0.5, 0.3, 0.2], 2)
    assert c1 == [0, 1]
    np.testing.assert_allclose(v1, [0.625, 0.375], rtol=1e-15)
    # ties: the smaller column stays
    c2, v2 = amg.truncate_row([1, 2, 3], [0.5, 0.25, 0.25], 2)
    assert c2 == [1, 2]
    np.testing.assert_allclose(v2, [2 / 3, 1 / 3], rtol=1e-15)
    # short rows are untouched
    assert amg.truncate_row([4, 8], [0.7, 0.3], 4) == ([4, 8], [0.7, 0.3])


def test_truncated_ext_i_rows_and_constants():
    A = make_problem((12, 12, 12), (2, 2, 2)).A
    S = amg.strength(A)
    cf = amg.pmis(S, amg.pmis_random(0, A.shape[0]))
    P0 = amg.ext_i_interpolation(A, S, cf)
    P4 = amg.ext_i_interpolation(A, S, cf, pmax=4)
    assert np.diff(P0.indptr).max() > 4 and np.diff(P4.indptr).max() <= 4
    np.testing.assert_allclose(np.asarray(P4.sum(axis=1)).ravel(), np.asarray(P0.sum(axis=1)).ravel(),
                               rtol=1e-13, atol=1e-15)
