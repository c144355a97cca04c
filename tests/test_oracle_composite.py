"""Pins for the oracle's composite grids: closed-form level-0 sets (the L1
ball of radius eta around a block, clipped to the domain), all-pairs BFS on
tiny grids, monotonicity and the degenerate cases."""

import numpy as np
import pytest

from oracle import amg, composite
from synth import make_problem


def l1_ball_counts(dims, parts, eta):
    """Closed form: |D_0^p| and |Dbar_0^p| per block.  A grid point's L1
    distance to an axis-aligned box is sum_a max(0, lo_a - x_a, x_a - hi_a);
    D_0 is distance <= eta, Dbar_0 is distance <= eta + 1 (the 5/7-point
    stencil graph distance on a grid equals the L1 distance).  Counted from
    per-axis distance histograms (their convolution is the histogram of the
    total distance)."""
    dims = list(dims)
    nd = len(dims)
    out_d, out_db = [], []
    for bid in range(int(np.prod(parts))):
        r = bid
        hist = np.array([1], dtype=np.int64)
        for a in range(nd):
            bc = r % parts[a]
            r //= parts[a]
            x = np.arange(dims[a])
            inb = (x * parts[a]) // dims[a] == bc
            lo, hi = x[inb].min(), x[inb].max()
            da = np.maximum(0, np.maximum(lo - x, x - hi))
            hist = np.convolve(hist, np.bincount(da))
        c = np.cumsum(hist)
        out_d.append(int(c[min(eta, c.size - 1)]))
        out_db.append(int(c[min(eta + 1, c.size - 1)]))
    return np.array(out_d), np.array(out_db)


def level0_sets(p):
    G = composite.adjacency(p.A)
    d, db = [], []
    for q in range(p.nparts):
        m = composite.bfs_ball(G, p.part == q, p.eta)
        d.append(int(m.sum()))
        db.append(int((m | composite.neighbours(G, m)).sum()))
    return np.array(d), np.array(db)


@pytest.mark.parametrize("dims,parts,eta", [((64, 64), (2, 2), 1), ((20, 17), (3, 2), 2), ((12, 12, 12), (2, 3, 2), 1),
                                            ((16, 16, 16), (4, 4, 4), 2)])
def test_level0_closed_form(dims, parts, eta):
    p = make_problem(dims, parts, eta=eta)
    d, db = level0_sets(p)
    cd, cdb = l1_ball_counts(dims, parts, eta)
    assert d.tolist() == cd.tolist()
    assert db.tolist() == cdb.tolist()


def test_cfg1_totals():
    # the survey's exact totals for the 64^2 / 2x2 / eta = 1 workload
    p = make_problem((64, 64), (2, 2), eta=1)
    d, db = level0_sets(p)
    assert d.tolist() == [1088] * 4 and db.tolist() == [1153] * 4
    assert d.sum() == 4352 and db.sum() == 4612


def test_cfg2_cfg3_level0_totals_closed_form():
    # closed form only (no BFS at this size): 128^3 / 4^3 / eta 1 and 192^3 / 8^3 / eta 2
    d, db = l1_ball_counts((128,) * 3, (4,) * 3, 1)
    assert (d.sum(), db.sum(), d.max(), db.max()) == (2392064, 2700800, 38912, 45440)
    d, db = l1_ball_counts((192,) * 3, (8,) * 3, 2)
    assert (d.sum(), db.sum(), d.max(), db.max()) == (10287360, 12064184, 21024, 25064)


@pytest.mark.parametrize("dims,parts,eta", [((10, 9), (2, 2), 1), ((9, 9), (3, 3), 2), ((6, 5, 5), (2, 2, 1), 1)])
def test_all_levels_frontier_equals_all_pairs(dims, parts, eta):
    p = make_problem(dims, parts, eta=eta)
    H = amg.setup(p.A, max_coarse=4)
    for q in range(p.nparts):
        D1, Db1 = composite.composite_sets(H, p.part, q, eta)
        D2, Db2 = composite.composite_sets(H, p.part, q, eta, brute=True)
        for l in range(H.L + 1):
            assert np.array_equal(D1[l], D2[l]) and np.array_equal(Db1[l], Db2[l])


def test_monotone_in_padding_and_degenerate_cases():
    p = make_problem((24, 24), (3, 3))
    H = amg.setup(p.A)
    prev = None
    for eta in (0, 1, 2, 3):
        D, Db = composite.composite_sets(H, p.part, 4, eta)
        if prev is not None:
            for l in range(H.L + 1):
                assert np.all(prev[l] <= D[l])
        prev = D
        assert D[H.L].all() and Db[H.L].all()   # coarsest stored whole
        for l in range(H.L + 1):
            assert np.all(D[l] <= Db[l])
    # one subdomain: the composite grid is the whole hierarchy
    p1 = make_problem((24, 24), (1, 1))
    H1 = amg.setup(p1.A)
    D, Db = composite.composite_sets(H1, p1.part, 0, 1)
    assert all(d.all() for d in D)
    # padding >= graph diameter: every level is whole
    D, Db = composite.composite_sets(H, p.part, 0, 48)
    assert all(d.all() for d in D)


def test_local_operators_and_ownership():
    p = make_problem((32, 32), (2, 2), eta=1)
    H = amg.setup(p.A)
    comps = composite.build_all(H, p.part, p.nparts, p.eta)
    owned = np.concatenate([cg.owned_gid for cg in comps])
    assert np.array_equal(np.sort(owned), np.arange(p.n))        # each fine point owned once
    for cg in comps:
        for l, lev in enumerate(cg.levels):
            g = lev.gid
            assert np.all(np.diff(g[: lev.n_real]) > 0) and np.all(np.diff(g[lev.n_real:]) > 0)
            # real rows keep their whole global row
            Ag = H.A[l][g[: lev.n_real]]
            assert Ag.nnz == lev.A[: lev.n_real].nnz
            np.testing.assert_allclose(lev.d, np.abs(Ag).sum(1).A1, rtol=1e-15)
            if l < cg.L:
                assert lev.omissions == 0
                assert (lev.R != lev.P.T).nnz == 0
        assert cg.owned_local.size == cg.owned_gid.size
        assert np.all(cg.levels[0].gid[cg.owned_local] == cg.owned_gid)
