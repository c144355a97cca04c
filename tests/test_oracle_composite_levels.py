"""Pins for the oracle's composite sets on the coarse levels (l >= 1).

The set rule (Section 3, Figure 1): level l+1 of subdomain p is seeded with
the C-points of D_l, mapped to their coarse ids, and grown by the padding
eta_{l+1} through the graph of A_{l+1}; the coarsest level is stored whole;
the ghost layer Dbar_l is D_l plus its graph neighbours (Section 4.1).

Two cases whose sets can be derived without running any set code:
* a 1D chain (tests/golden/composite_chain33.json, derived by hand, uniform and
  per-level padding);
* a 2D operator with strong couplings along x only, where RS coarsens each
  x-line like the chain (C = odd x on every level) and the coarse graphs are
  9-point stencils, so every set is a clipped Manhattan (level 0) or
  Chebyshev (levels >= 1) ball written here as coordinate arithmetic.
Each pin fails for the plausible slips listed in the derivation: seeding from
Dbar_l instead of D_l, seeding from the F-points, growing coarse levels by
eta - 1."""

import json
import os

import numpy as np
import pytest
from scipy import sparse

from oracle import amg, composite
from synth import make_problem

GOLD = os.path.join(os.path.dirname(__file__), "golden", "composite_chain33.json")


def _interval_mask(n, ab):
    m = np.zeros(n, dtype=bool)
    m[ab[0]: ab[1] + 1] = True
    return m


def chain_case():
    g = json.load(open(GOLD))
    p = make_problem((g["problem"]["n"],), (2,), eta=1)
    H = amg.setup(p.A, max_coarse=g["problem"]["max_coarse"])
    return g, p, H


def test_chain_hierarchy_is_the_hand_derived_one():
    g, p, H = chain_case()
    assert [A.shape[0] for A in H.A] == g["levels"]
    assert p.part.tolist() == [0] * 17 + [1] * 16
    for l in range(H.L):
        n = H.A[l].shape[0]
        assert H.cf[l].tolist() == [1 if i % 2 else -1 for i in range(n)], l


@pytest.mark.parametrize("case", [0, 1])
def test_chain_sets_match_hand_derivation(case):
    g, p, H = chain_case()
    c = g["cases"][case]
    eta = c["padding"] + [0]  # the coarsest entry is unused (stored whole)
    for q in range(2):
        D, Db = composite.composite_sets(H, p.part, q, eta)
        for l in range(H.L + 1):
            n = H.A[l].shape[0]
            assert np.array_equal(D[l], _interval_mask(n, c["sets"][str(q)]["D"][l])), (q, l)
            assert np.array_equal(Db[l], _interval_mask(n, c["sets"][str(q)]["Dbar"][l])), (q, l)


# ---------------------------------------------------------------- 2D, x-line coarsening

NX, NY, EPS = 33, 6, 1e-3


def xline_operator(nx=NX, ny=NY, eps=EPS):
    """5-point operator with couplings -1 along x and -eps along y (Dirichlet
    nodes eliminated, diagonal = sum of the four face coefficients)."""
    idx = np.arange(nx * ny).reshape(ny, nx)
    rows, cols, vals = [idx.ravel()], [idx.ravel()], [np.full(nx * ny, 2.0 + 2.0 * eps)]
    for (sl_a, sl_b, c) in (((slice(None), slice(0, -1)), (slice(None), slice(1, None)), 1.0),
                            ((slice(0, -1), slice(None)), (slice(1, None), slice(None)), eps)):
        a, b = idx[sl_a].ravel(), idx[sl_b].ravel()
        rows += [a, b]
        cols += [b, a]
        vals += [np.full(a.size, -c), np.full(a.size, -c)]
    A = sparse.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                          shape=(nx * ny, nx * ny))
    A.sort_indices()
    return A


def xline_part(nx=NX, ny=NY):
    x = np.arange(nx)[None, :].repeat(ny, 0)
    y = np.arange(ny)[:, None].repeat(nx, 1)
    return ((x * 2) // nx + 2 * ((y * 2) // ny)).ravel()


def closed_form_sets(part, p, etas, nlev):
    """Expected D_l, Dbar_l of subdomain p from coordinates only.  Level l has
    nx_l = nx_{l-1} // 2 points per line (the odd x of the level above; coarse
    point (X, y) comes from (2X + 1, y)).  Level 0's graph is the 5-point
    stencil (Manhattan distance), every coarser graph the 9-point stencil
    (Chebyshev distance)."""
    nx = [NX]
    for _ in range(nlev - 1):
        nx.append(nx[-1] // 2)
    xs0, ys0 = np.meshgrid(np.arange(NX), np.arange(NY))
    seed = (part == p).reshape(NY, NX)
    D, Db = [], []
    for l in range(nlev):
        X, Y = np.meshgrid(np.arange(nx[l]), np.arange(NY))
        sx, sy = np.nonzero(seed.T)
        if l == nlev - 1:
            d = np.ones((NY, nx[l]), dtype=bool)
            db = d
        else:
            if l == 0:
                dist = np.abs(X[..., None] - sx) + np.abs(Y[..., None] - sy)
            else:
                dist = np.maximum(np.abs(X[..., None] - sx), np.abs(Y[..., None] - sy))
            d = dist.min(-1) <= etas[l]
            dx, dy = np.nonzero(d.T)
            if l == 0:
                nd = np.abs(X[..., None] - dx) + np.abs(Y[..., None] - dy)
            else:
                nd = np.maximum(np.abs(X[..., None] - dx), np.abs(Y[..., None] - dy))
            db = nd.min(-1) <= 1
            # next seeds: the odd-x points of D_l, at coarse x = (x - 1) / 2
            seed = np.zeros((NY, nx[l + 1]), dtype=bool)
            yy, xx = np.nonzero(d)
            odd = xx % 2 == 1
            seed[yy[odd], (xx[odd] - 1) // 2] = True
        D.append(d.ravel())
        Db.append(db.ravel())
    return D, Db


def xline_hierarchy():
    A = xline_operator()
    return A, amg.setup(A)


def test_xline_hierarchy_coarsens_each_line_like_the_chain():
    A, H = xline_hierarchy()
    assert [M.shape[0] for M in H.A] == [NY * NX, NY * 16, NY * 8, NY * 4, NY * 2]
    for l in range(H.L):
        nx = H.A[l].shape[0] // NY
        xs = np.tile(np.arange(nx), NY)
        assert H.cf[l].tolist() == np.where(xs % 2 == 1, 1, -1).tolist(), l
    # coarse graphs are 9-point stencils: Chebyshev neighbours on the level's grid
    for l in range(1, H.L + 1):
        nx = H.A[l].shape[0] // NY
        G = composite.adjacency(H.A[l]).tocoo()
        ax, ay = G.row % nx, G.row // nx
        bx, by = G.col % nx, G.col // nx
        assert np.all(np.maximum(np.abs(ax - bx), np.abs(ay - by)) == 1)
        assert G.nnz == sum(1 for x in range(nx) for y in range(NY) for dx in (-1, 0, 1) for dy in (-1, 0, 1)
                            if (dx or dy) and 0 <= x + dx < nx and 0 <= y + dy < NY)


@pytest.mark.parametrize("etas", [(2, 2, 2, 2), (1, 2, 3, 1), (0, 1, 0, 2)])
def test_xline_sets_match_closed_form(etas):
    A, H = xline_hierarchy()
    part = xline_part()
    for q in range(4):
        D, Db = composite.composite_sets(H, part, q, list(etas) + [0])
        Dc, Dbc = closed_form_sets(part, q, etas, H.L + 1)
        for l in range(H.L + 1):
            assert np.array_equal(D[l], Dc[l]), (q, l)
            assert np.array_equal(Db[l], Dbc[l]), (q, l)
        # padding 2 on level >= 1 is a proper subset there (the pin is not saturated)
        if etas[1] >= 1:
            assert not D[1].all()


# ---------------------------------------------------------------- the pins reject plausible slips

def mutated_sets(H, part, p, etas, slip):
    """The set rule with one plausible slip, built from the oracle's own
    graph helpers: 'dbar' seeds level l+1 from the C-points of Dbar_l, 'f'
    tests the F-points instead of the C-points, 'shrink' grows coarse levels
    by eta - 1."""
    graphs = [composite.adjacency(A) for A in H.A]
    seed = np.asarray(part) == p
    D, Db = [], []
    for l in range(H.L + 1):
        n = H.A[l].shape[0]
        if l == H.L:
            d = np.ones(n, dtype=bool)
        else:
            e = etas[l] - (1 if slip == "shrink" and l > 0 else 0)
            d = composite.bfs_ball(graphs[l], seed, max(e, 0))
        db = d | composite.neighbours(graphs[l], d)
        D.append(d)
        Db.append(db)
        if l < H.L:
            cm = composite.coarse_map(H.cf[l])
            src = db if slip == "dbar" else d
            kind = -1 if slip == "f" else 1
            sel = np.nonzero(src & (H.cf[l] == kind))[0]
            seed = np.zeros(H.A[l + 1].shape[0], dtype=bool)
            seed[cm[sel]] = True
    return D, Db


@pytest.mark.parametrize("slip", ["dbar", "f", "shrink"])
def test_pins_reject_plausible_slips(slip):
    # chain, uniform padding 1
    g, p, H = chain_case()
    c = g["cases"][0]
    chain_differs = False
    for q in range(2):
        D, Db = mutated_sets(H, p.part, q, [1, 1, 1, 0], slip)
        for l in range(H.L + 1):
            n = H.A[l].shape[0]
            ok = np.array_equal(D[l], _interval_mask(n, c["sets"][str(q)]["D"][l]))
            chain_differs |= not ok
    assert chain_differs
    # 2D x-line case, padding 2
    A, H2 = xline_hierarchy()
    part = xline_part()
    differs = False
    for q in range(4):
        D, Db = mutated_sets(H2, part, q, [2, 2, 2, 2, 0], slip)
        Dc, Dbc = closed_form_sets(part, q, (2, 2, 2, 2), H2.L + 1)
        differs |= any(not np.array_equal(D[l], Dc[l]) for l in range(1, H2.L + 1))
    assert differs
