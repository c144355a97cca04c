"""CPU tests of the C-ABI library: it loads, exports every symbol the header
declares, rejects malformed input, and its host setup (RS hierarchy,
composite grids) matches the oracle bit-exactly.  No device calls: handles
are created with device = -1 (host-only)."""

import os
import re

import numpy as np
import pytest
from scipy import sparse

from oracle import amg, composite, cycles
from synth import config, grf, make_problem

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
amgdd = pytest.importorskip("paper_1906_10575_amd.amgdd")


def _header_functions():
    txt = open(os.path.join(ROOT, "include", "amgdd.h")).read()
    txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
    return sorted(set(re.findall(r"\b(amg[a-z_]+)\s*\(", txt)))


def test_library_exports_every_declared_symbol():
    lib = amgdd.load()
    names = _header_functions()
    assert len(names) >= 15
    for n in names:
        assert hasattr(lib, n), n
    assert sorted(amgdd.SIGNATURES) == names


def _host(p, **kw):
    return amgdd.Solver(p.A, p.part, p.nparts, padding=p.eta, device=-1, **kw)


CASES = [
    ("cfg1", lambda: config("cfg1")),
    ("2d_var_eta2", lambda: make_problem((40, 36), (3, 2), eta=2, k=np.exp(grf((40, 36), 1.0, 8.0, 3)))),
    ("3d_16_eta1", lambda: make_problem((16, 16, 16), (2, 2, 2), eta=1)),
    ("3d_12_var_eta2", lambda: make_problem((12, 12, 12), (2, 3, 2), eta=2, k=np.exp(grf((12, 12, 12), 1.0, 8.0, 1)))),
    ("cfg4_16", lambda: config("cfg4", scale=16)),
    ("p2_48_aniso", lambda: config("p2", scale=48)),
    # padding 0: two subdomains have no points on level 4 (above the coarsest)
    ("3d_pad0_empty_levels", lambda: make_problem((20, 18, 20), (2, 2, 3), eta=0,
                                                  k=np.exp(grf((20, 18, 20), 1.0, 8.0, 1)))),
]


@pytest.mark.parametrize("name,make", CASES)
def test_host_setup_bit_exact_with_oracle(name, make):
    p = make()
    s = _host(p)
    H = amg.setup(p.A)
    n, z = s.levels(0)
    assert n.tolist() == [A.shape[0] for A in H.A]
    assert z.tolist() == [A.nnz for A in H.A]
    for l in range(H.L):
        assert np.array_equal(s.cf(0, l), H.cf[l]), f"C/F level {l}"
        P = s.operator(0, l, 1)
        assert (P != H.P[l]).nnz == 0 and np.array_equal(P.indptr, H.P[l].indptr)
        A = s.operator(0, l + 1, 0)
        assert np.array_equal(A.indptr, H.A[l + 1].indptr) and np.array_equal(A.indices, H.A[l + 1].indices)
        np.testing.assert_array_equal(A.data, H.A[l + 1].data)
    comps = composite.build_all(H, p.part, p.nparts, p.eta)
    for q, cg in enumerate(comps):
        for l, lv in enumerate(cg.levels):
            g, nr, om = s.composite(0, q, l)
            assert nr == lv.n_real and np.array_equal(g, lv.gid), f"p {q} level {l}"
            assert om == lv.omissions
    if name == "3d_pad0_empty_levels":
        assert any(lv.n_bar == 0 for cg in comps for lv in cg.levels)
    st = s.stats()
    assert st["n_grids"] == p.nparts
    assert abs(st["composite_overhead"] - composite.composite_overhead(H, comps)) < 1e-14


def test_batched_host_setup_matches_each_problem():
    probs = [make_problem((24, 20), (2, 2), eta=1), make_problem((33, 33), (3, 3), eta=2),
             make_problem((10, 10, 10), (2, 2, 1), eta=1, k=np.exp(grf((10, 10, 10), 1.0, 4.0, 5)))]
    s = amgdd.Solver([p.A for p in probs], [p.part for p in probs], [p.nparts for p in probs],
                     padding=[p.eta for p in probs], device=-1)
    st = s.stats()
    assert st["n_problems"] == 3 and st["n_grids"] == sum(p.nparts for p in probs)
    for i, p in enumerate(probs):
        H = amg.setup(p.A)
        assert s.levels(i)[0].tolist() == [A.shape[0] for A in H.A]
        for q in range(p.nparts):
            D, Dbar = composite.composite_sets(H, p.part, q, p.eta)
            for l in range(H.L + 1):
                g, nr, _ = s.composite(i, q, l)
                assert nr == D[l].sum() and set(g.tolist()) == set(np.nonzero(Dbar[l])[0].tolist())


def test_cfg2_level0_sets_closed_form():
    """Full-size 128^3 / 4^3 / eta 1: every subdomain's level-0 real and ghost
    counts equal the L1-ball closed form (setup only, no solve)."""
    from tests.test_oracle_composite import l1_ball_counts
    p = config("cfg2")
    s = _host(p)
    d, db = l1_ball_counts((128,) * 3, (4,) * 3, 1)
    for q in range(p.nparts):
        g, nr, om = s.composite(0, q, 0)
        assert (nr, g.size) == (d[q], db[q])
    st = s.stats()
    assert st["omissions"] == 0


def _bad(A, part=None, nparts=1, **kw):
    n = A.shape[0]
    part = np.zeros(n, dtype=np.int32) if part is None else part
    with pytest.raises(amgdd.AmgddError) as e:
        amgdd.Solver(A, part, nparts, device=-1, **kw)
    return e.value.status


def test_error_paths():
    p = make_problem((8, 8), (1, 1))
    A = p.A.copy()
    # unsorted columns
    B = A.copy()
    B.indices = B.indices.copy()
    B.indices[[0, 1]] = B.indices[[1, 0]]
    assert _bad(B) == amgdd.EINVAL
    # zero diagonal
    C = A.copy().tolil()
    C[3, 3] = 0.0
    C = C.tocsr()
    C.eliminate_zeros()
    assert _bad(C) == amgdd.EINVAL
    # non-finite entry
    D = A.copy()
    D.data = D.data.copy()
    D.data[5] = np.nan
    assert _bad(D) == amgdd.EINVAL
    # partition out of range / empty subdomain
    assert _bad(A, part=np.full(64, 3, dtype=np.int32), nparts=2) == amgdd.EINVAL
    assert _bad(A, part=np.zeros(64, dtype=np.int32), nparts=2) == amgdd.EINVAL
    # too small for a hierarchy
    small = make_problem((4, 4), (1, 1)).A
    assert _bad(small) == amgdd.EUNSUPPORTED
    # host-only handle refuses device work
    s = amgdd.Solver(A, np.zeros(64, dtype=np.int32), 1, device=-1)
    lib = amgdd.load()
    info = amgdd.Info()
    assert lib.amgdd_solve(s._h, None, None, 1e-8, 10, None) in (amgdd.EINVAL, amgdd.EDEVICE)
    assert lib.amgdd_profile(s._h, 0, 1, None, 0, None) in (amgdd.EINVAL, amgdd.EDEVICE)
    s.close()
    s.close()  # idempotent
    lib.amgdd_destroy(None)  # NULL accepted


HYBRID_CASES = [
    ("2d_var_lt1", lambda: make_problem((40, 36), (3, 2), eta=2, k=np.exp(grf((40, 36), 1.0, 8.0, 3))), 1),
    ("3d_16_lt2", lambda: make_problem((16, 16, 16), (2, 2, 2), eta=1), 2),
    ("2d_64parts_lt2", lambda: make_problem((16, 16), (8, 8), eta=1), 2),
]


@pytest.mark.parametrize("name,make,lt", HYBRID_CASES)
def test_hybrid_host_setup_matches_oracle(name, make, lt):
    # the level-L~ problems' composite grids equal the oracle's grids built on
    # the sub-hierarchy with the inherited partition; empty subdomains dropped
    p = make()
    s = _host(p, hybrid_level=lt)
    H = amg.setup(p.A)
    assert H.L > lt
    n, _ = s.levels(0)
    assert n.tolist() == [A.shape[0] for A in H.A]
    lt_, Hs, comps = cycles.hybrid_setup(H, p.part, p.nparts, p.eta, lt)
    part = cycles.inherited_partition(H, p.part, lt)
    nonempty = [q for q in range(p.nparts) if np.any(part == q)]
    for q in range(p.nparts):
        if q not in nonempty:
            with pytest.raises(amgdd.AmgddError):
                s.composite(0, q, lt)
            continue
        for l, lv in enumerate(comps[q].levels):
            g, nr, om = s.composite(0, q, lt + l)
            assert nr == lv.n_real and np.array_equal(g, lv.gid), f"p {q} level {lt + l}"
            assert om == lv.omissions
    with pytest.raises(amgdd.AmgddError):
        s.composite(0, nonempty[0], lt - 1)
    st = s.stats()
    assert st["hybrid_level"] == lt
    assert st["n_grids"] == len(nonempty)
    upper = sum(H.A[l].nnz for l in range(lt))
    real = sum(composite.composite_overhead(Hs, [comps[q]]) for q in nonempty) * sum(A.nnz for A in Hs.A)
    want = (upper + real) / sum(A.nnz for A in H.A)
    assert abs(st["composite_overhead"] - want) < 1e-12
    assert st["composite_overhead"] < _host(p).stats()["composite_overhead"]


def test_hybrid_level_below_every_hierarchy():
    # L~ at or beyond the coarsest level of every problem: no level-L~ AMG-DD
    # problem, the handle cycles plain V-cycles and holds no composite grid
    p = make_problem((24, 24), (2, 2))
    H = amg.setup(p.A)
    s = _host(p, hybrid_level=H.L)
    st = s.stats()
    assert st["hybrid_level"] == H.L and st["n_grids"] == 0
    assert abs(st["composite_overhead"] - 1.0) < 1e-15
    with pytest.raises(amgdd.AmgddError):
        s.composite(0, 0, H.L)
    with pytest.raises(amgdd.AmgddError) as e:
        _host(p, hybrid_level=-1)
    assert e.value.status == amgdd.EINVAL


def test_cf_handle_setup_and_parameter_check():
    # CF ordering stores each grid's real rows C-points first internally; the
    # composite sets reported through the ABI are those of the oracle
    p = make_problem((40, 36), (3, 2), eta=2, k=np.exp(grf((40, 36), 1.0, 8.0, 3)))
    s = _host(p, relax="cf")
    H = amg.setup(p.A)
    comps = composite.build_all(H, p.part, p.nparts, p.eta)
    for q, cg in enumerate(comps):
        for l, lv in enumerate(cg.levels):
            g, nr, om = s.composite(0, q, l)
            assert nr == lv.n_real and np.array_equal(g, lv.gid)
    assert s.stats()["composite_overhead"] == _host(p).stats()["composite_overhead"]
    with pytest.raises(ValueError):
        _host(p, relax="gs")
    prm = amgdd.default_params()
    assert prm.relax_order == 0


BP_CASES = [
    ("2d_var", lambda: make_problem((40, 36), (3, 2), eta=2, k=np.exp(grf((40, 36), 1.0, 8.0, 3)))),
    ("3d_12_var", lambda: make_problem((12, 12, 12), (2, 3, 2), eta=1, k=np.exp(grf((12, 12, 12), 1.0, 8.0, 1)))),
    ("p2_40", lambda: config("p2", scale=40)),
]


@pytest.mark.parametrize("coarsen,interp", [("hmis", "ext+i"), ("hmis", "direct"), ("rs", "ext+i")])
@pytest.mark.parametrize("name,make", BP_CASES)
def test_best_practice_setup_bit_exact_with_oracle(name, make, coarsen, interp):
    # HMIS (with its SplitMix64 tie-breaks) and extended+i: identical C/F
    # splittings, bitwise identical P and coarse operators, same composite sets
    p = make()
    s = _host(p, coarsen=coarsen, interp=interp)
    H = amg.setup(p.A, coarsen=coarsen, interp=interp, part=p.part)
    n, z = s.levels(0)
    assert n.tolist() == [A.shape[0] for A in H.A]
    for l in range(H.L):
        assert np.array_equal(s.cf(0, l), H.cf[l]), f"C/F level {l}"
        P = s.operator(0, l, 1)
        assert np.array_equal(P.indptr, H.P[l].indptr) and np.array_equal(P.indices, H.P[l].indices)
        np.testing.assert_array_equal(P.data, H.P[l].data)
        A = s.operator(0, l + 1, 0)
        assert np.array_equal(A.indices, H.A[l + 1].indices)
        np.testing.assert_array_equal(A.data, H.A[l + 1].data)
    comps = composite.build_all(H, p.part, p.nparts, p.eta)
    for q, cg in enumerate(comps):
        for l, lv in enumerate(cg.levels):
            g, nr, om = s.composite(0, q, l)
            assert nr == lv.n_real and np.array_equal(g, lv.gid)
            assert om == lv.omissions


# ---------------------------------------------------------------- per-level padding

def _mask(n, gids):
    m = np.zeros(n, dtype=bool)
    m[gids] = True
    return m


def test_per_level_padding_matches_hand_derived_chain():
    import json
    g = json.load(open(os.path.join(ROOT, "tests", "golden", "composite_chain33.json")))
    p = make_problem((33,), (2,), eta=1)
    for case in g["cases"]:
        s = amgdd.Solver(p.A, p.part, 2, padding=1, padding_per_level=case["padding"], max_coarse=4, device=-1)
        n, _ = s.levels(0)
        assert n.tolist() == g["levels"]
        for q in range(2):
            for l in range(len(n)):
                gids, nr, om = s.composite(0, q, l)
                a, b = case["sets"][str(q)]["D"][l]
                ab, bb = case["sets"][str(q)]["Dbar"][l]
                assert gids[:nr].tolist() == list(range(a, b + 1)), (case["padding"], q, l)
                assert sorted(gids.tolist()) == list(range(ab, bb + 1)), (case["padding"], q, l)
                assert om == 0


def test_per_level_padding_matches_closed_form_and_oracle():
    from tests.test_oracle_composite_levels import closed_form_sets, xline_operator, xline_part
    A = xline_operator()
    part = xline_part()
    etas = [1, 2, 0, 3]
    s = amgdd.Solver(A, part, 4, padding=5, padding_per_level=etas, device=-1)
    H = amg.setup(A)
    n, _ = s.levels(0)
    for q in range(4):
        Dc, Dbc = closed_form_sets(part, q, etas, H.L + 1)
        D, Db = composite.composite_sets(H, part, q, etas + [0])
        for l in range(H.L + 1):
            gids, nr, om = s.composite(0, q, l)
            assert np.array_equal(_mask(n[l], gids[:nr]), Dc[l]) and np.array_equal(_mask(n[l], gids), Dbc[l])
            assert np.array_equal(D[l], Dc[l])
    # a shorter list: deeper levels take `padding`
    p = make_problem((20, 18, 20), (2, 2, 3), eta=2, k=np.exp(grf((20, 18, 20), 1.0, 8.0, 1)))
    s = amgdd.Solver(p.A, p.part, p.nparts, padding=2, padding_per_level=[1, 3], device=-1)
    H = amg.setup(p.A)
    etas = [1, 3] + [2] * (H.L - 1)
    for q in range(p.nparts):
        D, Db = composite.composite_sets(H, p.part, q, etas)
        for l in range(H.L + 1):
            gids, nr, om = s.composite(0, q, l)
            assert np.array_equal(_mask(H.A[l].shape[0], gids[:nr]), D[l]), (q, l)
            assert np.array_equal(_mask(H.A[l].shape[0], gids), Db[l]), (q, l)


def test_per_level_padding_in_a_batch_and_errors():
    p1 = make_problem((33,), (2,), eta=1)
    p2 = make_problem((24, 24), (2, 2), eta=1)
    s = amgdd.Solver([p1.A, p2.A], [p1.part, p2.part], [2, 4], padding=[1, 1], padding_per_level=[[2, 0, 1], None],
                     max_coarse=4, device=-1)
    gids, nr, om = s.composite(0, 1, 1)
    assert gids[:nr].tolist() == list(range(7, 16))        # hand-derived chain, eta (2, 0, 1)
    ref = amgdd.Solver(p2.A, p2.part, 4, padding=1, max_coarse=4, device=-1)
    for q in range(4):
        assert np.array_equal(s.composite(1, q, 1)[0], ref.composite(0, q, 1)[0])
    with pytest.raises(amgdd.AmgddError) as e:
        amgdd.Solver(p1.A, p1.part, 2, padding_per_level=[1, -1], device=-1)
    assert e.value.status == amgdd.EINVAL
    with pytest.raises(ValueError):
        amgdd.Solver([p1.A, p2.A], [p1.part, p2.part], [2, 4], padding_per_level=[[1]], device=-1)


# ---------------------------------------------------------------- binding argument checks

def test_binding_rejects_bad_vectors_and_face_indices():
    torch = pytest.importorskip("torch")
    p = make_problem((24, 24), (2, 2), eta=1)
    s = _host(p)
    with pytest.raises(TypeError):
        s.solve(torch.zeros(p.n, dtype=torch.float64))             # host tensor
    with pytest.raises(TypeError):
        s.solve(np.zeros(p.n))
    with pytest.raises(ValueError):
        s.face_gradient(None, None, np.array([0, p.n]), np.array([1, -1]))   # face_i past the end
    with pytest.raises(ValueError):
        s.face_gradient(None, None, np.array([0, 1]), np.array([-2, 3]))     # face_j below -1
    with pytest.raises(ValueError):
        s.face_gradient(None, None, np.array([0, 1]), np.array([2]))         # length mismatch
