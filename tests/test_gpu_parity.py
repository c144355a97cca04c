"""GPU parity: the HIP path through the C ABI against the oracle, element by
element, on seeded inputs.

Bar: FP64 iterates within 1e-12 element-wise (max_i |x_gpu,i - x_oracle,i|
<= 1e-12 max_i |x_oracle,i|, tests/parity.py) after every outer iteration /
V-cycle; mixed precision reaches
1e-8 relative residual evaluated in FP64 and its error against the FP64
oracle is reported; adjoint gradients within 1e-6 of central differences."""

import sys

import numpy as np
import pytest
from scipy.sparse import linalg as spla

from oracle import adjoint, amg, composite, cycles
from synth import batch_config, config, grf, make_problem

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")
amgdd = pytest.importorskip("paper_1906_10575_amd.amgdd")

DEV = "cuda:0"


def say(*a):
    print("[gpu-test]", *a, flush=True)
    sys.stdout.flush()


def _t(x):
    return torch.as_tensor(np.ascontiguousarray(x, dtype=np.float64), device=DEV)


def _np(t):
    return t.detach().cpu().numpy()


CASES = {
    "cfg1": lambda: config("cfg1"),
    "2d_var_eta2_nfac3": lambda: make_problem((44, 38), (3, 2), eta=2, n_fac=3, k=np.exp(grf((44, 38), 1.0, 8.0, 3))),
    "3d_16_eta1": lambda: make_problem((16, 16, 16), (2, 2, 2), eta=1, n_fac=2),
    "3d_20_var_eta2": lambda: make_problem((20, 18, 20), (2, 2, 3), eta=2, n_fac=2,
                                           k=np.exp(grf((20, 18, 20), 1.0, 8.0, 1))),
    "3d_30_ragged_4x4x4": lambda: make_problem((30, 30, 30), (4, 4, 4), eta=1, n_fac=2),
    "p2_aniso_72": lambda: config("p2", scale=72),
}
ITERS = {"cfg1": 10, "2d_var_eta2_nfac3": 5, "3d_16_eta1": 6, "3d_20_var_eta2": 4, "3d_30_ragged_4x4x4": 4,
         "p2_aniso_72": 5}


@pytest.fixture(scope="module")
def oracle_cache():
    return {}


def _oracle(name, cache):
    if name not in cache:
        p = CASES[name]()
        H = amg.setup(p.A)
        comps = composite.build_all(H, p.part, p.nparts, p.eta)
        cache[name] = (p, H, comps)
    return cache[name]


from tests.parity import rel_2, rel_inf as _rel  # noqa: E402  (element-wise bar)


@pytest.mark.parametrize("name", list(CASES))
def test_amgdd_iterates_match_oracle(name, oracle_cache):
    p, H, comps = _oracle(name, oracle_cache)
    say("amgdd iterates", name, p.n, p.nparts, "eta", p.eta, "n_fac", p.n_fac)
    s = amgdd.Solver(p.A, p.part, p.nparts, padding=p.eta, n_fac=p.n_fac)
    b = _t(p.b)
    x = torch.zeros_like(b)
    xo = np.zeros(p.n)
    coarse = cycles.CoarseSolver(H.A[H.L])
    for k in range(ITERS[name]):
        x, info, st = s.solve(b, x, rtol=0, maxit=1)
        assert st == amgdd.OK and info.iters == 1
        xo = cycles.amgdd_iteration(H, comps, p.b, xo, p.n_fac, coarse)
        err = _rel(_np(x), xo)
        say(f"  iter {k + 1}: max-entry rel err {err:.3e}, 2-norm {rel_2(_np(x), xo):.3e}")
        assert err <= 1e-12, (k, err)


@pytest.mark.parametrize("name", list(CASES))
def test_vcycle_iterates_match_oracle(name, oracle_cache):
    p, H, comps = _oracle(name, oracle_cache)
    say("vcycle iterates", name)
    s = amgdd.Solver(p.A, p.part, p.nparts, padding=p.eta, n_fac=p.n_fac)
    b = _t(p.b)
    x = torch.zeros_like(b)
    xo = np.zeros(p.n)
    coarse = cycles.CoarseSolver(H.A[H.L])
    for k in range(10):
        x, info, st = s.vsolve(b, x, rtol=0, maxit=1)
        xo = cycles.vcycle(H, xo, p.b, coarse=coarse)
        err = _rel(_np(x), xo)
        assert err <= 1e-12, (k, err)


def test_graph_eager_and_repeat_are_bitwise_identical():
    p = CASES["3d_20_var_eta2"]()
    say("graph vs eager", p.n)
    b = _t(p.b)
    outs = []
    for use_graph in (True, False, True):
        s = amgdd.Solver(p.A, p.part, p.nparts, padding=p.eta, n_fac=p.n_fac, use_graph=use_graph)
        x, info, st = s.solve(b, rtol=0, maxit=5)
        xv, _, _ = s.vsolve(b, rtol=0, maxit=5)
        # a second solve on the same handle replays the same graph
        x2, _, _ = s.solve(b, rtol=0, maxit=5)
        assert torch.equal(x, x2)
        outs.append((_np(x), _np(xv)))
    for o in outs[1:]:
        assert np.array_equal(o[0], outs[0][0]) and np.array_equal(o[1], outs[0][1])


def test_stopping_history_matches_oracle(oracle_cache):
    p, H, comps = _oracle("3d_16_eta1", oracle_cache)
    say("rtol stop 1e-8")
    s = amgdd.Solver(p.A, p.part, p.nparts, padding=p.eta, n_fac=p.n_fac)
    x, info, st = s.solve(_t(p.b), rtol=1e-8, maxit=100)
    xo, ho = cycles.amgdd_solve(H, comps, p.b, np.zeros(p.n), p.n_fac, rtol=1e-8, maxit=100)
    hist = s.history(0)
    assert st == amgdd.OK and info.iters == len(ho) - 1
    np.testing.assert_allclose(hist, ho, rtol=1e-9, atol=1e-12 * ho[0])
    assert info.relres <= 1e-8
    xv, infov, stv = s.vsolve(_t(p.b), rtol=1e-8, maxit=100)
    xvo, hvo = cycles.vcycle_solve(H, p.b, np.zeros(p.n), rtol=1e-8, maxit=100)
    assert infov.iters == len(hvo) - 1
    assert _rel(_np(xv), xvo) <= 1e-12


def test_mixed_precision_reaches_1e8_and_reports_error():
    """cfg3's shape at reduced size: 3D variable k (sigma 1, l = 8), 4^3
    subdomains, padding 2.  FP32 inner FAC, FP64 outer residual/patch/coarse."""
    p = make_problem((32, 32, 32), (4, 4, 4), eta=2, n_fac=2, k=np.exp(grf((32,) * 3, 1.0, 8.0, 1)))
    say("mixed", p.n)
    H = amg.setup(p.A)
    comps = composite.build_all(H, p.part, p.nparts, p.eta)
    s = amgdd.Solver(p.A, p.part, p.nparts, padding=p.eta, n_fac=2, precision="mixed")
    b = _t(p.b)
    x = torch.zeros_like(b)
    xo = np.zeros(p.n)
    coarse = cycles.CoarseSolver(H.A[H.L])
    errs = []
    for k in range(6):
        x, info, st = s.solve(b, x, rtol=0, maxit=1)
        xo = cycles.amgdd_iteration(H, comps, p.b, xo, 2, coarse)
        errs.append(_rel(_np(x), xo))
    say("  mixed vs FP64 oracle per iteration:", " ".join(f"{e:.2e}" for e in errs))
    assert max(errs) < 1e-3  # the FP32 inner cycle perturbs the correction, not the iteration
    x, info, st = s.solve(b, rtol=1e-8, maxit=100)
    r = p.b - p.A @ _np(x)
    assert st == amgdd.OK and np.linalg.norm(r) <= 1e-8 * np.linalg.norm(p.b)
    s64 = amgdd.Solver(p.A, p.part, p.nparts, padding=p.eta, n_fac=2)
    _, info64, _ = s64.solve(b, rtol=1e-8, maxit=100)
    say(f"  iterations to 1e-8: mixed {info.iters}, fp64 {info64.iters}")
    assert info.iters <= info64.iters + 2


def test_batched_uneven_problems_match_oracle():
    probs = batch_config(n_problems=5, seed0=77, side_range=(40, 90), parts_range=(2, 4))
    say("batched", [pp.n for pp in probs], [pp.eta for pp in probs])
    s = amgdd.Solver([pp.A for pp in probs], [pp.part for pp in probs], [pp.nparts for pp in probs],
                     padding=[pp.eta for pp in probs], n_fac=2)
    b = _t(np.concatenate([pp.b for pp in probs]))
    x = torch.zeros_like(b)
    refs = []
    for pp in probs:
        H = amg.setup(pp.A)
        refs.append((H, composite.build_all(H, pp.part, pp.nparts, pp.eta), cycles.CoarseSolver(H.A[H.L])))
    xo = [np.zeros(pp.n) for pp in probs]
    off = np.cumsum([0] + [pp.n for pp in probs])
    for k in range(4):
        x, info, st = s.solve(b, x, rtol=0, maxit=1)
        xg = _np(x)
        for i, pp in enumerate(probs):
            H, comps, co = refs[i]
            xo[i] = cycles.amgdd_iteration(H, comps, pp.b, xo[i], 2, co)
            err = _rel(xg[off[i]:off[i + 1]], xo[i])
            assert err <= 1e-12, (k, i, err)
    # V-cycles on the batch as well
    xv, _, _ = s.vsolve(b, rtol=0, maxit=3)
    xg = _np(xv)
    for i, pp in enumerate(probs):
        H = refs[i][0]
        e = np.zeros(pp.n)
        for _ in range(3):
            e = cycles.vcycle(H, e, pp.b)
        assert _rel(xg[off[i]:off[i + 1]], e) <= 1e-12
    # mixed batch converges for every problem
    sm = amgdd.Solver([pp.A for pp in probs], [pp.part for pp in probs], [pp.nparts for pp in probs],
                      padding=[pp.eta for pp in probs], n_fac=2, precision="mixed")
    xm, info, st = sm.solve(b, rtol=1e-8, maxit=100)
    assert st == amgdd.OK
    xg = _np(xm)
    for i, pp in enumerate(probs):
        r = pp.b - pp.A @ xg[off[i]:off[i + 1]]
        assert np.linalg.norm(r) <= 1e-8 * np.linalg.norm(pp.b)


def _faces_ij(p):
    fi = np.concatenate([p.faces.inner_i, p.faces.bnd_i])
    fj = np.concatenate([p.faces.inner_j, -np.ones(p.faces.bnd_i.size, dtype=np.int64)])
    return fi, fj


def test_face_gradient_kernel_matches_formula():
    p = make_problem((9, 8, 7), (1, 1, 1))
    rng = np.random.default_rng(3)
    u = rng.standard_normal(p.n)
    lam = rng.standard_normal(p.n)
    s = amgdd.Solver(p.A, p.part, 1)
    fi, fj = _faces_ij(p)
    g = s.face_gradient(_t(u), _t(lam), torch.as_tensor(fi), torch.as_tensor(fj))
    np.testing.assert_array_equal(_np(g), adjoint.face_gradient(p.faces, u, lam))


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_adjoint_gradients_vs_central_differences(precision):
    """cfg4's operator at 16^3 (2^3 subdomains, padding 1): forward and
    adjoint AMG-DD to 1e-10; dL/df = lambda on every cell and dL/dc on 64
    seeded faces against central differences (h = 1e-6) through exact
    sparse-LU solves; all of dL/dc against the dense adjoint."""
    from paper_1906_10575_amd.autograd import FaceProblem, diffusion_solve
    p = config("cfg4", scale=16)
    ut = p.extra["u_target"]
    say("adjoint", precision, p.n)
    fi, fj = _faces_ij(p)
    prob = FaceProblem(p.n, fi, fj, p.part, p.nparts, padding=1, n_fac=2, precision=precision, rtol=1e-10)
    c = _t(p.c).requires_grad_(True)
    f = _t(p.b).requires_grad_(True)
    u = diffusion_solve(c, f, prob)
    loss = ((u - _t(ut)) ** 2).sum()
    loss.backward()
    gc = _np(c.grad)
    gf = _np(f.grad)
    L, u_d, lam_d, gc_d = adjoint.loss_and_grads(p.A, p.faces, p.b, ut)
    assert _rel(_np(u), u_d) <= 1e-9
    assert _rel(gf, lam_d) <= 1e-8
    assert np.abs(gc - gc_d).max() <= 1e-8 * np.abs(gc_d).max()
    from synth import assemble

    def loss_of(cv, fv):
        uu = spla.splu(assemble(p.n, p.faces, cv).tocsc()).solve(fv)
        return float(np.sum((uu - ut) ** 2))

    h = 1e-6
    lu = spla.splu(p.A.tocsc())
    Ainv_cols = None
    fd_f = np.empty(p.n)
    for i in range(p.n):
        e = np.zeros(p.n)
        e[i] = h
        up = lu.solve(p.b + e)
        um = lu.solve(p.b - e)
        fd_f[i] = (np.sum((up - ut) ** 2) - np.sum((um - ut) ** 2)) / (2 * h)
    assert np.abs(gf - fd_f).max() <= 1e-6 * np.abs(fd_f).max()
    rng = np.random.default_rng(42)
    sel = rng.choice(p.faces.n_faces, 64, replace=False)
    fd_c = []
    for k in sel:
        cp = p.c.copy()
        cp[k] += h
        cm = p.c.copy()
        cm[k] -= h
        fd_c.append((loss_of(cp, p.b) - loss_of(cm, p.b)) / (2 * h))
    fd_c = np.array(fd_c)
    assert np.abs(gc[sel] - fd_c).max() <= 1e-6 * np.abs(gc).max()


@pytest.mark.parametrize("lt,bs", [(-2, 0), (-1, 256), (0, 256), (1, 512)])
def test_error_paths_on_device(lt, bs):
    """Non-finite input is reported as EBREAKDOWN; iterations that ran on
    non-finite data (the autotuner on the first solve, or the profiler on the
    handle's stored right-hand side) leave nothing behind: the next clean solve
    is bitwise identical to one on a fresh handle, for every schedule (padding
    of empty rows never reads another grid's rows)."""
    p = CASES["3d_16_eta1"]()
    say("error paths, schedule", lt, bs)
    b = _t(p.b)
    fresh = amgdd.Solver(p.A, p.part, p.nparts, padding=1, tail_level=lt, tail_block=bs)
    x_ref, _, _ = fresh.solve(b, rtol=0, maxit=2)
    s = amgdd.Solver(p.A, p.part, p.nparts, padding=1, tail_level=lt, tail_block=bs)
    bad = b.clone()
    bad[7] = float("nan")
    with pytest.raises(amgdd.AmgddError) as e:
        s.solve(bad, rtol=1e-8, maxit=5)
    assert e.value.status == amgdd.EBREAKDOWN
    s.profile(kind=0, reps=2)
    x, info, st = s.solve(b, rtol=1e-14, maxit=2)
    assert st == amgdd.ENOCONV and info.iters == 2
    assert torch.equal(x, x_ref)
    x2, _, st2 = s.solve(b, rtol=0, maxit=2)
    assert st2 == amgdd.OK and torch.equal(x, x2)


@pytest.mark.parametrize("name", ["3d_20_var_eta2", "2d_var_eta2_nfac3"])
def test_every_schedule_gives_identical_iterates(name, oracle_cache):
    """The per-grid persistent schedule (cut level lt, workgroup size) performs
    the same per-row arithmetic as the level-synchronous one: results are
    bitwise identical for every choice, and match the oracle."""
    p, H, comps = _oracle(name, oracle_cache)
    b = _t(p.b)
    ref = None
    nlev = H.L + 1
    xo = np.zeros(p.n)
    coarse = cycles.CoarseSolver(H.A[H.L])
    for _ in range(3):
        xo = cycles.amgdd_iteration(H, comps, p.b, xo, p.n_fac, coarse)
    for lt, bs in [(-1, 256), (0, 256), (0, 1024), (1, 512), (nlev - 1, 256), (nlev // 2, 1024)]:
        say("schedule", name, lt, bs)
        s = amgdd.Solver(p.A, p.part, p.nparts, padding=p.eta, n_fac=p.n_fac, tail_level=lt, tail_block=bs)
        x, info, st = s.solve(b, rtol=0, maxit=3)
        st_ = s.stats()
        assert st_["tail_level"] == lt and st_["tail_block"] == bs
        xn = _np(x)
        if ref is None:
            ref = xn
        assert np.array_equal(xn, ref), (lt, bs)
        assert _rel(xn, xo) <= 1e-12
    s = amgdd.Solver(p.A, p.part, p.nparts, padding=p.eta, n_fac=p.n_fac)
    x, info, st = s.solve(b, rtol=0, maxit=3)
    st_ = s.stats()
    say("  autotuned:", st_["tail_level"], st_["tail_block"], f"{st_['autotune_s']:.3f} s")
    assert np.array_equal(_np(x), ref)


@pytest.mark.parametrize("name", ["3d_20_var_eta2", "3d_30_ragged_4x4x4"])
def test_mixed_every_schedule_gives_identical_iterates(name, oracle_cache):
    """Mixed precision (FP32 composite operators with four entries per lane
    and step): every launch schedule gives bitwise identical iterates, and
    they stay within the float32 error scale of the FP64 oracle."""
    p, H, comps = _oracle(name, oracle_cache)
    b = _t(p.b)
    nlev = H.L + 1
    xo = np.zeros(p.n)
    coarse = cycles.CoarseSolver(H.A[H.L])
    for _ in range(3):
        xo = cycles.amgdd_iteration(H, comps, p.b, xo, p.n_fac, coarse)
    ref = None
    for lt, bs in [(-1, 256), (0, 512), (1, 1024), (nlev // 2, 256)]:
        say("mixed schedule", name, lt, bs)
        s = amgdd.Solver(p.A, p.part, p.nparts, padding=p.eta, n_fac=p.n_fac, precision="mixed", tail_level=lt,
                         tail_block=bs)
        x, info, st = s.solve(b, rtol=0, maxit=3)
        xn = _np(x)
        if ref is None:
            ref = xn
        assert np.array_equal(xn, ref), (lt, bs)
        assert _rel(xn, xo) <= 1e-5


@pytest.mark.parametrize("name", ["3d_20_var_eta2", "p2_aniso_72", "2d_var_eta2_nfac3"])
@pytest.mark.parametrize("relax", ["l1", "cf"])
def test_best_practice_hierarchy_iterates(name, relax):
    # HMIS coarsening + truncated extended+i interpolation: AMG-DD and V-cycle
    # iterates against the oracle on the same hierarchy
    p = CASES[name]()
    say("hmis/ext+i iterates", name, relax)
    H = amg.setup(p.A, coarsen="hmis", interp="ext+i", part=p.part)
    comps = composite.build_all(H, p.part, p.nparts, p.eta)
    s = amgdd.Solver(p.A, p.part, p.nparts, padding=p.eta, n_fac=p.n_fac, coarsen="hmis", interp="ext+i", relax=relax)
    b = _t(p.b)
    coarse = cycles.CoarseSolver(H.A[H.L])
    x = torch.zeros_like(b)
    xo = np.zeros(p.n)
    for k in range(3):
        x, info, st = s.solve(b, x, rtol=0, maxit=1)
        xo = cycles.amgdd_iteration(H, comps, p.b, xo, p.n_fac, coarse, relax=relax)
        err = _rel(_np(x), xo)
        assert err <= 1e-12, (k, err)
    xv, _, _ = s.vsolve(b, rtol=0, maxit=3)
    e = np.zeros(p.n)
    for _ in range(3):
        e = cycles.vcycle(H, e, p.b, coarse=coarse, relax=relax)
    assert _rel(_np(xv), e) <= 1e-12
    x, info, st = s.solve(b, rtol=1e-8, maxit=200)
    assert st == amgdd.OK
    say(f"  converged in {info.iters} iterations, last iterate err {err:.2e}")


def test_mixed_iterates_track_the_float32_emulation():
    # the oracle's float32 emulation (FP32 operators, restriction chain and
    # AlgFAC; FP64 residual, patch and coarsest solve) deviates from FP64 by
    # d_k after k iterations; the device's mixed iterates must sit within a
    # few d_k of the emulation (a residual or coarse solve in FP32 would not:
    # its error stops shrinking with the corrections)
    p = CASES["3d_20_var_eta2"]()
    say("mixed vs float32 emulation", p.n)
    H = amg.setup(p.A)
    comps = composite.build_all(H, p.part, p.nparts, p.eta)
    co = cycles.CoarseSolver(H.A[H.L])
    s = amgdd.Solver(p.A, p.part, p.nparts, padding=p.eta, n_fac=p.n_fac, precision="mixed")
    b = _t(p.b)
    x = torch.zeros_like(b)
    x64 = np.zeros(p.n)
    x32 = np.zeros(p.n)
    for k in range(5):
        x, info, st = s.solve(b, x, rtol=0, maxit=1)
        x64 = cycles.amgdd_iteration(H, comps, p.b, x64, p.n_fac, co)
        x32 = cycles.amgdd_iteration(H, comps, p.b, x32, p.n_fac, co, dtype=np.float32)
        d = np.linalg.norm(x32 - x64)
        e = np.linalg.norm(_np(x) - x32)
        di = np.abs(x32 - x64).max()
        ei = np.abs(_np(x) - x32).max()
        say(f"  iter {k + 1}: emulation vs FP64 {d / np.linalg.norm(x64):.2e} (max entry "
            f"{di / np.abs(x64).max():.2e}), device vs emulation {e / np.linalg.norm(x64):.2e} (max entry "
            f"{ei / np.abs(x64).max():.2e})")
        assert e <= 4.0 * d + 1e-13 * np.linalg.norm(x64), (k, e, d)
        assert ei <= 4.0 * di + 1e-13 * np.abs(x64).max(), (k, ei, di)
