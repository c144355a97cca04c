"""GPU parity of the adjoint solve for a non-symmetric operator (diffusion
plus upwind convection: symmetric pattern, non-symmetric values), through
the transposed composite operators.

Against the oracle's AMG-DD on the transposed hierarchy (oracle.adjoint.
transposed_hierarchy; pinned in tests/test_oracle_adjoint_transposed.py):
* adjoint iterates element-wise within 1e-12 (FP64), plain and hybrid cycles;
* the converged adjoint within 1e-10 of the dense solve of A^T lambda = g;
* mixed precision reaches 1e-8 (residual g - A^T lambda evaluated in FP64);
* forward solves on the same handle are unchanged by the adjoint setup;
* dL/dc and dL/dk (cell coefficients through harmonic face means) of
  L = ||u - u_t||^2 within 1e-6 of central differences (h = 1e-6, sparse LU)."""

import sys

import numpy as np
import pytest
from scipy.sparse import linalg as spla

from oracle import adjoint, amg, composite, cycles
from synth import convection_diffusion_problem, face_coefficients, grf
from tests.parity import rel_2, rel_inf

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
    "2d_24x20": lambda: convection_diffusion_problem((24, 20), (2, 2), velocity=(1.0, 0.5), eta=1, n_fac=2),
    "3d_10x9x8_var": lambda: convection_diffusion_problem((10, 9, 8), (2, 2, 2), velocity=(0.7, -0.4, 0.3), eta=2,
                                                          n_fac=2, k=np.exp(grf((10, 9, 8), 0.5, 4.0, 3))),
    "2d_40x36_eta2_nfac3": lambda: convection_diffusion_problem((40, 36), (3, 2), velocity=(-1.5, 0.8), eta=2,
                                                                n_fac=3, k=np.exp(grf((40, 36), 0.5, 4.0, 5))),
}


@pytest.mark.parametrize("name", list(CASES))
def test_adjoint_iterates_match_transposed_oracle(name):
    p = CASES[name]()
    say("nonsym adjoint iterates", name, p.n)
    H = amg.setup(p.A)
    HT = adjoint.transposed_hierarchy(H)
    comps = composite.build_all(HT, p.part, p.nparts, p.eta)
    co = cycles.CoarseSolver(HT.A[HT.L])
    s = amgdd.Solver(p.A, p.part, p.nparts, padding=p.eta, n_fac=p.n_fac)
    g = np.random.default_rng(9).uniform(-1, 1, p.n)
    gt = _t(g)
    lam = torch.zeros_like(gt)
    lo = np.zeros(p.n)
    for k in range(5):
        lam, info, st = s.solve_adjoint(gt, lam, rtol=0, maxit=1)
        lo = cycles.amgdd_iteration(HT, comps, g, lo, p.n_fac, co)
        err = rel_inf(_np(lam), lo)
        say(f"  iteration {k + 1}: max-entry rel err {err:.2e} (2-norm {rel_2(_np(lam), lo):.2e})")
        assert err <= 1e-12
    lam, info, st = s.solve_adjoint(gt, rtol=1e-12, maxit=200)
    assert st == amgdd.OK
    ref = adjoint.dense_adjoint(p.A, g)
    assert rel_inf(_np(lam), ref) <= 1e-10
    r = g - p.A.T @ _np(lam)
    assert np.linalg.norm(r) <= 1e-12 * np.linalg.norm(g) * 1.01
    assert s.stats()["device_bytes"] > 0


def test_forward_unchanged_and_mixed_adjoint_reaches_1e8():
    p = CASES["3d_10x9x8_var"]()
    say("nonsym forward/mixed", p.n)
    b = _t(p.b)
    s = amgdd.Solver(p.A, p.part, p.nparts, padding=p.eta, n_fac=p.n_fac)
    x1, _, st1 = s.solve(b, rtol=1e-10, maxit=100)
    g = _t(np.random.default_rng(4).uniform(-1, 1, p.n))
    s.solve_adjoint(g, rtol=1e-10, maxit=100)
    x2, _, st2 = s.solve(b, rtol=1e-10, maxit=100)
    assert st1 == st2 == amgdd.OK and torch.equal(x1, x2)
    xr = np.linalg.solve(p.A.toarray(), p.b)
    assert rel_inf(_np(x1), xr) <= 1e-8
    sm = amgdd.Solver(p.A, p.part, p.nparts, padding=p.eta, n_fac=p.n_fac, precision="mixed")
    lam, info, st = sm.solve_adjoint(g, rtol=1e-8, maxit=200)
    assert st == amgdd.OK
    gh = _np(g)
    rel = np.linalg.norm(gh - p.A.T @ _np(lam)) / np.linalg.norm(gh)
    say(f"  mixed adjoint: {info.iters} iterations, FP64 relres {rel:.2e}")
    assert rel <= 1e-8
    ref = adjoint.dense_adjoint(p.A, gh)
    say(f"  mixed adjoint error vs dense adjoint: {rel_2(_np(lam), ref):.2e}")


@pytest.mark.parametrize("lt", [1, 2])
def test_hybrid_adjoint_iterates_match_transposed_oracle(lt):
    p = convection_diffusion_problem((32, 30), (2, 2), velocity=(1.0, -0.5), eta=1, n_fac=2,
                                     k=np.exp(grf((32, 30), 0.5, 4.0, 8)))
    say("nonsym hybrid adjoint", lt, p.n)
    H = amg.setup(p.A)
    HT = adjoint.transposed_hierarchy(H)
    lt_, Hs, comps_s = cycles.hybrid_setup(HT, p.part, p.nparts, p.eta, lt)
    co = cycles.CoarseSolver(Hs.A[Hs.L])
    s = amgdd.Solver(p.A, p.part, p.nparts, padding=p.eta, n_fac=2, hybrid_level=lt)
    g = np.random.default_rng(1).uniform(-1, 1, p.n)
    gt = _t(g)
    lam = torch.zeros_like(gt)
    lo = np.zeros(p.n)
    for k in range(4):
        lam, info, st = s.solve_adjoint(gt, lam, rtol=0, maxit=1)
        lo = cycles.hybrid_vcycle(HT, Hs, comps_s, lo, g, lt_, 2, coarse=co)
        err = rel_inf(_np(lam), lo)
        say(f"  hybrid iteration {k + 1}: max-entry rel err {err:.2e}")
        assert err <= 1e-12


def test_nonsymmetric_gradients_vs_central_differences():
    """L = ||u - u_t||^2, A(c) = diffusion(c(k)) + convection; dL/dc on 48
    seeded faces, dL/dk on 48 seeded cells, dL/df on all cells."""
    from paper_1906_10575_amd.autograd import FaceProblem, diffusion_solve, harmonic_face_coefficients
    dims = (14, 12, 10)
    k0 = np.exp(grf(dims, 0.5, 4.0, 2)).ravel()
    p = convection_diffusion_problem(dims, (2, 2, 2), velocity=(0.8, 0.4, -0.3), eta=1, n_fac=2,
                                     k=k0.reshape(dims[::-1]))
    C = p.extra["convection"]
    ut = np.random.default_rng(12).uniform(0, 1, p.n)
    say("nonsym gradients", p.n)
    fi = np.concatenate([p.faces.inner_i, p.faces.bnd_i])
    fj = np.concatenate([p.faces.inner_j, -np.ones(p.faces.bnd_i.size, dtype=np.int64)])
    prob = FaceProblem(p.n, fi, fj, p.part, p.nparts, padding=1, n_fac=2, rtol=1e-11, fixed=C)
    kt = _t(k0).requires_grad_(True)
    f = _t(p.b).requires_grad_(True)
    c = harmonic_face_coefficients(kt, fi, fj)
    c.retain_grad()
    u = diffusion_solve(c, f, prob)
    loss = ((u - _t(ut)) ** 2).sum()
    loss.backward()
    gk, gc, gf = _np(kt.grad), _np(c.grad), _np(f.grad)
    np.testing.assert_allclose(_np(c), face_coefficients(k0.reshape(dims[::-1]), p.faces), rtol=1e-15, atol=0)

    def loss_of(A, fv):
        uu = spla.splu(A.tocsc()).solve(fv)
        return float(np.sum((uu - ut) ** 2))

    A0 = prob.assemble(p.c)
    # same operator; the diagonal sums the face coefficients in another order
    assert abs(A0 - p.A).max() <= 1e-14 * abs(p.A).max()
    lam_d = adjoint.dense_adjoint(A0, 2 * (np.linalg.solve(A0.toarray(), p.b) - ut))
    assert rel_inf(gf, lam_d) <= 1e-8
    h = 1e-6
    rng = np.random.default_rng(3)
    sel = rng.choice(p.faces.n_faces, 48, replace=False)
    fd_c = []
    for kf in sel:
        cp, cm = p.c.copy(), p.c.copy()
        cp[kf] += h
        cm[kf] -= h
        fd_c.append((loss_of(prob.assemble(cp), p.b) - loss_of(prob.assemble(cm), p.b)) / (2 * h))
    fd_c = np.array(fd_c)
    err_c = np.abs(gc[sel] - fd_c).max() / np.abs(gc).max()
    cells = rng.choice(p.n, 48, replace=False)
    fd_k = []
    for i in cells:
        kp, km = k0.copy(), k0.copy()
        kp[i] += h
        km[i] -= h
        Ap = prob.assemble(face_coefficients(kp.reshape(dims[::-1]), p.faces))
        Am = prob.assemble(face_coefficients(km.reshape(dims[::-1]), p.faces))
        fd_k.append((loss_of(Ap, p.b) - loss_of(Am, p.b)) / (2 * h))
    fd_k = np.array(fd_k)
    err_k = np.abs(gk[cells] - fd_k).max() / np.abs(fd_k).max()
    say(f"  dL/dc vs FD {err_c:.2e}, dL/dk vs FD {err_k:.2e}")
    assert err_c <= 1e-6 and err_k <= 1e-6
