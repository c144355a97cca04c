"""Pins for the oracle's adjoint: central finite differences of the loss
through exact sparse solves, and the AMG-DD-solved adjoint against the dense
one."""

import numpy as np
import pytest
from scipy.sparse import linalg as spla

from oracle import adjoint, amg, composite, cycles
from synth import assemble, config, face_coefficients, grf, make_problem


def _loss(A, f, ut):
    u = spla.splu(A.tocsc()).solve(f)
    return float(np.sum((u - ut) ** 2))


@pytest.mark.parametrize("dims", [(5, 4, 4), (7, 6)])
def test_face_and_rhs_gradients_match_central_differences(dims):
    k = np.exp(grf(dims, 0.5, 2.0, 2))
    p = make_problem(dims, [1] * len(dims), k=k, rhs_range=(0.0, 1.0))
    rng = np.random.default_rng(4)
    ut = rng.uniform(0, 1, p.n)
    L, u, lam, gc = adjoint.loss_and_grads(p.A, p.faces, p.b, ut)
    h = 1e-6
    fd_c = np.empty(p.faces.n_faces)
    for f in range(p.faces.n_faces):
        cp = p.c.copy()
        cp[f] += h
        cm = p.c.copy()
        cm[f] -= h
        fd_c[f] = (_loss(assemble(p.n, p.faces, cp), p.b, ut) - _loss(assemble(p.n, p.faces, cm), p.b, ut)) / (2 * h)
    assert np.abs(gc - fd_c).max() <= 1e-6 * np.abs(fd_c).max()
    fd_f = np.empty(p.n)
    for i in range(p.n):
        fp = p.b.copy()
        fp[i] += h
        fm = p.b.copy()
        fm[i] -= h
        fd_f[i] = (_loss(p.A, fp, ut) - _loss(p.A, fm, ut)) / (2 * h)
    assert np.abs(lam - fd_f).max() <= 1e-6 * np.abs(fd_f).max()


def test_cell_coefficient_chain_rule():
    # dL/dk through the harmonic-mean face coefficients, against differences in k
    dims = (6, 5)
    k = np.exp(grf(dims, 0.5, 2.0, 8)).ravel()
    p = make_problem(dims, (1, 1), k=k.reshape(5, 6), rhs_range=(0.0, 1.0))
    ut = np.random.default_rng(1).uniform(0, 1, p.n)
    _, u, lam, gc = adjoint.loss_and_grads(p.A, p.faces, p.b, ut)
    fi, fj, fb = p.faces.inner_i, p.faces.inner_j, p.faces.bnd_i
    ni = fi.size
    dk = np.zeros(p.n)
    # dc/dk_i = 2 k_j^2 / (k_i + k_j)^2 on an interior face, 1 on a boundary face
    np.add.at(dk, fi, gc[:ni] * 2 * k[fj] ** 2 / (k[fi] + k[fj]) ** 2)
    np.add.at(dk, fj, gc[:ni] * 2 * k[fi] ** 2 / (k[fi] + k[fj]) ** 2)
    np.add.at(dk, fb, gc[ni:])
    h = 1e-6
    fd = np.empty(p.n)
    for i in range(p.n):
        kp = k.copy()
        kp[i] += h
        km = k.copy()
        km[i] -= h
        Ap = assemble(p.n, p.faces, face_coefficients(kp, p.faces))
        Am = assemble(p.n, p.faces, face_coefficients(km, p.faces))
        fd[i] = (_loss(Ap, p.b, ut) - _loss(Am, p.b, ut)) / (2 * h)
    assert np.abs(dk - fd).max() <= 1e-6 * np.abs(fd).max()


def test_amgdd_adjoint_matches_dense():
    p = config("cfg4", scale=12)
    ut = p.extra["u_target"]
    _, u, lam_dense, _ = adjoint.loss_and_grads(p.A, p.faces, p.b, ut)
    H = amg.setup(p.A)
    comps = composite.build_all(H, p.part, p.nparts, p.eta)
    u_dd, _ = cycles.amgdd_solve(H, comps, p.b, np.zeros(p.n), n_fac=2, rtol=1e-13, maxit=200)
    g = 2 * (u_dd - ut)
    lam, _ = cycles.amgdd_solve(H, comps, g, np.zeros(p.n), n_fac=2, rtol=1e-13, maxit=200)
    assert np.linalg.norm(lam - lam_dense) <= 1e-10 * np.linalg.norm(lam_dense)
