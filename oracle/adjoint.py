"""Oracle: dense adjoint of the diffusion solve, plain FP64.

TEST INFRASTRUCTURE ONLY (see oracle/amg.py).

For u = A(c)^{-1} f and a loss L(u), the adjoint lambda solves
A^T lambda = dL/du; then dL/df = lambda and, because A depends linearly on
the face coefficients (A = sum_f c_f E_f with E_f = (e_i - e_j)(e_i - e_j)^T
for an interior face and e_i e_i^T for a boundary face of cell i),
dL/dc_f = -lambda^T E_f u, i.e.
    interior face (i, j):  -(lambda_i - lambda_j)(u_i - u_j)
    boundary face of i:    -lambda_i u_i
This is the textbook derivative of a linear solve; the paper itself has no
adjoint.
"""

from __future__ import annotations

import numpy as np
import scipy.linalg as sla


def dense_solve(A, f):
    return sla.solve(np.asarray(A.toarray(), dtype=np.float64), np.asarray(f, dtype=np.float64))


def dense_adjoint(A, g):
    """lambda = A^{-T} g by a dense solve."""
    return sla.solve(np.asarray(A.toarray(), dtype=np.float64).T, np.asarray(g, dtype=np.float64))


def face_gradient(faces, u, lam):
    """dL/dc for every face (interior faces first, then boundary faces)."""
    u = np.asarray(u, dtype=np.float64)
    lam = np.asarray(lam, dtype=np.float64)
    gi = -(lam[faces.inner_i] - lam[faces.inner_j]) * (u[faces.inner_i] - u[faces.inner_j])
    gb = -lam[faces.bnd_i] * u[faces.bnd_i]
    return np.concatenate([gi, gb])


def loss_and_grads(A, faces, f, u_target):
    """L = ||u - u_target||^2 with u = A^{-1} f; returns (L, u, dL/df, dL/dc)."""
    u = dense_solve(A, f)
    g = 2.0 * (u - u_target)
    lam = dense_adjoint(A, g)
    return float(np.sum((u - u_target) ** 2)), u, lam, face_gradient(faces, u, lam)
