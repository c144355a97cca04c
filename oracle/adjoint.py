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

The AMG-DD adjoint solve uses the forward hierarchy transposed
(transposed_hierarchy): the paper's hierarchy has R_l = P_l^T and
A_{l+1} = R_l A_l P_l (Section 2), hence A_{l+1}^T = R_l A_l^T P_l, so the
same C/F splittings, P_l and R_l form a Galerkin hierarchy for A^T with
operators A_l^T; its l1-Jacobi diagonals are then sum_j |(A_l^T)_ij| and its
coarsest solve is with A_L^T.  The composite sets (Section 3) depend only on
the undirected graph of A_l, which A_l^T shares.  AMG-DD (Algorithm 2) on that
hierarchy is the adjoint iteration.
"""

from __future__ import annotations

import numpy as np
import scipy.linalg as sla

from .amg import Hierarchy


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


def transposed_hierarchy(H: Hierarchy) -> Hierarchy:
    """The Galerkin hierarchy of A^T with the forward C/F splittings, P_l and
    R_l = P_l^T: operators A_l^T (explicit transposes, sorted columns)."""
    AT = []
    for A in H.A:
        T = A.T.tocsr()
        T.sort_indices()
        AT.append(T)
    return Hierarchy(A=AT, P=list(H.P), R=list(H.R), cf=list(H.cf), S=list(H.S))
