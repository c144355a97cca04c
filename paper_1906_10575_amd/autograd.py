"""Differentiable AMG-DD solve of a face-coefficient diffusion operator.

A(c) = sum_f c_f E_f + B with E_f = (e_i - e_j)(e_i - e_j)^T for an interior
face (i, j) and e_i e_i^T for a boundary face of cell i, and B an optional
fixed operator independent of c (for example upwind convection, which makes
A non-symmetric; the library then solves the adjoint with the transposed
composite operators).  Forward: assemble A(c) on
the host, build the hierarchy and composite grids (host setup in the
library), solve A u = f by AMG-DD on the device.  Backward (adjoint): solve
A^T lambda = dL/du by AMG-DD with the same hierarchy, then dL/df = lambda and
dL/dc_f = -(lambda_i - lambda_j)(u_i - u_j) (interior), -lambda_i u_i
(boundary), computed by the library's face-gradient kernel.  Gradients with
respect to cell coefficients k follow from torch's own autograd through
whatever differentiable map the caller uses for c(k).
"""

from __future__ import annotations

from dataclasses import dataclass
from typing import Optional

import numpy as np
import torch
from scipy import sparse

from .amgdd import OK, AmgddError, Solver


@dataclass
class FaceProblem:
    """Structure of the operator: n cells, face endpoints (face_j = -1 marks a
    boundary face), subdomain partition and AMG-DD parameters."""

    n: int
    face_i: np.ndarray
    face_j: np.ndarray
    part: np.ndarray
    nparts: int
    padding: int = 1
    n_fac: int = 2
    precision: str = "fp64"
    rtol: float = 1e-10
    maxit: int = 200
    fixed: Optional[sparse.csr_matrix] = None  # B: added to sum_f c_f E_f, independent of c

    def assemble(self, c: np.ndarray) -> sparse.csr_matrix:
        fi = np.asarray(self.face_i, dtype=np.int64)
        fj = np.asarray(self.face_j, dtype=np.int64)
        inner = fj >= 0
        diag = np.zeros(self.n)
        np.add.at(diag, fi, c)
        np.add.at(diag, fj[inner], c[inner])
        rows = np.concatenate([np.arange(self.n), fi[inner], fj[inner]])
        cols = np.concatenate([np.arange(self.n), fj[inner], fi[inner]])
        vals = np.concatenate([diag, -c[inner], -c[inner]])
        A = sparse.coo_matrix((vals, (rows, cols)), shape=(self.n, self.n)).tocsr()
        if self.fixed is not None:
            A = (A + self.fixed).tocsr()
        A.sum_duplicates()
        A.sort_indices()
        return A


class _DiffusionSolve(torch.autograd.Function):
    @staticmethod
    def forward(ctx, c, f, prob: FaceProblem):
        dev = f.device
        A = prob.assemble(c.detach().double().cpu().numpy())
        solver = Solver(A, prob.part, prob.nparts, padding=prob.padding, n_fac=prob.n_fac, precision=prob.precision,
                        device=dev.index or 0)
        u, info, st = solver.solve(f.detach().double().contiguous(), rtol=prob.rtol, maxit=prob.maxit)
        if st != OK:
            # an unconverged forward solve would give a wrong u and wrong gradients
            raise AmgddError(st, f"forward AMG-DD solve stopped at relative residual {info.relres:.3e} "
                                 f"after {info.iters} iterations (rtol {prob.rtol}, maxit {prob.maxit})")
        ctx.solver = solver
        ctx.prob = prob
        ctx.forward_info = info
        ctx.save_for_backward(u)
        return u

    @staticmethod
    def backward(ctx, gu):
        (u,) = ctx.saved_tensors
        prob = ctx.prob
        lam, info, st = ctx.solver.solve_adjoint(gu.detach().double().contiguous(), rtol=prob.rtol, maxit=prob.maxit)
        if st != OK:
            raise AmgddError(st, f"adjoint AMG-DD solve stopped at relative residual {info.relres:.3e} "
                                 f"after {info.iters} iterations (rtol {prob.rtol}, maxit {prob.maxit})")
        ctx.adjoint_info = info
        fi = torch.as_tensor(np.asarray(prob.face_i, dtype=np.int32), device=u.device)
        fj = torch.as_tensor(np.asarray(prob.face_j, dtype=np.int32), device=u.device)
        dc = ctx.solver.face_gradient(u, lam, fi, fj)
        return dc, lam, None


def diffusion_solve(c: torch.Tensor, f: torch.Tensor, prob: FaceProblem) -> torch.Tensor:
    """u = A(c)^{-1} f by AMG-DD, differentiable in c and f."""
    return _DiffusionSolve.apply(c, f, prob)


def harmonic_face_coefficients(k: torch.Tensor, face_i, face_j) -> torch.Tensor:
    """Face coefficients from cell coefficients as torch operations (so dL/dk
    follows from dL/dc by autograd): 2 k_i k_j / (k_i + k_j) for an interior
    face (i, j), k_i for a boundary face of cell i (face_j = -1)."""
    fi = torch.as_tensor(np.asarray(face_i, dtype=np.int64), device=k.device)
    fj = torch.as_tensor(np.asarray(face_j, dtype=np.int64), device=k.device)
    inner = fj >= 0
    ki = k[fi]
    kj = k[torch.where(inner, fj, fi)]
    return torch.where(inner, 2.0 * ki * kj / (ki + kj), ki)
