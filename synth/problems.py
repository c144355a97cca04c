"""Seeded synthetic inputs for the AMG-DD solve phase.

This module builds the *inputs* of the method only: structured-grid diffusion
operators (cell-centred finite differences, homogeneous Dirichlet nodes
eliminated), log-normal coefficient fields, block partitions into subdomains,
right-hand sides and face lists.  It contains none of the multigrid arithmetic
(no coarsening, interpolation, composite grids or cycles); both the oracle and
the GPU path consume what it returns.

The paper's workloads (Section 6) are finite-element discretisations of
-div(K grad u) = f on regular meshes partitioned by METIS; these generators
stand in for them with 5-point (2D) and 7-point (3D) stencils on block
partitions, and (Problem 2, the rotated anisotropic case) with bilinear
finite elements on a regular square mesh of the unit square.

Conventions
-----------
* Grid points are numbered lexicographically with x fastest:
  i = x + nx*y (+ nx*ny*z).  Arrays of grid values have numpy shape
  (nz, ny, nx) / (ny, nx) so that C-order flattening gives that numbering.
* Face coefficient of an interior face (i, j): harmonic mean
  2 k_i k_j / (k_i + k_j).  Face coefficient of a boundary face of cell i: k_i.
* A_ii = sum of the coefficients of the faces of i; A_ij = -c_f for the
  interior face f = (i, j).  No h^-2 scaling.  With k == 1 this is the
  standard 5/7-point Laplacian (diagonal 4/6, off-diagonals -1).
"""

from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Optional, Sequence, Tuple

import numpy as np
from scipy import ndimage, sparse

__all__ = [
    "Faces",
    "Problem",
    "grid_faces",
    "face_coefficients",
    "assemble",
    "grf",
    "block_partition",
    "uniform_rhs",
    "make_problem",
    "config",
    "batch_config",
    "anisotropic_tensor",
    "q1_stiffness",
    "anisotropic_problem",
    "isolated_column_problem",
    "upwind_convection",
    "convection_diffusion_problem",
    "CONFIG_NAMES",
]


@dataclass
class Faces:
    """Face list of a structured grid.

    inner_i, inner_j : int64 arrays, the two cells of each interior face (i < j)
    bnd_i            : int64 array, the cell of each boundary face (a corner
                       cell appears once per boundary side it touches)
    """

    inner_i: np.ndarray
    inner_j: np.ndarray
    bnd_i: np.ndarray

    @property
    def n_inner(self) -> int:
        return int(self.inner_i.size)

    @property
    def n_faces(self) -> int:
        return int(self.inner_i.size + self.bnd_i.size)


def _np_shape(dims: Sequence[int]) -> Tuple[int, ...]:
    # dims are given as (nx, ny[, nz]); numpy arrays use the reversed order
    return tuple(int(d) for d in reversed(dims))


def grid_faces(dims: Sequence[int]) -> Faces:
    """Interior and boundary faces of an nx x ny (x nz) cell grid."""
    shape = _np_shape(dims)
    n = int(np.prod(shape))
    idx = np.arange(n, dtype=np.int64).reshape(shape)
    inner_i, inner_j, bnd = [], [], []
    nd = len(shape)
    # axis order: x (last numpy axis) first, then y, then z
    for ax in range(nd - 1, -1, -1):
        lo = [slice(None)] * nd
        hi = [slice(None)] * nd
        lo[ax] = slice(0, shape[ax] - 1)
        hi[ax] = slice(1, shape[ax])
        inner_i.append(idx[tuple(lo)].ravel())
        inner_j.append(idx[tuple(hi)].ravel())
        first = [slice(None)] * nd
        last = [slice(None)] * nd
        first[ax] = 0
        last[ax] = shape[ax] - 1
        bnd.append(idx[tuple(first)].ravel())
        bnd.append(idx[tuple(last)].ravel())
    return Faces(np.concatenate(inner_i), np.concatenate(inner_j), np.concatenate(bnd))


def face_coefficients(k: np.ndarray, faces: Faces) -> np.ndarray:
    """Face coefficients: harmonic mean of the two cells for interior faces,
    the cell value for boundary faces.  Returned in face order
    (interior faces first, then boundary faces)."""
    kf = np.asarray(k, dtype=np.float64).ravel()
    ki = kf[faces.inner_i]
    kj = kf[faces.inner_j]
    c_in = 2.0 * ki * kj / (ki + kj)
    c_bd = kf[faces.bnd_i]
    return np.concatenate([c_in, c_bd])


def assemble(n: int, faces: Faces, c: np.ndarray) -> sparse.csr_matrix:
    """CSR matrix of the diffusion operator for face coefficients c.

    Rows have sorted column indices, int32 indices, float64 values.  The
    diagonal accumulates face coefficients in face order."""
    c = np.asarray(c, dtype=np.float64)
    ni = faces.n_inner
    c_in = c[:ni]
    c_bd = c[ni:]
    diag = np.zeros(n, dtype=np.float64)
    np.add.at(diag, faces.inner_i, c_in)
    np.add.at(diag, faces.inner_j, c_in)
    np.add.at(diag, faces.bnd_i, c_bd)
    rows = np.concatenate([np.arange(n), faces.inner_i, faces.inner_j])
    cols = np.concatenate([np.arange(n), faces.inner_j, faces.inner_i])
    vals = np.concatenate([diag, -c_in, -c_in])
    A = sparse.coo_matrix((vals, (rows, cols)), shape=(n, n)).tocsr()
    A.sum_duplicates()
    A.sort_indices()
    A.indices = A.indices.astype(np.int32)
    A.indptr = A.indptr.astype(np.int32)
    return A


def grf(dims: Sequence[int], sigma: float, corr_len: float, seed: int) -> np.ndarray:
    """Gaussian random field with squared-exponential covariance
    exp(-r^2 / (2 l^2)), l = corr_len cells, periodic filtering, standardised
    to zero mean and standard deviation sigma.  Returns numpy shape
    (nz, ny, nx) / (ny, nx)."""
    rng = np.random.default_rng(seed)
    shape = _np_shape(dims)
    w = rng.standard_normal(shape)
    g = ndimage.gaussian_filter(w, sigma=corr_len / np.sqrt(2.0), mode="wrap", truncate=4.0)
    g = (g - g.mean()) / g.std()
    return sigma * g


def block_partition(dims: Sequence[int], parts: Sequence[int]) -> np.ndarray:
    """Subdomain id of every grid point for a block partition with parts[a]
    blocks along axis a (x first).  Block coordinate along an axis of length n
    with P blocks is floor(x * P / n); ids are lexicographic over block
    coordinates, x fastest."""
    dims = [int(d) for d in dims]
    parts = [int(p) for p in parts]
    assert len(dims) == len(parts)
    coords = np.meshgrid(*[np.arange(d) for d in reversed(dims)], indexing="ij")
    # coords[0] is the slowest axis (z or y), coords[-1] is x
    bid = np.zeros(_np_shape(dims), dtype=np.int64)
    stride = 1
    for a in range(len(dims)):
        x = coords[len(dims) - 1 - a]
        bc = (x * parts[a]) // dims[a]
        bid += bc * stride
        stride *= parts[a]
    return bid.ravel().astype(np.int32)


def uniform_rhs(n: int, seed: int, lo: float = -1.0, hi: float = 1.0) -> np.ndarray:
    rng = np.random.default_rng(seed)
    return rng.uniform(lo, hi, size=n)


@dataclass
class Problem:
    """One linear system A u = b with its subdomain partition and solver
    parameters.  `k` is the cell coefficient field (None for k == 1)."""

    name: str
    dims: Tuple[int, ...]
    A: sparse.csr_matrix
    b: np.ndarray
    part: np.ndarray
    nparts: int
    eta: int
    n_fac: int
    faces: Faces
    c: np.ndarray
    k: Optional[np.ndarray] = None
    extra: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return int(self.A.shape[0])


def make_problem(
    dims: Sequence[int],
    parts: Sequence[int],
    eta: int = 1,
    n_fac: int = 1,
    k: Optional[np.ndarray] = None,
    rhs_seed: int = 0,
    rhs_range: Tuple[float, float] = (-1.0, 1.0),
    name: str = "",
) -> Problem:
    dims = tuple(int(d) for d in dims)
    n = int(np.prod(dims))
    faces = grid_faces(dims)
    kk = np.ones(_np_shape(dims)) if k is None else np.asarray(k, dtype=np.float64)
    c = face_coefficients(kk, faces)
    A = assemble(n, faces, c)
    b = uniform_rhs(n, rhs_seed, *rhs_range)
    part = block_partition(dims, parts)
    return Problem(
        name=name or "x".join(map(str, dims)),
        dims=dims,
        A=A,
        b=b,
        part=part,
        nparts=int(np.prod(parts)),
        eta=int(eta),
        n_fac=int(n_fac),
        faces=faces,
        c=c,
        k=None if k is None else kk,
    )


def upwind_convection(dims: Sequence[int], velocity: Sequence[float]) -> sparse.csr_matrix:
    """First-order upwind convection b . grad u on the cell grid (unscaled, as
    the diffusion operator): for each axis with velocity b_a != 0, row i gets
    +|b_a| on the diagonal and -|b_a| at its upstream neighbour (x - 1 for
    b_a > 0, x + 1 for b_a < 0) when that neighbour is inside the grid
    (homogeneous Dirichlet outside).  Off-diagonals are non-positive and every
    interior row sums to zero; the matrix is not symmetric, and its pattern
    lies inside the 5/7-point stencil."""
    dims = tuple(int(d) for d in dims)
    n = int(np.prod(dims))
    idx = np.arange(n).reshape(_np_shape(dims))
    rows, cols, vals = [np.arange(n)], [np.arange(n)], [np.zeros(n)]
    for a, b in enumerate(velocity):
        if b == 0.0:
            continue
        ax = len(dims) - 1 - a  # numpy axis of grid axis a (x is the last)
        vals[0] = vals[0] + abs(b)
        src = [slice(None)] * len(dims)
        dst = [slice(None)] * len(dims)
        if b > 0:
            dst[ax], src[ax] = slice(1, None), slice(None, -1)
        else:
            dst[ax], src[ax] = slice(None, -1), slice(1, None)
        rows.append(idx[tuple(dst)].ravel())
        cols.append(idx[tuple(src)].ravel())
        vals.append(np.full(rows[-1].size, -abs(b)))
    C = sparse.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))), shape=(n, n)).tocsr()
    C.sum_duplicates()
    C.sort_indices()
    return C


def convection_diffusion_problem(dims: Sequence[int], parts: Sequence[int], velocity: Sequence[float] = (1.0, 0.5),
                                 eta: int = 1, n_fac: int = 2, k: Optional[np.ndarray] = None, rhs_seed: int = 0,
                                 name: str = "") -> Problem:
    """Diffusion (face coefficients c from k, as make_problem) plus upwind
    convection: A = A_diff(c) + C.  A non-symmetric M-matrix whose stored
    pattern is the symmetric 5/7-point pattern of A_diff (C's entries fall on
    it).  C does not depend on c; it is kept in extra["convection"]."""
    p = make_problem(dims, parts, eta=eta, n_fac=n_fac, k=k, rhs_seed=rhs_seed, name=name or "convdiff")
    C = upwind_convection(p.dims, velocity)
    A = (p.A + C).tocsr()
    A.sum_duplicates()
    A.sort_indices()
    A.indices = A.indices.astype(np.int32)
    A.indptr = A.indptr.astype(np.int32)
    assert A.nnz == p.A.nnz, "convection entries must fall on the diffusion pattern"
    p.A = A
    p.extra["convection"] = C
    p.extra["velocity"] = tuple(float(v) for v in velocity)
    return p


def isolated_column_problem(dims: Sequence[int] = (40, 40), parts: Sequence[int] = (2, 2), col: Optional[int] = None,
                            eta: int = 1, n_fac: int = 2, rhs_seed: int = 0, name: str = "") -> Problem:
    """2D 5-point operator (diagonal 4, couplings -1) in which every point of
    one grid column x = col couples to its four neighbours with +0.25 instead
    (symmetric, strictly diagonally dominant, so SPD).  Those points have no
    negative coupling at all, so no strength-of-connection rule links them to
    anything: they become F-points with empty interpolation rows, and the
    grids to their left and right fall apart on every coarse level.  A
    subdomain whose padding reaches across the column then has ghost points
    whose interpolation columns lie outside its coarse composite grid: the
    omitted entries of Section 4.2 (its Figure 4 draws such a point)."""
    dims = tuple(int(d) for d in dims)
    nx, ny = dims
    col = nx // 2 - 1 if col is None else int(col)
    n = nx * ny
    idx = np.arange(n).reshape(ny, nx)
    xs = np.tile(np.arange(nx), ny)
    rows, cols, vals = [np.arange(n)], [np.arange(n)], [np.full(n, 4.0)]
    for a_, b_ in ((idx[:, :-1].ravel(), idx[:, 1:].ravel()), (idx[:-1, :].ravel(), idx[1:, :].ravel())):
        c = np.where((xs[a_] == col) | (xs[b_] == col), 0.25, -1.0)
        rows += [a_, b_]
        cols += [b_, a_]
        vals += [c, c]
    A = sparse.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))), shape=(n, n))
    A.sort_indices()
    empty = np.zeros(0, dtype=np.int64)
    return Problem(name=name or f"isolated_column{nx}x{ny}", dims=dims, A=A, b=uniform_rhs(n, rhs_seed),
                   part=block_partition(dims, parts), nparts=int(np.prod(parts)), eta=int(eta), n_fac=int(n_fac),
                   faces=Faces(empty, empty, empty), c=np.zeros(0), extra={"column": col})


def anisotropic_tensor(theta: float, eps: float) -> np.ndarray:
    """K = Q^T D Q with Q the rotation [[cos, sin], [-sin, cos]] by theta and
    D = diag(1, eps) (Problem 2 of the paper's experiments)."""
    c, s = np.cos(theta), np.sin(theta)
    Q = np.array([[c, s], [-s, c]])
    return Q.T @ np.diag([1.0, eps]) @ Q


def q1_stiffness(dims: Sequence[int], K: np.ndarray) -> sparse.csr_matrix:
    """Bilinear (Q1) finite-element stiffness matrix of -div(K grad u) for a
    constant 2x2 tensor K on the unit square, meshed with (nx+1) x (ny+1)
    rectangles; homogeneous Dirichlet nodes eliminated, so the unknowns are
    the nx x ny interior nodes, numbered x fastest.  Element matrices by 2x2
    Gauss quadrature (exact for these integrands)."""
    nx, ny = (int(d) for d in dims)
    hx, hy = 1.0 / (nx + 1), 1.0 / (ny + 1)
    # reference nodes (0,0), (1,0), (1,1), (0,1)
    corners = [(0, 0), (1, 0), (1, 1), (0, 1)]

    def grad(a, xi, et):
        cx, cy = corners[a]
        gx = (1.0 if cx else -1.0) * (et if cy else 1.0 - et)
        gy = (1.0 if cy else -1.0) * (xi if cx else 1.0 - xi)
        return np.array([gx / hx, gy / hy])

    g = [0.5 - 0.5 / np.sqrt(3.0), 0.5 + 0.5 / np.sqrt(3.0)]
    Ke = np.zeros((4, 4))
    for xi in g:
        for et in g:
            G = [grad(a, xi, et) for a in range(4)]
            for a in range(4):
                for b in range(4):
                    Ke[a, b] += 0.25 * hx * hy * (G[a] @ K @ G[b])
    Ke = 0.5 * (Ke + Ke.T)  # exactly symmetric (the two products round differently)
    # elements (ex, ey), ex in 0..nx, ey in 0..ny; mesh node (ix, iy), interior
    # when 1 <= ix <= nx and 1 <= iy <= ny, unknown index (ix-1) + nx (iy-1)
    ex, ey = np.meshgrid(np.arange(nx + 1), np.arange(ny + 1), indexing="xy")
    ex, ey = ex.ravel(), ey.ravel()
    rows, cols, vals = [], [], []
    for a in range(4):
        ax, ay = corners[a]
        ia, ja = ex + ax, ey + ay
        ina = (ia >= 1) & (ia <= nx) & (ja >= 1) & (ja <= ny)
        for b in range(4):
            bx, by = corners[b]
            ib, jb = ex + bx, ey + by
            m = ina & (ib >= 1) & (ib <= nx) & (jb >= 1) & (jb <= ny)
            rows.append((ia[m] - 1) + nx * (ja[m] - 1))
            cols.append((ib[m] - 1) + nx * (jb[m] - 1))
            vals.append(np.full(int(m.sum()), Ke[a, b]))
    n = nx * ny
    A = sparse.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))), shape=(n, n)).tocsr()
    A.sum_duplicates()
    A.sort_indices()
    A.indices = A.indices.astype(np.int32)
    A.indptr = A.indptr.astype(np.int32)
    return A


def anisotropic_problem(dims: Sequence[int], parts: Sequence[int], theta: float = 3 * np.pi / 16, eps: float = 1e-3,
                        eta: int = 1, n_fac: int = 2, rhs_seed: int = 0, name: str = "") -> Problem:
    """Problem 2 stand-in: 2D rotated anisotropic diffusion, K = Q^T D Q
    (theta = 3 pi / 16, eps = 1e-3 by default), Q1 elements on the unit
    square, block partition, b ~ U[-1, 1]."""
    dims = tuple(int(d) for d in dims)
    A = q1_stiffness(dims, anisotropic_tensor(theta, eps))
    n = A.shape[0]
    empty = np.zeros(0, dtype=np.int64)
    return Problem(name=name or "aniso" + "x".join(map(str, dims)), dims=dims, A=A, b=uniform_rhs(n, rhs_seed),
                   part=block_partition(dims, parts), nparts=int(np.prod(parts)), eta=int(eta), n_fac=int(n_fac),
                   faces=Faces(empty, empty, empty), c=np.zeros(0),
                   extra={"theta": float(theta), "eps": float(eps)})


CONFIG_NAMES = ("cfg1", "cfg2", "cfg3", "cfg4", "cfg5", "p2")


def config(name: str, scale: Optional[int] = None) -> Problem:
    """The named single-problem workloads.

    cfg1  2D 5-point Laplacian, 64^2, 2x2 subdomains, padding 1, 1 FAC cycle
    cfg2  3D 7-point Laplacian, 128^3, 4^3 subdomains of 32^3, padding 1, 2 FAC cycles
    cfg3  3D 7-point diffusion, 192^3, k = exp(GRF sigma 1, l = 8, seed 1),
          8^3 subdomains of 24^3, padding 2, 2 FAC cycles
    cfg4  3D 7-point diffusion, 96^3, k = exp(GRF sigma 0.5, l = 8, seed 2),
          f ~ U[0,1] (seed 3), 3^3 subdomains of 32^3, padding 1, 2 FAC cycles;
          extra['u_target'] ~ U[0,1] (seed 4)
    p2    2D rotated anisotropic diffusion (theta = 3 pi/16, eps = 1e-3), Q1
          elements, 1024^2 interior nodes, 4x4 subdomains of 256^2, padding 1,
          2 FAC cycles

    `scale` replaces the grid side while keeping the subdomain count (reduced
    instances for tests)."""
    if name == "cfg1":
        s = scale or 64
        return make_problem((s, s), (2, 2), eta=1, n_fac=1, rhs_seed=0, name="cfg1")
    if name == "cfg2":
        s = scale or 128
        return make_problem((s, s, s), (4, 4, 4), eta=1, n_fac=2, rhs_seed=0, name="cfg2")
    if name == "cfg3":
        s = scale or 192
        dims = (s, s, s)
        k = np.exp(grf(dims, 1.0, 8.0, seed=1))
        return make_problem(dims, (8, 8, 8), eta=2, n_fac=2, k=k, rhs_seed=0, name="cfg3")
    if name == "cfg4":
        s = scale or 96
        dims = (s, s, s)
        k = np.exp(grf(dims, 0.5, 8.0, seed=2))
        parts = (3, 3, 3) if s >= 24 else (2, 2, 2)
        p = make_problem(dims, parts, eta=1, n_fac=2, k=k, rhs_seed=3, rhs_range=(0.0, 1.0), name="cfg4")
        p.extra["u_target"] = uniform_rhs(p.n, 4, 0.0, 1.0)
        return p
    if name == "p2":
        s = scale or 1024
        return anisotropic_problem((s, s), (4, 4), eta=1, n_fac=2, rhs_seed=0, name="p2")
    raise KeyError(name)


def batch_config(n_problems: int = 256, seed0: int = 5000, side_range=(64, 512), parts_range=(2, 8),
                 eta_range=(1, 3)) -> List[Problem]:
    """Batched uneven workload: independent 2D 5-point diffusion problems.

    Problem i draws from default_rng(seed0 + i): side s ~ U{lo..hi} (square
    s x s grid), blocks Px, Py ~ U{2..8}, padding eta ~ U{1..3}; k = exp(GRF
    sigma 1, l = 8) and b ~ U[-1, 1] from further seeds derived from the same
    generator."""
    probs = []
    for i in range(n_problems):
        rng = np.random.default_rng(seed0 + i)
        s = int(rng.integers(side_range[0], side_range[1] + 1))
        px = int(rng.integers(parts_range[0], parts_range[1] + 1))
        py = int(rng.integers(parts_range[0], parts_range[1] + 1))
        eta = int(rng.integers(eta_range[0], eta_range[1] + 1))
        kseed = int(rng.integers(0, 2**31 - 1))
        bseed = int(rng.integers(0, 2**31 - 1))
        px = min(px, s)
        py = min(py, s)
        dims = (s, s)
        k = np.exp(grf(dims, 1.0, 8.0, seed=kseed))
        probs.append(make_problem(dims, (px, py), eta=eta, n_fac=2, k=k, rhs_seed=bseed, name=f"b{i}"))
    return probs
