"""Oracle: multigrid cycles, plain serial FP64.

TEST INFRASTRUCTURE ONLY (see oracle/amg.py).

* vcycle          -- AMG V(nu1, nu2) cycle, Algorithm 1 of the paper, with
                     l1-Jacobi relaxation and a direct coarsest solve.
* algfac          -- the AlgFAC V-cycle, Algorithm 4 (Section 4.5), on one
                     composite grid, taken step by step in the paper's order
                     and notation (u_l, t_l, s_l, f_l).
* masked_vcycle   -- the plain definition AlgFAC must reproduce (guiding
                     principle of Section 4): a full-grid V-cycle on the
                     residual equation in which relaxation is suppressed
                     outside D_l on each level.
* amgdd           -- the AMG-DD outer iteration, Algorithm 2 (Section 3).
* hybrid_vcycle   -- the hybrid AMG-DD V-cycle, Algorithm 3 (Section 3.1):
                     V-cycle levels above a transition level, one AMG-DD
                     cycle on the transition level's problem as the coarse
                     solver (partition inherited along the C-points).

Relaxation is point l1-Jacobi with weight 1: u <- u + (f - A u) / d with
d_i = sum_j |a_ij| over the full row, in natural order (relax="l1": every
point at once) or CF order (relax="cf", the smoother of the paper's
experiments, Section 6): one Jacobi half-sweep over the C-points of the level
and then one over its F-points on the downsweep, F-points first on the
upsweep; each half-sweep sees the update of the one before.
"""

from __future__ import annotations

from typing import Callable, List, Optional, Sequence

import numpy as np
import scipy.linalg as sla

from .amg import C_PT, F_PT, Hierarchy
from .composite import CompositeGrid

C_FIRST = (C_PT, F_PT)  # CF order on the downsweep
F_FIRST = (F_PT, C_PT)  # and on the upsweep


class CoarseSolver:
    """Direct solve with A_L: LU with partial pivoting (Gaussian elimination)."""

    def __init__(self, AL):
        self.lu = sla.lu_factor(np.asarray(AL.toarray() if hasattr(AL, "toarray") else AL, dtype=np.float64))

    def __call__(self, f: np.ndarray) -> np.ndarray:
        return sla.lu_solve(self.lu, f)


def l1_relax(A, d, u, f, mask=None):
    """One l1-Jacobi sweep; returns the update delta (zero where mask is False)."""
    delta = (f - A @ u) / d
    if mask is not None:
        delta = np.where(mask, delta, 0.0)
    return delta


def smooth(A, d, u, f, mask=None, cls=None, order=None):
    """One l1-Jacobi sweep from u, returning the new iterate.  order None:
    every point at once.  Otherwise one half-sweep per class in `order`, over
    the points with cls == class (and mask), each from the iterate the
    previous half-sweep left."""
    if order is None:
        return u + l1_relax(A, d, u, f, mask)
    for c in order:
        m = cls == c if mask is None else (cls == c) & mask
        u = u + l1_relax(A, d, u, f, m)
    return u


def _orders(relax):
    if relax == "l1":
        return None, None
    if relax == "cf":
        return C_FIRST, F_FIRST
    raise ValueError(f"unknown relaxation {relax!r}")


def vcycle(H: Hierarchy, u0: np.ndarray, f0: np.ndarray, nu1: int = 1, nu2: int = 1,
           coarse: Optional[CoarseSolver] = None, relax: str = "l1") -> np.ndarray:
    """One AMG V(nu1, nu2) cycle on A_0 u = f_0 starting from u0 (Algorithm 1)."""
    down, up = _orders(relax)
    L = H.L
    coarse = coarse or CoarseSolver(H.A[L])
    d = [H.l1_diag(l) for l in range(L)]
    u = [None] * (L + 1)
    f = [None] * (L + 1)
    u[0] = np.array(u0, dtype=np.float64)
    f[0] = np.asarray(f0, dtype=np.float64)
    for l in range(L):
        for _ in range(nu1):
            u[l] = smooth(H.A[l], d[l], u[l], f[l], cls=H.cf[l], order=down)
        f[l + 1] = H.R[l] @ (f[l] - H.A[l] @ u[l])
        u[l + 1] = np.zeros(H.A[l + 1].shape[0])
    u[L] = coarse(f[L])
    for l in range(L - 1, -1, -1):
        u[l] = u[l] + H.P[l] @ u[l + 1]
        for _ in range(nu2):
            u[l] = smooth(H.A[l], d[l], u[l], f[l], cls=H.cf[l], order=up)
    return u[0]


def masked_vcycle(H: Hierarchy, masks: Sequence[np.ndarray], e0: np.ndarray, r0: np.ndarray,
                  n_cycles: int, coarse: Optional[CoarseSolver] = None, trace: Optional[list] = None,
                  relax: str = "l1"):
    """n_cycles V(1,1) cycles on A_0 e = r0 from e0 with relaxation applied only
    at masks[l] on level l; full-grid residual restriction, interpolation and
    exact coarsest solve.  Returns the list of level iterates after the last
    cycle (level l value just before it is interpolated from / returned).

    trace, if given, receives per cycle the list of restricted right-hand
    sides f_{l}, l >= 1, as seen on the downsweep."""
    down, up = _orders(relax)
    L = H.L
    coarse = coarse or CoarseSolver(H.A[L])
    d = [H.l1_diag(l) for l in range(L)]
    e = np.array(e0, dtype=np.float64)
    out = None
    for _ in range(n_cycles):
        u = [None] * (L + 1)
        f = [None] * (L + 1)
        u[0] = e
        f[0] = r0
        fs = []
        for l in range(L):
            u[l] = smooth(H.A[l], d[l], u[l], f[l], masks[l], H.cf[l], down)
            f[l + 1] = H.R[l] @ (f[l] - H.A[l] @ u[l])
            fs.append(f[l + 1])
            u[l + 1] = np.zeros(H.A[l + 1].shape[0])
        u[L] = coarse(f[L])
        for l in range(L - 1, -1, -1):
            u[l] = u[l] + H.P[l] @ u[l + 1]
            u[l] = smooth(H.A[l], d[l], u[l], f[l], masks[l], H.cf[l], up)
        e = u[0]
        out = u
        if trace is not None:
            trace.append(fs)
    return out


def algfac(cg: CompositeGrid, f_real: Sequence[np.ndarray], n_cycles: int, AL_solver: CoarseSolver,
           trace: Optional[list] = None, dtype=np.float64, cls: Optional[Sequence[np.ndarray]] = None,
           relax: str = "l1"):
    """AlgFAC V(1,1) cycles on one composite grid (Algorithm 4).

    f_real[l]: right-hand side at the real points of level l (local order).
    Returns (u, f): level corrections on Dbar_l and the final right-hand sides.

    Step order per cycle, as the algorithm states it:
      downsweep l = 0..L-1:
        u_l <- 0 if l != 0;  relax: u_l += delta1, t_l += delta1
        s_{l+1} <- R_l (s_l + A_l t_l)
        f_{l+1} <- f_{l+1} - A_{l+1} u_{l+1};  f_{l+1} <- f_{l+1} - s_{l+1}
        t_l <- 0, s_l <- 0
      coarse solve u_L <- A_L^{-1} f_L
      upsweep l = L-1..0: u_l += P_l u_{l+1};  relax: u_l += delta2, t_l += delta2

    `dtype` = np.float32 emulates the mixed-precision form: every composite
    array and every operation of the cycle in float32 except the coarsest
    solve, which upcasts f_L, solves in float64 and rounds u_L back.

    trace, if given, receives per cycle the right-hand sides f_{l} (real points,
    l >= 1) right after the subtraction of the restricted update.

    relax="cf": each relaxation is the CF-ordered sweep; cls[l] holds the C/F
    class of the real points of level l (l < L)."""
    lv = cg.levels
    L = cg.L
    T = dtype
    A = [x.A.astype(T) for x in lv]
    P = [x.P.astype(T) if x.P is not None else None for x in lv]
    R = [x.R.astype(T) if x.R is not None else None for x in lv]
    dd = [x.d.astype(T) for x in lv]
    nr = [x.n_real for x in lv]
    u = [np.zeros(x.n_bar, dtype=T) for x in lv]
    t = [np.zeros(x.n_bar, dtype=T) for x in lv]
    s = [np.zeros(x.n_bar, dtype=T) for x in lv]
    f = [np.array(fr, dtype=T) for fr in f_real]

    down, up = _orders(relax)

    def sweep(l, m=None):
        res = f[l] - (A[l] @ u[l])[: nr[l]]
        delta = (res / dd[l]).astype(T)
        if m is not None:
            delta = np.where(m, delta, T(0)).astype(T)
        u[l][: nr[l]] += delta
        t[l][: nr[l]] += delta

    def relax_l(l, order):
        if order is None:
            sweep(l)
        else:
            for c in order:
                sweep(l, cls[l] == c)

    for _ in range(n_cycles):
        fs = []
        for l in range(L):
            if l != 0:
                u[l][:] = 0
            relax_l(l, down)
            s[l + 1] = (R[l] @ (s[l] + A[l] @ t[l])).astype(T)
            f[l + 1] = f[l + 1] - (A[l + 1] @ u[l + 1])[: nr[l + 1]]
            f[l + 1] = f[l + 1] - s[l + 1][: nr[l + 1]]
            fs.append(f[l + 1].copy())
            t[l][:] = 0
            s[l][:] = 0
        u[L] = AL_solver(f[L].astype(np.float64)).astype(T)
        for l in range(L - 1, -1, -1):
            u[l] = u[l] + P[l] @ u[l + 1]
            relax_l(l, up)
        if trace is not None:
            trace.append(fs)
    return u, f


def restrict_all(H: Hierarchy, r0: np.ndarray, dtype=np.float64) -> List[np.ndarray]:
    """r_{l+1} = R_l r_l on every level (Algorithm 2, second step)."""
    rs = [np.asarray(r0).astype(dtype)]
    for l in range(H.L):
        rs.append((H.R[l].astype(dtype) @ rs[-1]).astype(dtype))
    return rs


def amgdd_iteration(H: Hierarchy, comps: Sequence[CompositeGrid], b: np.ndarray, x: np.ndarray,
                    n_fac: int, coarse: Optional[CoarseSolver] = None, dtype=np.float64,
                    relax: str = "l1") -> np.ndarray:
    """One AMG-DD cycle (Algorithm 2): fine residual, restriction to all levels,
    composite right-hand sides, n_fac AlgFAC cycles per subdomain, correction
    patched on each owned subdomain Omega_0^p.  Returns the new iterate.

    dtype = np.float32 emulates the mixed form: the residual and the patch stay
    float64, the restriction chain runs in float32 after rounding r_0."""
    coarse = coarse or CoarseSolver(H.A[H.L])
    r = b - H.A[0] @ x
    rs = restrict_all(H, r, dtype)
    xn = np.array(x, dtype=np.float64)
    for cg in comps:
        f = [rs[l][lev.gid[: lev.n_real]] for l, lev in enumerate(cg.levels)]
        cls = [H.cf[l][lev.gid[: lev.n_real]] for l, lev in enumerate(cg.levels[:-1])]
        u, _ = algfac(cg, f, n_fac, coarse, dtype=dtype, cls=cls, relax=relax)
        xn[cg.owned_gid] += u[0][cg.owned_local].astype(np.float64)
    return xn


def amgdd_solve(H, comps, b, x0, n_fac, rtol=1e-8, maxit=100, dtype=np.float64, callback=None, relax="l1"):
    """AMG-DD iterations until ||b - A x|| <= rtol ||b - A x0|| or maxit.
    Returns (x, residual-norm history)."""
    coarse = CoarseSolver(H.A[H.L])
    x = np.array(x0, dtype=np.float64)
    hist = [float(np.linalg.norm(b - H.A[0] @ x))]
    for _ in range(maxit):
        if hist[-1] <= rtol * hist[0]:
            break
        x = amgdd_iteration(H, comps, b, x, n_fac, coarse, dtype=dtype, relax=relax)
        if callback:
            callback(x)
        hist.append(float(np.linalg.norm(b - H.A[0] @ x)))
    return x, hist


def vcycle_solve(H, b, x0, rtol=1e-8, maxit=100, callback=None, relax="l1"):
    coarse = CoarseSolver(H.A[H.L])
    x = np.array(x0, dtype=np.float64)
    hist = [float(np.linalg.norm(b - H.A[0] @ x))]
    for _ in range(maxit):
        if hist[-1] <= rtol * hist[0]:
            break
        x = vcycle(H, x, b, coarse=coarse, relax=relax)
        if callback:
            callback(x)
        hist.append(float(np.linalg.norm(b - H.A[0] @ x)))
    return x, hist


def inherited_partition(H: Hierarchy, part: np.ndarray, level: int) -> np.ndarray:
    """Subdomain of every point of `level`: a coarse point is a C-point of the
    level above and keeps the subdomain of that point (Section 5: each
    processor's subdomain on level l is the part of Omega_l it owns)."""
    p = np.asarray(part)
    for l in range(level):
        p = p[H.cf[l] == 1]
    return p


def sub_hierarchy(H: Hierarchy, level: int) -> Hierarchy:
    """Levels `level`..L of H as a hierarchy of its own (A_level is its fine
    matrix)."""
    return Hierarchy(A=H.A[level:], P=H.P[level:], R=H.R[level:], cf=H.cf[level:], S=H.S[level:])


def hybrid_vcycle(H: Hierarchy, Hs: Hierarchy, comps_s, u0: np.ndarray, f0: np.ndarray, lt: int, n_fac: int,
                  coarse: Optional[CoarseSolver] = None, dtype=np.float64, relax: str = "l1") -> np.ndarray:
    """One hybrid AMG-DD V(1,1) cycle (Algorithm 3): V-cycle relaxation and
    residual restriction on levels 0..lt-1, one AMG-DD cycle (Algorithm 2,
    from a zero initial guess) on A_lt u_lt = f_lt as the coarse solver, then
    interpolation and relaxation back up.  Hs / comps_s: the hierarchy below
    lt and the composite grids built on it with the inherited partition.

    dtype = np.float32 runs the level-lt AMG-DD cycle in its mixed form (see
    amgdd_iteration); the V-cycle levels stay float64."""
    down, up = _orders(relax)
    coarse = coarse or CoarseSolver(Hs.A[Hs.L])
    d = [H.l1_diag(l) for l in range(lt)]
    u = [None] * (lt + 1)
    f = [None] * (lt + 1)
    u[0] = np.array(u0, dtype=np.float64)
    f[0] = np.asarray(f0, dtype=np.float64)
    for l in range(lt):
        u[l] = smooth(H.A[l], d[l], u[l], f[l], cls=H.cf[l], order=down)
        f[l + 1] = H.R[l] @ (f[l] - H.A[l] @ u[l])
        u[l + 1] = np.zeros(H.A[l + 1].shape[0])
    u[lt] = amgdd_iteration(Hs, comps_s, f[lt], np.zeros(H.A[lt].shape[0]), n_fac, coarse, dtype=dtype, relax=relax)
    for l in range(lt - 1, -1, -1):
        u[l] = u[l] + H.P[l] @ u[l + 1]
        u[l] = smooth(H.A[l], d[l], u[l], f[l], cls=H.cf[l], order=up)
    return u[0]


def hybrid_setup(H: Hierarchy, part: np.ndarray, nparts: int, eta, lt: int):
    """Level-lt AMG-DD problem of the hybrid cycle: the sub-hierarchy below
    lt (clamped to the coarsest level) and its composite grids over the
    inherited partition.  Returns (lt, Hs, comps)."""
    from .composite import build_all
    lt = min(lt, H.L)
    Hs = sub_hierarchy(H, lt)
    return lt, Hs, build_all(Hs, inherited_partition(H, part, lt), nparts, eta)


def hybrid_solve(H, Hs, comps_s, lt, b, x0, n_fac, rtol=1e-8, maxit=100, dtype=np.float64, callback=None,
                 relax="l1"):
    """Hybrid AMG-DD V-cycles in correction form, x <- x + C(b - A x), until
    ||b - A x|| <= rtol ||b - A x0|| or maxit.  Returns (x, history)."""
    coarse = CoarseSolver(Hs.A[Hs.L])
    x = np.array(x0, dtype=np.float64)
    hist = [float(np.linalg.norm(b - H.A[0] @ x))]
    for _ in range(maxit):
        if hist[-1] <= rtol * hist[0]:
            break
        r = b - H.A[0] @ x
        x = x + hybrid_vcycle(H, Hs, comps_s, np.zeros_like(r), r, lt, n_fac, coarse, dtype=dtype, relax=relax)
        if callback:
            callback(x)
        hist.append(float(np.linalg.norm(b - H.A[0] @ x)))
    return x, hist
