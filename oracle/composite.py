"""Oracle: AMG-DD composite grids, plain serial.

TEST INFRASTRUCTURE ONLY (see oracle/amg.py).

Composite-grid construction (Section 3 and its Figure 1): subdomain p's
level-0 real set D_0 is its subdomain Omega_0^p plus every point within graph
distance eta_0 in the graph of A_0; D_{l+1} is the set of C-points of D_l
(mapped to level l+1) plus every point within distance eta_{l+1} in the graph
of A_{l+1}; the coarsest level is stored whole.  The ghost extension
(Section 4.1) is Dbar_l = D_l plus every point j with a_ij stored for some
i in D_l.

Readings: the graph of A_l is its stored (symbolic) pattern without the
diagonal; the coarsest padding is infinite (D_L = Omega_L); the same padding
eta is used on every level below L unless a per-level list is given.

Local operators (Sections 4.1-4.4): A_l restricted to rows and columns in
Dbar_l; P_l restricted to rows in Dbar_l and columns in Dbar_{l+1}, columns
outside Dbar_{l+1} dropped and counted ("omissions", the connectivity
assumption of Section 4.2); R_l is the transpose of the kept P_l.

Local numbering: real points first in increasing global id, then ghost points
in increasing global id.
"""

from __future__ import annotations

from dataclasses import dataclass
from typing import List, Optional, Sequence

import numpy as np
from scipy import sparse
from scipy.sparse import csgraph

from .amg import C_PT, Hierarchy


def adjacency(A: sparse.csr_matrix) -> sparse.csr_matrix:
    """Undirected graph of the stored pattern of A without the diagonal."""
    G = sparse.csr_matrix((np.ones(A.nnz, dtype=np.int8), A.indices.copy(), A.indptr.copy()), shape=A.shape)
    G = ((G + G.T) > 0).astype(np.int8).tocsr()
    G.setdiag(0)
    G.eliminate_zeros()
    G.sort_indices()
    return G


def bfs_ball(G: sparse.csr_matrix, seeds: np.ndarray, eta: int) -> np.ndarray:
    """Boolean mask of points at graph distance <= eta from the seed mask,
    by eta rounds of level-synchronous frontier expansion."""
    inside = seeds.astype(bool).copy()
    frontier = inside.copy()
    for _ in range(int(eta)):
        if not frontier.any():
            break
        reach = (G @ frontier.astype(np.int8)) > 0
        new = reach & ~inside
        inside |= new
        frontier = new
    return inside


def ball_all_pairs(G: sparse.csr_matrix, seeds: np.ndarray, eta: int) -> np.ndarray:
    """Same set as bfs_ball from all-pairs unweighted shortest paths
    (tiny graphs only)."""
    D = csgraph.shortest_path(G, unweighted=True, directed=False)
    s = np.nonzero(seeds)[0]
    if s.size == 0:
        return np.zeros(G.shape[0], dtype=bool)
    return D[:, s].min(axis=1) <= eta


def neighbours(G: sparse.csr_matrix, mask: np.ndarray) -> np.ndarray:
    return (G @ mask.astype(np.int8)) > 0


def coarse_map(cf: np.ndarray) -> np.ndarray:
    """Fine index -> coarse index for C-points (-1 for F-points)."""
    is_c = cf == C_PT
    cm = np.full(cf.size, -1, dtype=np.int64)
    cm[is_c] = np.arange(int(is_c.sum()))
    return cm


def composite_sets(H: Hierarchy, part: np.ndarray, p: int, eta, brute: bool = False):
    """Real sets D_l and ghost-extended sets Dbar_l (boolean masks over
    Omega_l) of subdomain p on every level.

    eta: int (same padding on every level below the coarsest) or a sequence
    with one padding per level."""
    L = H.L
    etas = [int(eta)] * (L + 1) if np.isscalar(eta) else [int(e) for e in eta]
    ball = ball_all_pairs if brute else bfs_ball
    D, Dbar = [], []
    graphs = [adjacency(A) for A in H.A]
    seed = np.asarray(part) == p
    for l in range(L + 1):
        n = H.A[l].shape[0]
        if l == L:
            d = np.ones(n, dtype=bool)
        else:
            d = ball(graphs[l], seed, etas[l])
        D.append(d)
        Dbar.append(d | neighbours(graphs[l], d))
        if l < L:
            cm = coarse_map(H.cf[l])
            sel = np.nonzero(d & (H.cf[l] == C_PT))[0]
            seed = np.zeros(H.A[l + 1].shape[0], dtype=bool)
            seed[cm[sel]] = True
    return D, Dbar


@dataclass
class CompositeLevel:
    gid: np.ndarray          # global ids on level l, real first (sorted) then ghost (sorted)
    n_real: int
    A: sparse.csr_matrix     # A_l[Dbar, Dbar] in local numbering
    d: np.ndarray            # l1 diagonal at real points (full global row)
    P: Optional[sparse.csr_matrix]  # P_l[Dbar_l, Dbar_{l+1}] local numbering (None at L)
    R: Optional[sparse.csr_matrix]  # transpose of P
    omissions: int = 0       # P entries dropped because the column is outside Dbar_{l+1}

    @property
    def n_bar(self) -> int:
        return int(self.gid.size)


@dataclass
class CompositeGrid:
    p: int
    levels: List[CompositeLevel]
    owned_local: np.ndarray  # local level-0 indices of the owned points Omega_0^p
    owned_gid: np.ndarray    # their global ids

    @property
    def L(self) -> int:
        return len(self.levels) - 1


def local_order(D: np.ndarray, Dbar: np.ndarray) -> np.ndarray:
    real = np.nonzero(D)[0]
    ghost = np.nonzero(Dbar & ~D)[0]
    return np.concatenate([real, ghost])


def build_composite(H: Hierarchy, part: np.ndarray, p: int, eta, brute: bool = False) -> CompositeGrid:
    D, Dbar = composite_sets(H, part, p, eta, brute=brute)
    L = H.L
    gids = [local_order(D[l], Dbar[l]) for l in range(L + 1)]
    levels = []
    for l in range(L + 1):
        g = gids[l]
        A = H.A[l][g][:, g].tocsr()
        A.sort_indices()
        nr = int(D[l].sum())
        d = H.l1_diag(l)[g[:nr]]
        P = R = None
        om = 0
        if l < L:
            gc = gids[l + 1]
            Prow = H.P[l][g].tocsr()
            P = Prow[:, gc].tocsr()
            P.sort_indices()
            om = int(Prow.nnz - P.nnz)
            R = P.T.tocsr()
            R.sort_indices()
        levels.append(CompositeLevel(gid=g, n_real=nr, A=A, d=d, P=P, R=R, omissions=om))
    owned_g = np.nonzero(np.asarray(part) == p)[0]
    pos = {int(x): i for i, x in enumerate(gids[0])}
    owned_l = np.array([pos[int(x)] for x in owned_g], dtype=np.int64)
    return CompositeGrid(p=p, levels=levels, owned_local=owned_l, owned_gid=owned_g)


def build_all(H: Hierarchy, part: np.ndarray, nparts: int, eta, brute: bool = False) -> List[CompositeGrid]:
    return [build_composite(H, part, p, eta, brute=brute) for p in range(nparts)]


def composite_overhead(H: Hierarchy, comps: Sequence[CompositeGrid]) -> float:
    """Composite-grid overhead (Section 6.1): nonzeros of A_l at real points,
    summed over all levels and all composite grids, divided by the total
    nonzeros of the global hierarchy."""
    num = 0
    for cg in comps:
        for l, lev in enumerate(cg.levels):
            A = H.A[l]
            rows = lev.gid[: lev.n_real]
            num += int(np.diff(A.indptr)[rows].sum())
    den = sum(A.nnz for A in H.A)
    return num / den
