"""Oracle: classical (Ruge-Stueben) AMG setup, plain serial FP64.

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
benchmark's CPU-baseline leg may import this package; the product path never
does.  It shares no code with the HIP library.

Follows the paper's review of AMG (Section 2): a C/F splitting driven by
strength of connection, interpolation P_l, restriction R_l = P_l^T and the
Galerkin product A_{l+1} = R_l A_l P_l, repeated until the coarsest level is
small enough for a direct solve.  The paper leaves the AMG components to its
host library; the readings used here are:

* strength: j strongly influences i iff j != i, m_i = max_{k != i}(-a_ik) > 0
  and -a_ij >= theta * m_i * (1 - 1e-12)   (theta = 0.25)
* classical RS first pass only, ties broken by the smallest index, coarse
  points numbered in increasing fine index
* direct interpolation (Stueben), positive off-diagonals lumped into the
  diagonal, empty rows for F-points without strong C-neighbours
* Galerkin coarse operator on the *symbolic* product pattern (no dropping of
  exact cancellations); values from the product R (A P)
* stop at <= max_coarse points, when a level produces no C-point or no
  reduction, or at max_levels levels

The paper's own experiments use the host library's "best practices"
components (Section 6): HMIS coarsening and extended+i interpolation.  They
are here as options (coarsen="hmis", interp="ext+i"), written from their
published definitions (De Sterck, Yang, Heys 2006; De Sterck, Falgout,
Nolting, Yang 2008):

* PMIS: measure lambda_i = |S^T_i| + r_i with r_i uniform in [0, 1); points
  that influence nobody are F; repeatedly every undecided point whose measure
  exceeds that of each undecided strong neighbour (either direction; equal
  measures: smaller index wins) becomes C and the undecided points that
  strongly depend on it become F.
* HMIS: one RS first pass inside each subdomain (strong connections between
  points of the same subdomain only); its C-points with no strong connection
  to another subdomain form PMIS's first independent set (they are C and
  their dependents F before the first PMIS round).  Subdomains of a coarse
  level are inherited along the C-points.
* r_i of point i on level l: the 53 high bits of SplitMix64(2^32 l + i)
  divided by 2^53 (Steele, Lea, Flood 2014: add 0x9E3779B97F4A7C15, then
  z ^= z >> 30, z *= 0xBF58476D1CE4E5B9, z ^= z >> 27, z *= 0x94D049BB133111EB,
  z ^= z >> 31, all mod 2^64).
* extended+i interpolation: see ext_i_interpolation; rows truncated to at
  most 4 entries (the host library's default) by truncate_row.

Every floating-point row sum is accumulated sequentially in ascending column
order (the order a reader would write by hand).
"""

from __future__ import annotations

import heapq
from dataclasses import dataclass, field
from typing import List

import numpy as np
from scipy import sparse

C_PT = 1
F_PT = -1
U_PT = 0

STRENGTH_SLACK = 1e-12


def _csr(A) -> sparse.csr_matrix:
    A = sparse.csr_matrix(A)
    A.sort_indices()
    return A


def row_ids(A: sparse.csr_matrix) -> np.ndarray:
    return np.repeat(np.arange(A.shape[0]), np.diff(A.indptr))


def seq_row_sum(indptr: np.ndarray, vals: np.ndarray) -> np.ndarray:
    """Per-row sum of vals, added one entry at a time in storage order
    (0 + v0 + v1 + ...).  Vectorised over rows, sequential within a row."""
    n = len(indptr) - 1
    lens = np.diff(indptr)
    out = np.zeros(n, dtype=np.float64)
    start = indptr[:-1]
    for k in range(int(lens.max()) if n else 0):
        m = lens > k
        out[m] += vals[start[m] + k]
    return out


def strength(A: sparse.csr_matrix, theta: float = 0.25) -> sparse.csr_matrix:
    """Strength matrix S (CSR pattern, sorted): row i lists S_i, the points
    that strongly influence i (Section 2: strong influence decided by the
    relative size of the entries of A)."""
    A = _csr(A)
    n = A.shape[0]
    r = row_ids(A)
    c = A.indices
    off = c != r
    m = np.full(n, -np.inf)
    np.maximum.at(m, r[off], -A.data[off])
    mr = m[r]
    strong = off & (mr > 0) & (-A.data >= theta * mr * (1.0 - STRENGTH_SLACK))
    S = sparse.csr_matrix((np.ones(int(strong.sum())), (r[strong], c[strong])), shape=(n, n))
    S.sort_indices()
    return S


def rs_first_pass(S: sparse.csr_matrix) -> np.ndarray:
    """Classical Ruge-Stueben first-pass C/F splitting.

    lambda_i = |S^T_i| (how many points i strongly influences).  Repeatedly the
    undecided point of largest lambda (smallest index on ties) becomes C; the
    undecided points it strongly influences become F; every undecided point
    that strongly influences a new F-point gains 1; every undecided point that
    strongly influences the new C-point loses 1.  When the largest remaining
    lambda is 0, each remaining point becomes F if it has a strong C-neighbour
    and C otherwise.  Points with no strong connection in either direction are
    F (they get an empty interpolation row).

    Returns int8 array: +1 = C, -1 = F."""
    n = S.shape[0]
    S = _csr(S)
    ST = _csr(S.T)
    Sp, Sj = S.indptr, S.indices
    Tp, Tj = ST.indptr, ST.indices
    lam = np.diff(Tp).astype(np.int64)
    state = np.zeros(n, dtype=np.int8)
    nS = np.diff(Sp)
    isolated = (nS == 0) & (lam == 0)
    state[isolated] = F_PT
    heap = [(-int(lam[i]), i) for i in range(n) if state[i] == U_PT]
    heapq.heapify(heap)
    lam_l = lam.tolist()
    st = state.tolist()
    while heap:
        nl, i = heapq.heappop(heap)
        if st[i] != U_PT or -nl != lam_l[i]:
            continue
        if lam_l[i] == 0:
            rest = [u for u in range(n) if st[u] == U_PT]
            for u in rest:
                has_c = any(st[k] == C_PT for k in Sj[Sp[u]:Sp[u + 1]])
                st[u] = F_PT if has_c else C_PT
            break
        st[i] = C_PT
        new_f = [j for j in Tj[Tp[i]:Tp[i + 1]] if st[j] == U_PT]
        for j in new_f:
            st[j] = F_PT
        for j in new_f:
            for k in Sj[Sp[j]:Sp[j + 1]]:
                if st[k] == U_PT:
                    lam_l[k] += 1
                    heapq.heappush(heap, (-lam_l[k], k))
        for j in Sj[Sp[i]:Sp[i + 1]]:
            if st[j] == U_PT:
                lam_l[j] -= 1
                heapq.heappush(heap, (-lam_l[j], j))
    return np.asarray(st, dtype=np.int8)


def direct_interpolation(A: sparse.csr_matrix, S: sparse.csr_matrix, cf: np.ndarray) -> sparse.csr_matrix:
    """Direct interpolation P (N_l x N_{l+1}), coarse ids in increasing fine index.

    C-point i: injection, P[i, c(i)] = 1.
    F-point i with interpolatory set P_i = C intersect S_i (non-empty):
        w_ik = -alpha_i a_ik / at_ii,  k in P_i
        alpha_i = (sum_{j != i} min(a_ij, 0)) / (sum_{k in P_i} a_ik)
        at_ii   = a_ii + sum_{j != i} max(a_ij, 0)
    F-point with empty P_i: empty row."""
    A = _csr(A)
    S = _csr(S)
    n = A.shape[0]
    is_c = cf == C_PT
    cidx = np.cumsum(is_c) - 1
    nc = int(is_c.sum())
    r = row_ids(A)
    off = A.indices != r
    vals = A.data
    neg = np.where(off, np.minimum(vals, 0.0), 0.0)
    pos = np.where(off, np.maximum(vals, 0.0), 0.0)
    neg_sum = seq_row_sum(A.indptr, neg)
    pos_sum = seq_row_sum(A.indptr, pos)
    diag = A.diagonal()
    # membership of each A entry in the interpolatory set: strong and C
    Sr = row_ids(S)
    skey = Sr.astype(np.int64) * n + S.indices
    akey = r.astype(np.int64) * n + A.indices
    in_s = np.isin(akey, skey)
    in_p = in_s & is_c[A.indices] & ~is_c[r]
    den = seq_row_sum(A.indptr, np.where(in_p, vals, 0.0))
    at = diag + pos_sum
    rows, cols, ws = [], [], []
    # C rows
    ci = np.nonzero(is_c)[0]
    rows.append(ci)
    cols.append(cidx[ci])
    ws.append(np.ones(ci.size))
    # F rows
    ent = np.nonzero(in_p)[0]
    fi = r[ent]
    alpha = neg_sum[fi] / den[fi]
    w = -alpha * vals[ent] / at[fi]
    rows.append(fi)
    cols.append(cidx[A.indices[ent]])
    ws.append(w)
    rows = np.concatenate(rows)
    cols = np.concatenate(cols)
    ws = np.concatenate(ws)
    P = sparse.csr_matrix((ws, (rows, cols)), shape=(n, nc))
    P.sort_indices()
    return P


def symbolic_pattern(A: sparse.csr_matrix, P: sparse.csr_matrix) -> sparse.csr_matrix:
    """Pattern of P^T A P without numerical cancellation: the product of the
    0/1 patterns has strictly positive entries wherever a product term exists."""
    Ab = A.copy()
    Ab.data = np.ones_like(Ab.data)
    Pb = P.copy()
    Pb.data = np.ones_like(Pb.data)
    G = _csr(Pb.T @ (Ab @ Pb))
    return G


def galerkin(A: sparse.csr_matrix, P: sparse.csr_matrix) -> sparse.csr_matrix:
    """A_{l+1} = R (A P) with R = P^T, stored on the symbolic product pattern
    (exact zeros kept as explicit entries)."""
    A = _csr(A)
    P = _csr(P)
    R = _csr(P.T)
    AP = A @ P
    RAP = _csr(R @ AP)
    G = symbolic_pattern(A, P)
    nc = P.shape[1]
    gkey = row_ids(G).astype(np.int64) * nc + G.indices
    rkey = row_ids(RAP).astype(np.int64) * nc + RAP.indices
    pos = np.searchsorted(gkey, rkey)
    assert np.all(gkey[pos] == rkey), "value outside symbolic pattern"
    vals = np.zeros(G.nnz)
    vals[pos] = RAP.data
    out = sparse.csr_matrix((vals, G.indices.copy(), G.indptr.copy()), shape=(nc, nc))
    return out


@dataclass
class Hierarchy:
    A: List[sparse.csr_matrix]
    P: List[sparse.csr_matrix]
    R: List[sparse.csr_matrix]
    cf: List[np.ndarray]
    S: List[sparse.csr_matrix] = field(default_factory=list)

    @property
    def L(self) -> int:
        """Index of the coarsest level."""
        return len(self.A) - 1

    def l1_diag(self, l: int) -> np.ndarray:
        """l1-Jacobi diagonal: d_i = sum_j |a_ij| over the full row of A_l."""
        A = self.A[l]
        return seq_row_sum(A.indptr, np.abs(A.data))

    def coarse_dense(self) -> np.ndarray:
        return self.A[-1].toarray()


MASK64 = (1 << 64) - 1


def splitmix64(x: int) -> int:
    """SplitMix64 output for counter x (all arithmetic mod 2^64)."""
    z = (x + 0x9E3779B97F4A7C15) & MASK64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & MASK64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & MASK64
    return z ^ (z >> 31)


def pmis_random(level: int, n: int) -> np.ndarray:
    """r_i in [0, 1) for the n points of `level` (see the module header)."""
    return np.array([(splitmix64((level << 32) + i) >> 11) * 2.0 ** -53 for i in range(n)], dtype=np.float64)


def pmis(S: sparse.csr_matrix, rand: np.ndarray, c_init=None) -> np.ndarray:
    """PMIS C/F splitting (De Sterck, Yang, Heys 2006), optionally starting
    from a given independent set c_init (boolean mask) of C-points.
    Returns int8: +1 C, -1 F."""
    n = S.shape[0]
    S = _csr(S)
    ST = _csr(S.T)
    cnt = np.diff(ST.indptr)
    lam = cnt.astype(np.float64) + rand
    st = np.zeros(n, dtype=np.int8)
    if c_init is not None:
        st[np.asarray(c_init, dtype=bool)] = C_PT
    st[(st == U_PT) & (cnt == 0)] = F_PT

    def mark_dependents(cs):
        for i in cs:
            for j in ST.indices[ST.indptr[i]:ST.indptr[i + 1]]:
                if st[j] == U_PT:
                    st[j] = F_PT

    if c_init is not None:
        mark_dependents(np.nonzero(np.asarray(c_init, dtype=bool))[0])
    while (st == U_PT).any():
        und = np.nonzero(st == U_PT)[0]
        new_c = []
        for i in und:
            nb = np.concatenate([S.indices[S.indptr[i]:S.indptr[i + 1]], ST.indices[ST.indptr[i]:ST.indptr[i + 1]]])
            win = True
            for j in nb:
                if st[j] == U_PT and j != i and (lam[j] > lam[i] or (lam[j] == lam[i] and j < i)):
                    win = False
                    break
            if win:
                new_c.append(i)
        for i in new_c:
            st[i] = C_PT
        mark_dependents(new_c)
    return st


def hmis(S: sparse.csr_matrix, part: np.ndarray, rand: np.ndarray) -> np.ndarray:
    """HMIS: RS first pass inside each subdomain, then PMIS from its interior
    C-points (see the module header)."""
    S = _csr(S)
    part = np.asarray(part)
    r = row_ids(S)
    same = part[r] == part[S.indices]
    S_loc = sparse.csr_matrix((S.data[same], (r[same], S.indices[same])), shape=S.shape)
    cf_loc = rs_first_pass(S_loc)
    cross = ~same
    bnd = np.zeros(S.shape[0], dtype=bool)
    bnd[r[cross]] = True
    bnd[S.indices[cross]] = True
    return pmis(S, rand, (cf_loc == C_PT) & ~bnd)


def truncate_row(cols, vals, pmax):
    """Interpolation truncation: keep the pmax entries of largest magnitude
    (smaller column first on ties) and scale them by (sum of all entries) /
    (sum of the kept entries), both summed in ascending column order, so the
    row sum is preserved.  pmax = 0 or a row of at most pmax entries: as is."""
    if pmax <= 0 or len(vals) <= pmax:
        return list(cols), list(vals)
    order = sorted(range(len(vals)), key=lambda q: (-abs(vals[q]), cols[q]))
    keep = sorted(order[:pmax], key=lambda q: cols[q])
    total = 0.0
    for v in vals:
        total += v
    kept = 0.0
    for q in keep:
        kept += vals[q]
    if kept == 0.0:
        return [cols[q] for q in keep], [vals[q] for q in keep]
    f = total / kept
    return [cols[q] for q in keep], [vals[q] * f for q in keep]


def ext_i_interpolation(A: sparse.csr_matrix, S: sparse.csr_matrix, cf: np.ndarray, pmax: int = 0) -> sparse.csr_matrix:
    """Extended+i interpolation (De Sterck, Falgout, Nolting, Yang 2008),
    rows truncated to pmax entries by truncate_row (0: no truncation).  For
    an F-point i with strong C-neighbours C_i, strong F-neighbours F_i and
    weak neighbours W_i (every other off-diagonal entry):

        Chat_i = C_i united with the strong C-neighbours of every k in F_i
        abar_kl = a_kl if a_kl a_kk < 0, else 0
        d_k = sum over l in Chat_i + {i} of abar_kl              (k in F_i)
        w_ij = -num_ij / at_ii,  j in Chat_i,
        num_ij = a_ij + sum_{k in F_i} a_ik abar_kj / d_k
        at_ii  = a_ii + sum_{n in W_i, not in Chat_i} a_in + sum_{k in F_i} a_ik abar_ki / d_k

    (a_ij = 0 when j is no neighbour of i).  A k with d_k = 0 is lumped like
    a weak neighbour: a_ik goes into at_ii.  Every sum runs in ascending index
    order: num_ij adds the k terms to a_ij in ascending k; at_ii adds the W_i
    terms to a_ii, then the k terms.  C-points: injection.  F-points with an
    empty Chat_i: empty row.  Coarse ids in increasing fine index."""
    A = _csr(A)
    S = _csr(S)
    n = A.shape[0]
    is_c = cf == C_PT
    cidx = np.cumsum(is_c) - 1
    nc = int(is_c.sum())
    Ap, Aj, Av = A.indptr, A.indices, A.data
    Sp, Sj = S.indptr, S.indices

    def row(i):
        return {int(j): float(v) for j, v in zip(Aj[Ap[i]:Ap[i + 1]], Av[Ap[i]:Ap[i + 1]])}

    rows, cols, vals = [], [], []
    for i in range(n):
        if is_c[i]:
            rows.append(i)
            cols.append(int(cidx[i]))
            vals.append(1.0)
            continue
        Si = set(int(j) for j in Sj[Sp[i]:Sp[i + 1]])
        Ci = sorted(j for j in Si if is_c[j])
        Fi = sorted(k for k in Si if not is_c[k])
        chat = set(Ci)
        for k in Fi:
            chat.update(int(l) for l in Sj[Sp[k]:Sp[k + 1]] if is_c[l])
        chat = sorted(chat)
        if not chat:
            continue
        ai = row(i)
        at = ai[i]
        cset = set(chat)
        for jn in sorted(ai):
            if jn != i and jn not in Si and jn not in cset:
                at += ai[jn]
        num = {j: ai.get(j, 0.0) for j in chat}
        for k in Fi:
            ak = row(k)
            akk = ak[k]
            d = 0.0
            for l in sorted(ak):
                if (l in cset or l == i) and ak[l] * akk < 0:
                    d += ak[l]
            if d == 0.0:
                at += ai[k]
                continue
            for j in chat:
                abar = ak.get(j, 0.0)
                if abar * akk < 0:
                    num[j] += ai[k] * abar / d
            abar_ki = ak.get(i, 0.0)
            if abar_ki * akk < 0:
                at += ai[k] * abar_ki / d
        cj, wv = truncate_row([int(cidx[j]) for j in chat], [-(num[j] / at) for j in chat], pmax)
        rows.extend([i] * len(cj))
        cols.extend(cj)
        vals.extend(wv)
    P = sparse.csr_matrix((np.array(vals), (np.array(rows, dtype=np.int64), np.array(cols, dtype=np.int64))),
                          shape=(n, nc))
    P.sort_indices()
    return P


def setup(A0, theta: float = 0.25, max_coarse: int = 16, max_levels: int = 25, coarsen: str = "rs",
          interp: str = "direct", part=None, pmax: int = 4) -> Hierarchy:
    """Build the AMG hierarchy {A_l, P_l, R_l} (Section 2).  coarsen="hmis"
    needs `part`, the subdomain of every fine point; pmax truncates
    extended+i rows (the host library's default of 4 entries)."""
    A = _csr(A0).astype(np.float64)
    As, Ps, Rs, cfs, Ss = [A], [], [], [], []
    pl = None if part is None else np.asarray(part)
    while A.shape[0] > max_coarse and len(As) < max_levels:
        S = strength(A, theta)
        if coarsen == "rs":
            cf = rs_first_pass(S)
        elif coarsen == "hmis":
            cf = hmis(S, pl, pmis_random(len(As) - 1, A.shape[0]))
        else:
            raise ValueError(coarsen)
        nc = int((cf == C_PT).sum())
        if nc == 0 or nc == A.shape[0]:
            break
        if interp == "direct":
            P = direct_interpolation(A, S, cf)
        elif interp == "ext+i":
            P = ext_i_interpolation(A, S, cf, pmax)
        else:
            raise ValueError(interp)
        if pl is not None:
            pl = pl[cf == C_PT]
        Ac = galerkin(A, P)
        Ss.append(S)
        cfs.append(cf)
        Ps.append(P)
        Rs.append(_csr(P.T))
        As.append(Ac)
        A = Ac
    return Hierarchy(A=As, P=Ps, R=Rs, cf=cfs, S=Ss)
