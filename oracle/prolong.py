"""Prolongations.

* Tentative (Def. def:pwp, eq. pwp): ``P_iJ = Q^{J->i}`` for i in C_J, rows of D empty.  On the
  finest elasticity level only the displacement rows are kept (Def. def:pwp_el):
  ``P^f_iJ = [I_3, Skew(x_i - x_J)]`` (3 x 6 blocks).
* Auxiliary smoothed prolongation (Def. def:aux_sp): ``P_s = (I - omega (Dhat^0)^+ Ahat^0) P``
  with a row-wise choice between the real matrix ("S" rows) and edge matrices ("A" rows).

Readings (the paper gives only the row caps):

* S/A split: ``cols_S(i) = {agg(i)} U {agg(j) : A_ij structurally nonzero, j not in D}``;
  i is an S row iff ``|cols_S(i)| <= cap_S`` (8 on the finest level, 6 below).
* Filtered neighbours of an A row: group the edge neighbours l not in D by agg(l); keep the group
  agg(i) and the ``cap_A - 1`` other groups with the largest sum of tr E^il (picked one by one;
  sums within a relative 1e-12 of the largest tie, smaller coarse id first); F^i is the union of
  the kept groups.
* A rows use ``Dhat^0_ii = sum_{l in F^i} Q^{il,T} E^il Q^il`` and
  ``Ahat^0_il = -Q^{il,T} E^il Q^li`` (eq. auxa restricted to F^i; the definition's printed
  Q^{li,T} E^il Q^li and M^ij are read this way, which keeps rigid-body modes in the range).
  Pseudo-inverses replace inverses (remark after Def. def:aux_sp).
* Row pattern: {agg(i)} U agg(F^i) for A rows, cols_S(i) for S rows; columns sorted,
  structural zeros kept.
"""
from __future__ import annotations

import dataclasses

import numpy as np
import scipy.sparse as sp

from .dense import pinv_tau, q_half, q_transport

ROW_S, ROW_A, ROW_D = 0, 1, 2


@dataclasses.dataclass
class BCSR:
    """Block CSR with dense r x c blocks (row-major)."""
    n_rows: int
    n_cols: int
    row_ptr: np.ndarray
    col: np.ndarray
    val: np.ndarray   # (nnzb, r, c)

    @property
    def r(self):
        return self.val.shape[1]

    @property
    def c(self):
        return self.val.shape[2]

    @property
    def nnzb(self):
        return int(self.col.size)

    def to_scipy(self):
        return sp.bsr_matrix((self.val, self.col, self.row_ptr),
                             shape=(self.n_rows * self.r, self.n_cols * self.c)).tocsr()

    def block(self, i, j):
        s, e = self.row_ptr[i], self.row_ptr[i + 1]
        hit = np.nonzero(self.col[s:e] == j)[0]
        return self.val[s + hit[0]] if hit.size else None

    def transpose(self):
        """Explicit block transpose (blocks transposed, rows sorted by column)."""
        rows = np.repeat(np.arange(self.n_rows), np.diff(self.row_ptr))
        order = np.lexsort((rows, self.col))
        ptr = np.zeros(self.n_cols + 1, dtype=np.int64)
        np.add.at(ptr, self.col + 1, 1)
        return BCSR(self.n_cols, self.n_rows, np.cumsum(ptr), rows[order],
                    np.ascontiguousarray(self.val[order].transpose(0, 2, 1)))


def tentative_block(x_fine, x_coarse, k, bs):
    """P_iJ = Q^{J->i}, restricted to the first bs rows (displacements) when bs < k."""
    return q_transport(x_coarse, x_fine, k)[:bs, :]


def tentative_prolongation(n, k, bs, coords, agg_of, ccoords) -> BCSR:
    nc = ccoords.shape[0]
    rows = [i for i in range(n) if agg_of[i] >= 0]
    ptr = np.zeros(n + 1, dtype=np.int64)
    for i in rows:
        ptr[i + 1] = 1
    ptr = np.cumsum(ptr)
    col = np.array([agg_of[i] for i in rows], dtype=np.int64)
    val = np.array([tentative_block(coords[i], ccoords[agg_of[i]], k, bs) for i in rows])
    return BCSR(n, nc, ptr, col, val.reshape(-1, bs, k))


def row_split(A: BCSR, aux, agg_of, dmask, cap_S):
    """Row types (ROW_S / ROW_A / ROW_D) and the S-row column sets."""
    n = A.n_rows
    types = np.full(n, ROW_D, dtype=np.int64)
    colsS = {}
    for i in range(n):
        if dmask[i]:
            continue
        s, e = A.row_ptr[i], A.row_ptr[i + 1]
        cs = {int(agg_of[i])}
        for j in A.col[s:e]:
            if not dmask[j]:
                cs.add(int(agg_of[j]))
        if len(cs) <= cap_S:
            types[i] = ROW_S
            colsS[i] = sorted(cs)
        else:
            types[i] = ROW_A
    return types, colsS


def filtered_neighbors(aux, i, agg_of, dmask, cap_A, tie_rtol=1e-12):
    """F^i (sorted (vertex, edge) pairs) and the kept coarse groups.

    Groups are picked one at a time by largest sum of tr E^il; sums within the relative band
    ``tie_rtol`` of the largest tie and the smaller coarse id wins (the tie rule of the
    matching), so that round-off cannot reorder mathematically equal weights."""
    nb, eid = aux.neighbors(i)
    wsum = {}
    mem = {}
    for l, e in zip(nb.tolist(), eid.tolist()):
        if dmask[l]:
            continue
        g = int(agg_of[l])
        wsum[g] = wsum.get(g, 0.0) + float(np.trace(aux.E[e]))
        mem.setdefault(g, []).append((l, e))
    own = int(agg_of[i])
    others = [g for g in wsum if g != own]
    keep = [own]
    while others and len(keep) < cap_A:
        wmax = max(wsum[g] for g in others)
        g = min(g for g in others if wsum[g] >= wmax * (1.0 - tie_rtol))
        keep.append(g)
        others.remove(g)
    F = sorted(le for g in keep for le in mem.get(g, []))
    return F, sorted(keep)


def smoothed_prolongation(A: BCSR, aux, agg_of, dmask, ccoords, cap_S, cap_A, omega=2.0 / 3.0,
                          tau=1e-10):
    """Returns (P_s as BCSR with bs x k blocks, row types)."""
    n = A.n_rows
    k = aux.k
    bs = A.r
    x = aux.coords
    nc = ccoords.shape[0]
    types, colsS = row_split(A, aux, agg_of, dmask, cap_S)
    ptr = np.zeros(n + 1, dtype=np.int64)
    cols_all, vals_all = [], []
    for i in range(n):
        if types[i] == ROW_D:
            ptr[i + 1] = ptr[i]
            continue
        Ji = int(agg_of[i])
        if types[i] == ROW_S:
            cols = colsS[i]
            acc = {J: np.zeros((bs, k)) for J in cols}
            s, e = A.row_ptr[i], A.row_ptr[i + 1]
            Aii = None
            for p in range(s, e):
                j = int(A.col[p])
                if j == i:
                    Aii = A.val[p]
                if dmask[j]:
                    continue
                Jj = int(agg_of[j])
                acc[Jj] += A.val[p] @ tentative_block(x[j], ccoords[Jj], k, bs)
            Dinv = pinv_tau(Aii, tau)
            Pi = tentative_block(x[i], ccoords[Ji], k, bs)
            row = []
            for J in cols:
                blk = -omega * (Dinv @ acc[J])
                if J == Ji:
                    blk = blk + Pi
                row.append(blk)
        else:
            F, cols = filtered_neighbors(aux, i, agg_of, dmask, cap_A)
            Dh = np.zeros((k, k))
            for l, e in F:
                Dh += q_half(x[i], x[l], k).T @ aux.E[e] @ q_half(x[i], x[l], k)
            Pi_full = q_transport(ccoords[Ji], x[i], k)
            acc = {J: np.zeros((k, k)) for J in cols}
            acc[Ji] += Dh @ Pi_full
            for l, e in F:
                Jl = int(agg_of[l])
                Ail = -(q_half(x[i], x[l], k).T @ aux.E[e] @ q_half(x[l], x[i], k))
                acc[Jl] += Ail @ q_transport(ccoords[Jl], x[l], k)
            Dp = pinv_tau(Dh, tau)
            row = []
            for J in cols:
                blk = -omega * (Dp @ acc[J])
                if J == Ji:
                    blk = blk + Pi_full
                row.append(blk[:bs, :])
        ptr[i + 1] = ptr[i] + len(cols)
        cols_all.extend(cols)
        vals_all.extend(row)
    val = np.array(vals_all).reshape(-1, bs, k)
    return BCSR(n, nc, ptr, np.array(cols_all, dtype=np.int64), val), types
