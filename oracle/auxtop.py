"""Auxiliary topology: vertices with k x k vertex weights M^i, edges with k x k edge weights E^ij.

* Def. def:deng, eq. auxa: the auxiliary matrix
  ``Ahat_ii = M^i + sum_j Q^{ij,T} E^ij Q^ij``, ``Ahat_ij = -Q^{ij,T} E^ij Q^ji``.
* Finest level, elasticity (Thm thm:deng_elast and the remark on c^ij after it):
  ``E^ij = c^ij [[t t^T, 0], [0, 0]]``, ``M^i = 0``, with ``c^ij`` the mean absolute entry of the
  3x3 block ``(A_N)_ij`` and ``t`` the *unit* edge direction (our reading: the unit vector keeps
  ``tr E^ij = c^ij`` in the units of A, so real-matrix and edge-matrix rows mix consistently).
* Finest level, scalar (section "deng", after the remark on Q^ij): ``E^ij = |A_ij|`` and
  ``M^i = max(0, A_ii - sum_j |A_ij|)``.
* Coarse level (Thm thm:cemats): ``E^IJ = sum_{i in C_I, j in C_J} T^T E^ij T`` with
  ``T = Q^{IJ->ij} = Q^ij Q^{I->i} Q^JI``, and
  ``M^I = sum_{i in C_I} Q^{I->i,T} (M^i + sum_{j in D} Q^{ij,T} E^ij Q^ij) Q^{I->i}``.
"""
from __future__ import annotations

import dataclasses

import numpy as np

from .dense import q_half, q_transport


@dataclasses.dataclass
class AuxLevel:
    k: int
    coords: np.ndarray   # (n, 3)
    edges: np.ndarray    # (m, 2) int64, i < j, ascending lexicographic
    E: np.ndarray        # (m, k, k)
    M: np.ndarray        # (n, k, k)

    def __post_init__(self):
        n = self.coords.shape[0]
        m = self.edges.shape[0]
        ends = np.concatenate([self.edges[:, 0], self.edges[:, 1]])
        others = np.concatenate([self.edges[:, 1], self.edges[:, 0]])
        eids = np.concatenate([np.arange(m), np.arange(m)])
        order = np.lexsort((others, ends))
        self.nbr_ptr = np.zeros(n + 1, dtype=np.int64)
        np.add.at(self.nbr_ptr, ends + 1, 1)
        self.nbr_ptr = np.cumsum(self.nbr_ptr)
        self.nbr = others[order]
        self.nbr_edge = eids[order]
        self._eid = {(int(a), int(b)): e for e, (a, b) in enumerate(self.edges)}

    @property
    def n(self) -> int:
        return self.coords.shape[0]

    def neighbors(self, i):
        s, e = self.nbr_ptr[i], self.nbr_ptr[i + 1]
        return self.nbr[s:e], self.nbr_edge[s:e]

    def edge_id(self, i, j):
        """Edge id of {i, j} or None."""
        a, b = (i, j) if i < j else (j, i)
        return self._eid.get((int(a), int(b)))

    def pulled(self, e, at):
        """Q^{ab,T} E^ab Q^ab: edge weight of edge e seen from endpoint ``at`` (a = at)."""
        i, j = self.edges[e]
        other = j if at == i else i
        Q = q_half(self.coords[at], self.coords[other], self.k)
        return Q.T @ self.E[e] @ Q


def finest_aux(dim, coords, row_ptr, col_idx, vals) -> AuxLevel:
    """Finest level edge / vertex weights from the BC-free block matrix A_N.

    Edges are all off-diagonal block positions (i, j), i < j, of the (symmetric) pattern.
    """
    coords = np.asarray(coords, dtype=np.float64)
    n = coords.shape[0]
    row_ptr = np.asarray(row_ptr, dtype=np.int64)
    col_idx = np.asarray(col_idx, dtype=np.int64)
    vals = np.asarray(vals, dtype=np.float64).reshape(-1, dim, dim)
    rows = np.repeat(np.arange(n), np.diff(row_ptr))
    up = col_idx > rows
    edges = np.stack([rows[up], col_idx[up]], axis=1)
    order = np.lexsort((edges[:, 1], edges[:, 0]))
    edges = edges[order]
    blocks = vals[up][order]
    m = edges.shape[0]
    if dim == 3:
        k = 6
        c = np.abs(blocks).reshape(m, 9).mean(axis=1)
        t = coords[edges[:, 1]] - coords[edges[:, 0]]
        t = t / np.linalg.norm(t, axis=1)[:, None]
        E = np.zeros((m, 6, 6))
        E[:, :3, :3] = c[:, None, None] * t[:, :, None] * t[:, None, :]
        M = np.zeros((n, 6, 6))
    elif dim == 1:
        k = 1
        E = np.abs(blocks).reshape(m, 1, 1).copy()
        diag = np.zeros(n)
        offsum = np.zeros(n)
        flat = vals.reshape(-1)
        is_diag = col_idx == rows
        diag[rows[is_diag]] = flat[is_diag]
        np.add.at(offsum, rows[~is_diag], np.abs(flat[~is_diag]))
        M = np.maximum(0.0, diag - offsum).reshape(n, 1, 1)
    else:
        raise ValueError("dim must be 1 or 3")
    return AuxLevel(k, coords, edges.astype(np.int64), E, M)


def dhat_all(level: AuxLevel) -> np.ndarray:
    """Diagonal blocks of the auxiliary matrix: M^i + sum_{j~i} Q^{ij,T} E^ij Q^ij."""
    D = level.M.copy()
    for i in range(level.n):
        nb, eid = level.neighbors(i)
        for j, e in zip(nb, eid):
            D[i] += level.pulled(e, i)
    return D


def assemble_aux_dense(level: AuxLevel) -> np.ndarray:
    """Dense auxiliary matrix (eq. auxa), block (i, j) at rows i*k.., cols j*k.."""
    k, n = level.k, level.n
    A = np.zeros((n * k, n * k))
    for i in range(n):
        A[i * k:(i + 1) * k, i * k:(i + 1) * k] += level.M[i]
    for e, (i, j) in enumerate(level.edges):
        xi, xj = level.coords[i], level.coords[j]
        Qij = q_half(xi, xj, k)
        Qji = q_half(xj, xi, k)
        Ee = level.E[e]
        A[i * k:(i + 1) * k, i * k:(i + 1) * k] += Qij.T @ Ee @ Qij
        A[j * k:(j + 1) * k, j * k:(j + 1) * k] += Qji.T @ Ee @ Qji
        A[i * k:(i + 1) * k, j * k:(j + 1) * k] -= Qij.T @ Ee @ Qji
        A[j * k:(j + 1) * k, i * k:(i + 1) * k] -= Qji.T @ Ee @ Qij
    return A


def coarse_aux(level: AuxLevel, aggs, dmask, ccoords) -> AuxLevel:
    """Coarse edge / vertex weights of Thm thm:cemats.

    aggs: list of member-id arrays (coarse vertex I = list position); dmask: bool (n,) of the
    dropped set D; ccoords: (nc, 3) coarse vertex positions.  Edges inside one agglomerate and
    edges between two D vertices are dropped; edges between an agglomerate vertex and a D
    vertex go into M^I.  Fine edges are accumulated in ascending (i, j) order.
    """
    k = level.k
    n = level.n
    nc = len(aggs)
    agg_of = np.full(n, -1, dtype=np.int64)
    for I, mem in enumerate(aggs):
        agg_of[np.asarray(mem, dtype=np.int64)] = I
    x = level.coords
    Mc = np.zeros((nc, k, k))
    for I, mem in enumerate(aggs):
        for i in sorted(int(v) for v in mem):
            W = level.M[i].copy()
            nb, eid = level.neighbors(i)
            for j, e in zip(nb, eid):
                if dmask[j]:
                    W += level.pulled(e, i)
            QIi = q_transport(ccoords[I], x[i], k)
            Mc[I] += QIi.T @ W @ QIi
    acc = {}
    for e, (i, j) in enumerate(level.edges):
        I, J = agg_of[i], agg_of[j]
        if I < 0 or J < 0 or I == J:
            continue
        a, b = (I, J) if I < J else (J, I)
        # T = Q^ij Q^{I->i} Q^JI  (midpoint of (I, J) -> midpoint of (i, j))
        T = q_half(x[i], x[j], k) @ q_transport(ccoords[I], x[i], k) @ q_half(ccoords[J],
                                                                             ccoords[I], k)
        contrib = T.T @ level.E[e] @ T
        if (a, b) in acc:
            acc[(a, b)] += contrib
        else:
            acc[(a, b)] = contrib
    keys = sorted(acc)
    cedges = np.array(keys, dtype=np.int64).reshape(-1, 2)
    cE = np.array([acc[key] for key in keys]).reshape(-1, k, k)
    return AuxLevel(k, np.asarray(ccoords, dtype=np.float64), cedges, cE, Mc)
