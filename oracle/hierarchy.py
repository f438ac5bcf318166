"""Multilevel setup.

* Operator: the BC-free A_N with the Dirichlet block rows / columns replaced by identity / zero
  blocks (the system on V_h0 of section "fem", pattern kept).
* Coarse operators: ``A_{l+1} = P_s^T A_l P_s`` (Galerkin, section "prol"), structural pattern,
  no value-based dropping, not symmetrized.
* Smoother diagonals: pseudo-inverses of the diagonal blocks (the "pseudo smoother" of section
  "sing2", which implements the smoother of the restricted operator).
* Coarsest level: ``A_L + blockdiag(U_0 U_0^T)`` with U_0 the kernel of each diagonal block
  (section "sing2": the regularization ``I - E E^T`` leaves the coarse correction unchanged),
  then a dense Cholesky factorization.
* Colouring (not in the paper; needed by the multicolour Gauss-Seidel smoother): greedy in
  smallest-last order (min-degree removal, lowest id on ties, reversed), smallest colour not used
  by an already coloured neighbour in the block graph of A_l.
* Stop: level l is the coarsest when ``bs_l * n_l < coarsest_max_dofs``, when coarsening would
  keep more than 90 % of the vertices (or none), or when ``max_levels`` levels exist.
"""
from __future__ import annotations

import dataclasses
from typing import Optional

import numpy as np
import scipy.sparse as sp

from .auxtop import AuxLevel, finest_aux
from .coarsen import MatchingResult, successive_matching
from .dense import kernel_basis, pinv_tau
from .prolong import BCSR, smoothed_prolongation


@dataclasses.dataclass
class SetupParams:
    sigma: float = 20.0
    delta: int = 1
    R: int = 1
    rounds: int = 2
    coarsest_max_dofs: int = 500
    max_levels: int = 25
    omega: float = 2.0 / 3.0
    cap_aux: int = 4
    cap_std_l0: int = 8
    cap_std: int = 6
    pinv_rtol: float = 1e-10
    tie_rtol: float = 1e-12
    mu_s_only: bool = False    # scalar-only pairing (no mu_b / mu_g), for comparisons


@dataclasses.dataclass
class Level:
    A: BCSR
    aux: AuxLevel
    colors: np.ndarray
    Dinv: np.ndarray                       # (n, bs, bs)
    P: Optional[BCSR] = None               # P_s, (n x n_{l+1}) blocks bs x k
    agg_of: Optional[np.ndarray] = None    # coarse id or -1 (D)
    row_types: Optional[np.ndarray] = None
    match: Optional[MatchingResult] = None

    @property
    def n(self):
        return self.A.n_rows

    @property
    def bs(self):
        return self.A.r


@dataclasses.dataclass
class Hierarchy:
    levels: list
    params: SetupParams
    coarse_dense: np.ndarray      # regularized A_L (dense)
    coarse_chol: np.ndarray       # lower Cholesky factor
    dim: int

    @property
    def n_levels(self):
        return len(self.levels)

    def complexities(self):
        n0 = self.levels[0].n
        nnz0 = self.levels[0].A.nnzb * self.levels[0].bs ** 2
        vc = sum(lv.n for lv in self.levels) / n0
        oc = sum(lv.A.nnzb * lv.bs ** 2 for lv in self.levels) / nnz0
        return vc, oc


def apply_dirichlet(n, row_ptr, col, vals, dirichlet) -> BCSR:
    row_ptr = np.asarray(row_ptr, dtype=np.int64)
    col = np.asarray(col, dtype=np.int64)
    bs = vals.shape[1]
    val = np.array(vals, dtype=np.float64, copy=True)
    rows = np.repeat(np.arange(n), np.diff(row_ptr))
    d = np.asarray(dirichlet).astype(bool)
    hit = d[rows] | d[col]
    val[hit] = 0.0
    diag = hit & (rows == col)
    val[diag] = np.eye(bs)
    return BCSR(n, n, row_ptr, col, val)


def galerkin(A: BCSR, P: BCSR) -> BCSR:
    """P^T A P with the structural block pattern of the product."""
    k = P.c
    nc = P.n_cols
    pa = sp.csr_matrix((np.ones(A.nnzb), A.col, A.row_ptr), shape=(A.n_rows, A.n_cols))
    pp = sp.csr_matrix((np.ones(P.nnzb), P.col, P.row_ptr), shape=(P.n_rows, P.n_cols))
    pc = (pp.T @ (pa @ pp)).tocsr()
    pc.sort_indices()
    Ps = P.to_scipy()
    prod = (Ps.T @ (A.to_scipy() @ Ps)).tocsr()
    rows = np.repeat(np.arange(nc), np.diff(pc.indptr))
    cols = pc.indices
    a = np.arange(k)
    ri = (rows[:, None, None] * k + a[None, :, None]) * np.ones((1, 1, k), dtype=np.int64)
    ci = (cols[:, None, None] * k + a[None, None, :]) * np.ones((1, k, 1), dtype=np.int64)
    vals = np.asarray(prod[ri.ravel(), ci.ravel()]).reshape(-1, k, k)
    return BCSR(nc, nc, pc.indptr.astype(np.int64), cols.astype(np.int64), vals)


def smallest_last_order(A: BCSR) -> list:
    """Smallest-last vertex order of the block graph of A (self loops ignored): repeatedly remove
    a vertex of minimum remaining degree (lowest id on ties); the order is the reverse of the
    removal sequence."""
    import heapq
    n = A.n_rows
    adj = [[int(j) for j in A.col[A.row_ptr[i]:A.row_ptr[i + 1]] if j != i] for i in range(n)]
    deg = [len(a) for a in adj]
    removed = [False] * n
    heap = [(deg[v], v) for v in range(n)]
    heapq.heapify(heap)
    seq = []
    while heap:
        d, v = heapq.heappop(heap)
        if removed[v] or d != deg[v]:
            continue
        removed[v] = True
        seq.append(v)
        for u in adj[v]:
            if not removed[u]:
                deg[u] -= 1
                heapq.heappush(heap, (deg[u], u))
    return seq[::-1]


def greedy_coloring(A: BCSR) -> np.ndarray:
    """Greedy colouring in smallest-last order: each vertex takes the smallest colour not used
    by an already coloured neighbour."""
    n = A.n_rows
    colors = np.full(n, -1, dtype=np.int64)
    for i in smallest_last_order(A):
        used = set()
        for j in A.col[A.row_ptr[i]:A.row_ptr[i + 1]]:
            if j != i and colors[j] >= 0:
                used.add(int(colors[j]))
        c = 0
        while c in used:
            c += 1
        colors[i] = c
    return colors


def diag_blocks(A: BCSR) -> np.ndarray:
    out = np.zeros((A.n_rows, A.r, A.c))
    for i in range(A.n_rows):
        blk = A.block(i, i)
        if blk is None:
            raise ValueError(f"missing diagonal block in row {i}")
        out[i] = blk
    return out


def dense_matrix(A: BCSR) -> np.ndarray:
    return A.to_scipy().toarray()


def setup(dim, coords, row_ptr, col, vals, dirichlet, params: Optional[SetupParams] = None,
          verbose=False, factor_coarsest=True) -> Hierarchy:
    params = params or SetupParams()
    coords = np.asarray(coords, dtype=np.float64)
    n = coords.shape[0]
    vals = np.asarray(vals, dtype=np.float64).reshape(-1, dim, dim)
    A = apply_dirichlet(n, row_ptr, col, vals, dirichlet)
    aux = finest_aux(dim, coords, row_ptr, col, vals)
    tau = params.pinv_rtol
    levels = []
    lidx = 0
    while True:
        Dinv = np.array([pinv_tau(b, tau) for b in diag_blocks(A)]).reshape(-1, A.r, A.r)
        lev = Level(A, aux, greedy_coloring(A), Dinv)
        levels.append(lev)
        if A.r * A.n_rows < params.coarsest_max_dofs or len(levels) >= params.max_levels:
            break
        vd = np.asarray(dirichlet).astype(bool) if lidx == 0 else np.zeros(A.n_rows, bool)
        res = successive_matching(aux, vd, params.sigma, params.rounds, params.tie_rtol, tau,
                                  params.mu_s_only)
        nc = len(res.aggs)
        if nc == 0 or nc > 0.9 * A.n_rows:
            break
        agg_of = np.full(A.n_rows, -1, dtype=np.int64)
        for I, mem in enumerate(res.aggs):
            agg_of[mem] = I
        capS = params.cap_std_l0 if lidx == 0 else params.cap_std
        P, types = smoothed_prolongation(A, aux, agg_of, res.dmask, res.coarse_coords, capS,
                                         params.cap_aux, params.omega, tau)
        lev.P, lev.agg_of, lev.row_types, lev.match = P, agg_of, types, res
        if verbose:
            print(f"level {lidx}: n={A.n_rows} nnzb={A.nnzb} -> nc={nc} "
                  f"(margin {res.min_margin:.3g}, tie {res.max_tie})", flush=True)
        A = galerkin(A, P)
        aux = res.coarse_level
        lidx += 1
    AL = levels[-1].A
    Ad = dense_matrix(AL)
    bs = AL.r
    for i, blk in enumerate(diag_blocks(AL)):
        U0 = kernel_basis(blk, tau)
        Ad[i * bs:(i + 1) * bs, i * bs:(i + 1) * bs] += U0 @ U0.T
    Lf = np.linalg.cholesky(Ad) if factor_coarsest else None
    return Hierarchy(levels, params, Ad, Lf, dim)
