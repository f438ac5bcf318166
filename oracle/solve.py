"""V-cycle and preconditioned conjugate gradients (section "amg", Algorithm alg:tg; section
"res": CG preconditioned with one V-cycle).

V(l, b), starting from x = 0 (Algorithm alg:tg applied recursively, M forward and M^T backward,
so the cycle is symmetric):
  1. forward multicolour block Gauss-Seidel sweep: for colours c = 0..C-1, every row i of
     colour c at once: ``x_i += D^+_ii (b_i - sum_j A_ij x_j)``;
  2. ``r = b - A x``;
  3. ``x += P_s V(l+1, P_s^T r)``;
  4. backward sweep, colours C-1..0.
On the coarsest level V returns the Cholesky solution of the regularized A_L.

PCG: x0 = 0, r = b, z = V(0, r), p = z, rho = r.z; each iteration q = A p, alpha = rho / p.q,
x += alpha p, r -= alpha q; stop when ||r||_2 <= rtol ||b||_2; otherwise z = V(0, r),
rho' = r.z, p = z + (rho'/rho) p.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla


class _LevelOps:
    def __init__(self, lev):
        self.A = lev.A.to_scipy()
        bs = lev.bs
        self.bs = bs
        self.P = lev.P.to_scipy() if lev.P is not None else None
        self.rows = []
        self.dofs = []
        for c in range(int(lev.colors.max()) + 1 if lev.n else 0):
            rows = np.nonzero(lev.colors == c)[0]
            dofs = (rows[:, None] * bs + np.arange(bs)[None, :]).ravel()
            self.rows.append(rows)
            self.dofs.append(dofs)
        self.Ac = [self.A[d] for d in self.dofs]
        self.Dinv = lev.Dinv


def _ops(h):
    if not hasattr(h, "_ops_cache"):
        h._ops_cache = [_LevelOps(lev) for lev in h.levels]
    return h._ops_cache


def gs_sweep(ops, b, x, colors_order):
    bs = ops.bs
    for c in colors_order:
        rows, dofs, Ac = ops.rows[c], ops.dofs[c], ops.Ac[c]
        r = (b[dofs] - Ac @ x).reshape(-1, bs)
        x[dofs] += np.einsum("nij,nj->ni", ops.Dinv[rows], r).ravel()
    return x


def vcycle(h, b, level=0):
    ops = _ops(h)
    if level == h.n_levels - 1:
        return sla.cho_solve((h.coarse_chol, True), b)
    o = ops[level]
    x = np.zeros_like(b)
    nc = len(o.rows)
    gs_sweep(o, b, x, range(nc))
    r = b - o.A @ x
    x += o.P @ vcycle(h, o.P.T @ r, level + 1)
    gs_sweep(o, b, x, range(nc - 1, -1, -1))
    return x


def pcg(h, b, rtol=1e-8, max_it=1000, precond=True):
    """Returns (x, iterations, rel_res (recursive), rel_res_true, converged)."""
    A = _ops(h)[0].A
    b = np.asarray(b, dtype=np.float64)
    x = np.zeros_like(b)
    bnorm = np.linalg.norm(b)
    if bnorm == 0.0:
        return x, 0, 0.0, 0.0, True
    r = b.copy()
    z = vcycle(h, r) if precond else r.copy()
    p = z.copy()
    rho = r @ z
    it = 0
    converged = False
    while it < max_it:
        q = A @ p
        alpha = rho / (p @ q)
        x += alpha * p
        r -= alpha * q
        it += 1
        if np.linalg.norm(r) <= rtol * bnorm:
            converged = True
            break
        z = vcycle(h, r) if precond else r.copy()
        rho_new = r @ z
        p = z + (rho_new / rho) * p
        rho = rho_new
    rel = np.linalg.norm(r) / bnorm
    rel_true = np.linalg.norm(b - A @ x) / bnorm
    return x, it, rel, rel_true, converged
