"""Small dense primitives (all FP64).

* ``skew(t)``: the matrix with ``skew(t) @ r == cross(t, r)`` (paper section "amg", Skew).
* ``qmat(t, k)``: ``[[I, Skew(t)], [0, I]]`` for k = 6; ``[[1]]`` for the scalar case k = 1.
  ``Q^{a->b} = qmat(x_b - x_a)`` carries rigid-body coordinates (u, r) from vertex a to b
  (eq. qij_epseps); ``Q^{ab} = sqrt(Q^{a->b}) = qmat((x_b - x_a)/2)`` carries them to the
  midpoint of the edge (remark after Def. def:deng).
* ``pinv_tau(X)``: symmetric pseudo-inverse.  Eigenvalues at or below ``tau * max(lambda_max, 0)``
  are treated as zero (the pseudo-inverses of section "sing2" and of Def. def:aux_sp's remark).
* ``harmonic(A, B)``: ``H(A, B) = A (A + B)^+ B`` (Lemma thm:mu2), symmetrized.
* ``genmax(L, R)``: largest lambda of ``L v = lambda R v`` on PSD pencils, +inf when L is
  positive on a null direction of R (the smallest constant mu with ``L <= mu R``, the form
  in which Thm thm:mu1 and Lemma thm:mu2 define mu_g and mu_b).
"""
from __future__ import annotations

import numpy as np

TAU_DEFAULT = 1e-10


def skew(t) -> np.ndarray:
    t = np.asarray(t, dtype=np.float64)
    return np.array([[0.0, -t[2], t[1]],
                     [t[2], 0.0, -t[0]],
                     [-t[1], t[0], 0.0]])


def qmat(t, k: int) -> np.ndarray:
    if k == 1:
        return np.ones((1, 1))
    if k != 6:
        raise ValueError("k must be 1 (scalar) or 6 (3D elasticity)")
    Q = np.eye(6)
    Q[:3, 3:] = skew(t)
    return Q


def q_transport(xa, xb, k: int) -> np.ndarray:
    """Q^{a->b}: coordinates at x_a -> coordinates of the rigid extension at x_b."""
    return qmat(np.asarray(xb) - np.asarray(xa), k)


def q_half(xa, xb, k: int) -> np.ndarray:
    """Q^{ab} = sqrt(Q^{a->b}): coordinates at x_a -> coordinates at the midpoint of (a, b)."""
    return qmat(0.5 * (np.asarray(xb) - np.asarray(xa)), k)


def sym(X: np.ndarray) -> np.ndarray:
    return 0.5 * (X + X.T)


def pinv_tau(X: np.ndarray, tau: float = TAU_DEFAULT) -> np.ndarray:
    lam, U = np.linalg.eigh(sym(X))
    lmax = lam.max() if lam.size else 0.0
    if lmax <= 0.0:
        return np.zeros_like(X)
    keep = lam > tau * lmax
    Uk = U[:, keep]
    return (Uk / lam[keep]) @ Uk.T


def kernel_basis(X: np.ndarray, tau: float = TAU_DEFAULT) -> np.ndarray:
    """Orthonormal basis U_0 (columns) of the tau-kernel of symmetric X."""
    lam, U = np.linalg.eigh(sym(X))
    lmax = lam.max() if lam.size else 0.0
    if lmax <= 0.0:
        return U
    return U[:, ~(lam > tau * lmax)]


def harmonic(A: np.ndarray, B: np.ndarray, tau: float = TAU_DEFAULT) -> np.ndarray:
    return sym(A @ pinv_tau(A + B, tau) @ B)


def genmax(L: np.ndarray, R: np.ndarray, tau: float = TAU_DEFAULT) -> float:
    L = sym(L)
    R = sym(R)
    nL = np.linalg.norm(L)
    if nL == 0.0:
        return 0.0
    lam, U = np.linalg.eigh(R)
    lmax = lam.max()
    keep = lam > tau * lmax if lmax > 0.0 else np.zeros(lam.shape, dtype=bool)
    U0 = U[:, ~keep]
    if U0.shape[1] and np.linalg.norm(U0.T @ L @ U0) > tau * nL:
        return float("inf")
    if not keep.any():
        return 0.0
    W = U[:, keep] / np.sqrt(lam[keep])
    return float(np.linalg.eigvalsh(sym(W.T @ L @ W)).max())
