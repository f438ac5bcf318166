"""Coarsening measures (section "crs2").

* ``mu_D(i)`` (Thm thm:mu1, eq. mu_d): ``sup_v v^T Dhat_ii v / v^T M^i v`` (read with a sup over
  v and consistent indices) = genmax(Dhat_ii, M^i); +inf when M^i does not dominate.
* ``mu_s(i, j)`` (Def. def:muc): ``sqrt(m_i m_j) / tr E^ij`` with
  ``m_i = max(tr M^i, max_{l ~ i} tr E^il)``; +inf when ``tr E^ij = 0``.
* ``mu_b(i, j)`` (Lemma thm:mu2, delta = 1): largest eigenvalue of
  ``H(Q^{ji,T} Dhat_ii Q^ji, Q^{ij,T} Dhat_jj Q^ij) v = lambda (E^ij + 1/2 sum_{l in N}
  (Q^{i->l} Q^ji)^T H(Q^{li,T} E^il Q^li, Q^{lj,T} E^jl Q^lj) (Q^{i->l} Q^ji)) v`` over the
  common neighbours N of i and j; every term is pulled back to the midpoint of (i, j).
* ``mu_g(C)`` (Thm thm:mu1, eq. mu_a, delta = 1, and the remark that neighbours may be
  eliminated separately): the smallest mu with
  ``inf_w |v_C - P_C w|^2_{Dhat_C} <= mu (sum |v_i|^2_{M^i} + edges inside C
  + 1/2 sum_{l not in C} inf_w sum_{i in C} |Q^il v_i - Q^li w|^2_{E^il})``.
"""
from __future__ import annotations

import numpy as np

from .dense import TAU_DEFAULT, genmax, harmonic, pinv_tau, q_half, q_transport, sym


def mu_D(level, i, Dhat, tau=TAU_DEFAULT) -> float:
    return genmax(Dhat[i], level.M[i], tau)


def trace_strength(level) -> np.ndarray:
    """m_i = max(tr M^i, max_{l ~ i} tr E^il) for every vertex."""
    m = np.array([np.trace(level.M[i]) for i in range(level.n)], dtype=np.float64)
    trE = np.trace(level.E, axis1=1, axis2=2) if level.E.size else np.zeros(0)
    for e, (i, j) in enumerate(level.edges):
        if trE[e] > m[i]:
            m[i] = trE[e]
        if trE[e] > m[j]:
            m[j] = trE[e]
    return m


def mu_s(level, i, j, mtr) -> float:
    e = level.edge_id(i, j)
    t = np.trace(level.E[e]) if e is not None else 0.0
    if t == 0.0:
        return float("inf")
    return float(np.sqrt(mtr[i] * mtr[j]) / t)


def mu_b(level, i, j, Dhat, tau=TAU_DEFAULT) -> float:
    k = level.k
    x = level.coords
    Qij = q_half(x[i], x[j], k)
    Qji = q_half(x[j], x[i], k)
    L = harmonic(Qji.T @ Dhat[i] @ Qji, Qij.T @ Dhat[j] @ Qij, tau)
    R = level.E[level.edge_id(i, j)].copy()
    nbi, eidi = level.neighbors(i)
    nbj, eidj = level.neighbors(j)
    ej = dict(zip(nbj.tolist(), eidj.tolist()))
    for l, eil in zip(nbi.tolist(), eidi.tolist()):
        if l == j or l not in ej:
            continue
        ejl = ej[l]
        Qli = q_half(x[l], x[i], k)
        Qlj = q_half(x[l], x[j], k)
        Hl = harmonic(Qli.T @ level.E[eil] @ Qli, Qlj.T @ level.E[ejl] @ Qlj, tau)
        T = q_transport(x[i], x[l], k) @ Qji
        R += 0.5 * (T.T @ Hl @ T)
    return genmax(L, R, tau)


def mu_g(level, C, Dhat, tau=TAU_DEFAULT) -> float:
    k = level.k
    x = level.coords
    mem = sorted(int(v) for v in C)
    pos = {v: a for a, v in enumerate(mem)}
    nC = len(mem)
    xH = x[mem].mean(axis=0)
    PC = np.vstack([q_transport(xH, x[i], k) for i in mem])
    DC = np.zeros((nC * k, nC * k))
    R = np.zeros((nC * k, nC * k))
    for a, i in enumerate(mem):
        DC[a * k:(a + 1) * k, a * k:(a + 1) * k] = Dhat[i]
        R[a * k:(a + 1) * k, a * k:(a + 1) * k] += level.M[i]
    L = DC - DC @ PC @ pinv_tau(PC.T @ DC @ PC, tau) @ PC.T @ DC
    # edges inside C, assembled as in eq. auxa
    outside = {}
    for a, i in enumerate(mem):
        nb, eid = level.neighbors(i)
        for l, e in zip(nb.tolist(), eid.tolist()):
            if l in pos:
                if i < l:
                    b = pos[l]
                    Qil = q_half(x[i], x[l], k)
                    Qli = q_half(x[l], x[i], k)
                    Ee = level.E[e]
                    R[a * k:(a + 1) * k, a * k:(a + 1) * k] += Qil.T @ Ee @ Qil
                    R[b * k:(b + 1) * k, b * k:(b + 1) * k] += Qli.T @ Ee @ Qli
                    R[a * k:(a + 1) * k, b * k:(b + 1) * k] -= Qil.T @ Ee @ Qli
                    R[b * k:(b + 1) * k, a * k:(a + 1) * k] -= Qli.T @ Ee @ Qil
            else:
                outside.setdefault(l, []).append((a, i, e))
    # outside neighbours adjacent to >= 2 members: Schur complement of the local assembly
    for l in sorted(outside):
        adj = outside[l]
        if len(adj) < 2:
            continue
        KCC = np.zeros((nC * k, nC * k))
        KCw = np.zeros((nC * k, k))
        Kww = np.zeros((k, k))
        for a, i, e in adj:
            Qil = q_half(x[i], x[l], k)
            Qli = q_half(x[l], x[i], k)
            Ee = level.E[e]
            KCC[a * k:(a + 1) * k, a * k:(a + 1) * k] += Qil.T @ Ee @ Qil
            KCw[a * k:(a + 1) * k, :] -= Qil.T @ Ee @ Qli
            Kww += Qli.T @ Ee @ Qli
        S = KCC - KCw @ pinv_tau(Kww, tau) @ KCw.T
        R += 0.5 * sym(S)
    return genmax(sym(L), sym(R), tau)
