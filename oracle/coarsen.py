"""Successive matching (Algorithm alg:pwagg, section "spw").

Readings of the passages the paper leaves open (each is also listed in the design notes):

* D = V_D (finest level only) plus every vertex with mu_D < sigma; the first pass walks the
  remaining vertices in a Cuthill-McKee order of the graph induced on V minus D by the edges with
  positive trace: start at a vertex of minimum degree (lowest id on ties), breadth first, each
  vertex's unvisited neighbours appended by ascending (degree, id); further components restart
  the same way.
* A vertex leaves the pool T when it is walked (as C_i) or matched; candidates C_j come from T.
* The candidate is the neighbour with *minimal* mu_s (R = 1; the algorithm's form).  Values
  within a relative band ``tie_rtol`` of the minimum tie; among ties the one earliest in the
  current walk order wins.  It is accepted when mu_b < sigma and, if the union has more than two
  vertices, mu_g < sigma computed from the level's own (not intermediate) weight matrices.
* After a pass the new list is the pairs in formation order followed by the singles in order;
  the next pass walks that list in reverse.  Between passes the intermediate edge / vertex
  weights follow Thm thm:cemats (the first one also absorbs the edges to D).  The final coarse
  weights are computed from the level's weights and the final agglomerates directly.
* Coarse vertex I is the I-th final list entry; its position is the mean of its members'
  positions (remark after Def. def:pwp).
"""
from __future__ import annotations

import collections
import dataclasses

import numpy as np

from .auxtop import AuxLevel, coarse_aux, dhat_all
from .criteria import mu_D, mu_b, mu_g, mu_s, trace_strength


def cuthill_mckee(level: AuxLevel, free_mask) -> list:
    n = level.n
    trE = np.trace(level.E, axis1=1, axis2=2) if level.E.size else np.zeros(0)
    adj = [[] for _ in range(n)]
    for e, (i, j) in enumerate(level.edges):
        if trE[e] > 0.0 and free_mask[i] and free_mask[j]:
            adj[i].append(int(j))
            adj[j].append(int(i))
    deg = np.array([len(a) for a in adj], dtype=np.int64)
    starts = sorted((int(deg[v]), v) for v in range(n) if free_mask[v])
    visited = np.zeros(n, dtype=bool)
    order = []
    ptr = 0
    nfree = len(starts)
    while len(order) < nfree:
        while visited[starts[ptr][1]]:
            ptr += 1
        s = starts[ptr][1]
        visited[s] = True
        queue = collections.deque([s])
        while queue:
            v = queue.popleft()
            order.append(v)
            nb = sorted((int(deg[u]), u) for u in adj[v] if not visited[u])
            for _, u in nb:
                visited[u] = True
                queue.append(u)
    return order


@dataclasses.dataclass
class MatchingResult:
    aggs: list            # list of sorted member arrays; coarse id = position
    dmask: np.ndarray     # bool (n,), the dropped set D
    coarse_coords: np.ndarray
    coarse_level: AuxLevel
    cm_order: list
    pass_lists: list      # per pass: list of member tuples in list order
    min_margin: float     # min |mu - sigma| / sigma over all threshold decisions
    max_tie: int          # largest tie group met when picking a candidate


def _mean_pos(coords, members):
    s = np.zeros(3)
    for i in sorted(members):
        s = s + coords[i]
    return s / len(members)


def successive_matching(level: AuxLevel, vd_mask, sigma=20.0, rounds=2, tie_rtol=1e-12,
                        tau=1e-10, mu_s_only=False) -> MatchingResult:
    """mu_s_only: pair the candidate of smallest mu_s without the robust tests (mu_b, mu_g), the
    scalar-only coarsening of the paper's coefficient-jump comparison (Figs. fig:2dc_rob /
    fig:2dc_norob)."""
    n = level.n
    margin = [float("inf")]
    max_tie = [0]

    def note(mu):
        if np.isfinite(mu):
            margin[0] = min(margin[0], abs(mu - sigma) / sigma)

    Dhat = dhat_all(level)
    dmask = np.asarray(vd_mask, dtype=bool).copy()
    for i in range(n):
        if not dmask[i]:
            md = mu_D(level, i, Dhat, tau)
            note(md)
            if md < sigma:
                dmask[i] = True
    free = ~dmask
    cm = cuthill_mckee(level, free)

    work = level
    work_dhat = Dhat
    in_T = free.copy()
    members = {i: [i] for i in range(n)}
    order = cm
    pass_lists = []
    entries = []
    for p in range(1, rounds + 1):
        pos = {v: a for a, v in enumerate(order)}
        mtr = trace_strength(work)
        pairs, singles = [], []
        for ci in order:
            if not in_T[ci]:
                continue
            in_T[ci] = False
            nb, _ = work.neighbors(ci)
            cands = {}
            for cj in nb.tolist():
                if in_T[cj]:
                    ms = mu_s(work, ci, cj, mtr)
                    note(ms)
                    if ms < sigma:
                        cands[cj] = ms
            matched = None
            while cands:
                mmin = min(cands.values())
                tied = [c for c, v in cands.items() if v <= mmin * (1.0 + tie_rtol)]
                max_tie[0] = max(max_tie[0], len(tied))
                cj = min(tied, key=pos.__getitem__)
                if mu_s_only:
                    matched = cj
                    break
                mu = mu_b(work, ci, cj, work_dhat, tau)
                note(mu)
                ok = mu < sigma
                if ok and len(members[ci]) + len(members[cj]) > 2:
                    mg = mu_g(level, members[ci] + members[cj], Dhat, tau)
                    note(mg)
                    ok = mg < sigma
                if ok:
                    matched = cj
                    break
                del cands[cj]
            if matched is not None:
                pairs.append((ci, matched))
                in_T[matched] = False
            else:
                singles.append(ci)
        groups = [list(pq) for pq in pairs] + [[s] for s in singles]
        entries = [members[g[0]] + (members[g[1]] if len(g) == 2 else []) for g in groups]
        pass_lists.append([tuple(sorted(m)) for m in entries])
        if p < rounds:
            icoords = np.array([_mean_pos(level.coords, m) for m in entries]).reshape(-1, 3)
            wmask = dmask if p == 1 else np.zeros(work.n, dtype=bool)
            work = coarse_aux(work, groups, wmask, icoords)
            work_dhat = dhat_all(work)
            members = {I: list(m) for I, m in enumerate(entries)}
            in_T = np.ones(len(entries), dtype=bool)
            order = list(range(len(entries)))[::-1]
    aggs = [np.array(sorted(m), dtype=np.int64) for m in entries]
    ccoords = np.array([_mean_pos(level.coords, m) for m in aggs]).reshape(-1, 3)
    clevel = coarse_aux(level, aggs, dmask, ccoords)
    return MatchingResult(aggs, dmask, ccoords, clevel, cm, pass_lists, margin[0], max_tie[0])
