"""Pins of three parts of the setup that had only self-consistency checks:

* the Cuthill-McKee walk order that starts the first matching pass (Algorithm alg:pwagg names
  a Cuthill-McKee order without fixing its details; the reading: induced graph on V minus D with
  the edges of positive trace, start at a vertex of minimum degree with the lowest id, breadth
  first, unvisited neighbours appended by ascending (degree, id), restart per component);
* the smallest-last greedy colouring behind the multicolour Gauss-Seidel smoother (Algorithm
  alg:tg with M and M^T): every colour class must be an independent set of the block graph of
  A_l, or a colour sweep is not a Gauss-Seidel sweep;
* the neighbour maximum inside mu_s (Def. def:muc): m_i = max(tr M^i, max over l != i of
  tr E^il).

The expected orders and colours below were derived by hand from those definitions; the
degeneracy bound is checked against a brute-force degeneracy over all vertex subsets."""
import itertools

import numpy as np
import pytest

from gen import make_problem
from oracle import hierarchy as H
from oracle.auxtop import AuxLevel
from oracle.coarsen import cuthill_mckee
from oracle.criteria import mu_s, trace_strength
from oracle.prolong import BCSR


def _level(n, edges, traces, Mtr=None):
    """A k = 1 auxiliary level with the given edges (i < j) and edge traces."""
    edges = np.array(sorted(edges), dtype=np.int64).reshape(-1, 2)
    tr = dict(zip(map(tuple, sorted(edges.tolist())), traces)) if isinstance(traces, list) else traces
    E = np.array([[[tr[(int(i), int(j))]]] for i, j in edges], dtype=np.float64).reshape(-1, 1, 1)
    M = np.zeros((n, 1, 1)) if Mtr is None else np.asarray(Mtr, dtype=np.float64).reshape(n, 1, 1)
    coords = np.zeros((n, 3))
    coords[:, 0] = np.arange(n)
    return AuxLevel(1, coords, edges, E, M)


# ---------------------------------------------------------------- Cuthill-McKee walk order

def test_cuthill_mckee_hand_derived_order():
    # free component {0..5}: every vertex of degree 3 except the leaf 5; vertex 4's unvisited
    # neighbours 2 and 3 tie on degree (3) and go by id; vertex 6 is in D, so its edges (5,6),
    # (6,7) do not join the components; edge (1,5) has zero trace and does not count; vertex 10
    # only touches a zero-trace edge: degree 0, so it is the first start.  Second component
    # {7, 8, 9} is a path that restarts at its lowest-id leaf 7.
    edges = [(0, 1), (0, 2), (0, 3), (1, 2), (1, 3), (2, 4), (3, 4), (4, 5), (1, 5), (5, 6),
             (6, 7), (7, 8), (8, 9), (9, 10)]
    tr = {e: 1.0 + 0.1 * k for k, e in enumerate(edges)}
    tr[(1, 5)] = 0.0
    tr[(9, 10)] = 0.0
    lev = _level(11, edges, tr)
    free = np.ones(11, dtype=bool)
    free[6] = False
    assert cuthill_mckee(lev, free) == [10, 5, 4, 2, 3, 0, 1, 7, 8, 9]


def test_cuthill_mckee_neighbours_by_degree_then_id():
    # star centre 0 with leaves 1..3 and a second ring: the centre's neighbours have degrees
    # 3 (vertex 1), 1 (vertex 2), 2 (vertex 3); the walk starts at the lowest-id degree-1 vertex.
    #   0-1, 0-2, 0-3, 1-4, 1-5, 3-6, 4-5
    edges = [(0, 1), (0, 2), (0, 3), (1, 4), (1, 5), (3, 6), (4, 5)]
    lev = _level(7, edges, [1.0] * len(edges))
    free = np.ones(7, dtype=bool)
    # degrees: 0:3 1:3 2:1 3:2 4:2 5:2 6:1 -> start 2; then 0; 0's unvisited neighbours
    # 3 (deg 2) before 1 (deg 3); then 3 -> 6; then 1 -> 4, 5
    assert cuthill_mckee(lev, free) == [2, 0, 3, 1, 6, 4, 5]


def test_cuthill_mckee_covers_free_vertices_once():
    p = make_problem(6, seed=1)
    from oracle.auxtop import finest_aux
    lev = finest_aux(3, p.coords, p.row_ptr, p.col_idx, p.vals)
    free = ~p.dirichlet.astype(bool)
    order = cuthill_mckee(lev, free)
    assert sorted(order) == np.nonzero(free)[0].tolist()


# ------------------------------------------------------- smallest-last greedy colouring

def _graph_bcsr(n, edges):
    rows = [[i] for i in range(n)]
    for i, j in edges:
        rows[i].append(j)
        rows[j].append(i)
    rp = np.zeros(n + 1, dtype=np.int64)
    cols = []
    for i in range(n):
        c = sorted(set(rows[i]))
        cols += c
        rp[i + 1] = rp[i] + len(c)
    return BCSR(n, n, rp, np.array(cols, dtype=np.int64), np.ones((len(cols), 1, 1)))


def test_smallest_last_hand_derived():
    # triangle 0-1-2, pendant 3 at 0, vertex 4 joined to 1 and 2.  Removal by minimum remaining
    # degree (lowest id on ties): 3 (deg 1), 0 (deg 2), 1 (deg 2), 2 (deg 1), 4 -> order is the
    # reverse; first-fit colours in that order: 4:0, 2:1, 1:2, 0:0, 3:1.
    A = _graph_bcsr(5, [(0, 1), (0, 2), (1, 2), (0, 3), (1, 4), (2, 4)])
    assert H.smallest_last_order(A) == [4, 2, 1, 0, 3]
    assert H.greedy_coloring(A).tolist() == [0, 2, 1, 1, 0]


def _degeneracy_brute(n, edges):
    """max over non-empty vertex subsets S of the minimum degree of the graph induced on S."""
    best = 0
    for r in range(1, n + 1):
        for S in itertools.combinations(range(n), r):
            s = set(S)
            deg = {v: 0 for v in S}
            for i, j in edges:
                if i in s and j in s:
                    deg[i] += 1
                    deg[j] += 1
            best = max(best, min(deg.values()))
    return best


def test_smallest_last_colouring_within_degeneracy_bound():
    # greedy colouring in smallest-last order uses at most degeneracy + 1 colours (Matula &
    # Beck 1983); an order that is not smallest-last breaks this on some of these graphs
    rng = np.random.default_rng(11)
    for trial in range(40):
        n = int(rng.integers(4, 11))
        pairs = [(i, j) for i in range(n) for j in range(i + 1, n)]
        keep = rng.random(len(pairs)) < rng.uniform(0.15, 0.6)
        edges = [pq for pq, k in zip(pairs, keep) if k]
        A = _graph_bcsr(n, edges)
        col = H.greedy_coloring(A)
        assert all(col[i] != col[j] for i, j in edges)
        assert col.max() + 1 <= _degeneracy_brute(n, edges) + 1, (trial, n, edges)


def test_crown_graph_needs_two_colours():
    # crown graph S_4^0 (K_{4,4} minus a perfect matching): first-fit in the order
    # a0 b0 a1 b1 ... needs 4 colours; smallest-last colours the bipartite graph with 2
    n = 4
    edges = [(i, n + j) for i in range(n) for j in range(n) if i != j]
    col = H.greedy_coloring(_graph_bcsr(2 * n, edges))
    assert col.max() + 1 == 2
    assert all(col[i] != col[j] for i, j in edges)


@pytest.mark.parametrize("case", ["cube7", "ragged", "poisson8", "spheres9"])
def test_every_level_colour_class_is_independent(case):
    if case == "cube7":
        p = make_problem(7, seed=2)
    elif case == "ragged":
        p = make_problem(11, ny=7, nz=5, nu=0.35, seed=4)
    elif case == "poisson8":
        p = make_problem(8, kind="poisson", clamp="all")
    else:
        p = make_problem(9, inclusions=4, geometry_seed=2, seed=1)
    h = H.setup(p.dim, p.coords, p.row_ptr, p.col_idx, p.vals, p.dirichlet)
    assert h.n_levels >= 2
    for lv in h.levels:
        A = lv.A
        rows = np.repeat(np.arange(A.n_rows), np.diff(A.row_ptr))
        off = rows != A.col
        assert not np.any(lv.colors[rows[off]] == lv.colors[A.col[off]])
        assert lv.colors.min() == 0
        # colours are 0..C-1 with none skipped
        assert np.array_equal(np.unique(lv.colors), np.arange(lv.colors.max() + 1))


# ---------------------------------------------------------- mu_s neighbour maximum

def test_mu_s_uses_the_largest_incident_trace():
    # star: centre 0, leaves 1, 2, 3 with edge traces 1, 3, 2 and no vertex weights.
    # m_0 = max(1, 3, 2) = 3, m_1 = 1, m_2 = 3, m_3 = 2
    lev = _level(4, [(0, 1), (0, 2), (0, 3)], [1.0, 3.0, 2.0])
    m = trace_strength(lev)
    assert m.tolist() == [3.0, 1.0, 3.0, 2.0]
    assert mu_s(lev, 0, 1, m) == pytest.approx(np.sqrt(3.0 * 1.0) / 1.0, rel=1e-15)
    assert mu_s(lev, 0, 2, m) == pytest.approx(np.sqrt(3.0 * 3.0) / 3.0, rel=1e-15)
    assert mu_s(lev, 3, 0, m) == pytest.approx(np.sqrt(2.0 * 3.0) / 2.0, rel=1e-15)


def test_mu_s_vertex_weight_dominates_when_larger():
    # path 0-1-2 with traces 2 and 5, tr M = (0, 7, 1): m = (2, 7, 5)
    lev = _level(3, [(0, 1), (1, 2)], [2.0, 5.0], Mtr=[0.0, 7.0, 1.0])
    m = trace_strength(lev)
    assert m.tolist() == [2.0, 7.0, 5.0]
    assert mu_s(lev, 0, 1, m) == pytest.approx(np.sqrt(14.0) / 2.0, rel=1e-15)
    assert mu_s(lev, 2, 1, m) == pytest.approx(np.sqrt(35.0) / 5.0, rel=1e-15)
    # no edge (or a zero-trace edge): +inf
    assert mu_s(lev, 0, 2, m) == float("inf")


def test_mu_s_symmetric_and_at_least_one():
    # m_i >= tr E^ij and m_j >= tr E^ij, so mu_s >= 1, with equality iff the edge is the
    # strongest at both ends
    rng = np.random.default_rng(3)
    n = 9
    pairs = [(i, j) for i in range(n) for j in range(i + 1, n) if rng.random() < 0.4]
    lev = _level(n, pairs, list(rng.uniform(0.1, 5.0, len(pairs))),
                 Mtr=rng.uniform(0.0, 3.0, n))
    m = trace_strength(lev)
    for i, j in pairs:
        a, b = mu_s(lev, i, j, m), mu_s(lev, j, i, m)
        assert a == b and a >= 1.0 - 1e-15
