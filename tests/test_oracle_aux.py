"""Pins of the auxiliary topology (Def. def:deng, eq. auxa; Thm thm:deng_elast; Thm thm:cemats;
scalar M-matrix splitting of section "deng")."""
import numpy as np
import scipy.sparse as sp

from gen import make_problem
from oracle.auxtop import AuxLevel, assemble_aux_dense, coarse_aux, finest_aux
from oracle.dense import q_half, q_transport
from oracle.prolong import tentative_prolongation

rng = np.random.default_rng(5)


def _psd(n, rank=None):
    X = rng.standard_normal((n, n if rank is None else rank))
    return X @ X.T


def _csr(p):
    return sp.bsr_matrix((p.vals, p.col_idx, p.row_ptr), shape=(p.n_dofs,) * 2).tocsr()


def _random_level(p, full=True):
    base = finest_aux(3, p.coords, p.row_ptr, p.col_idx, p.vals)
    m, n = base.edges.shape[0], base.n
    E = np.array([_psd(6, 6 if full else 2) for _ in range(m)])
    M = np.array([_psd(6, 3) if rng.random() < 0.3 else np.zeros((6, 6)) for _ in range(n)])
    return AuxLevel(6, p.coords.copy(), base.edges, E, M)


def _global_rbm6(coords, w):
    # (u_i, r_i) = Q^{H->i} w for H at the origin
    return np.concatenate([q_transport(np.zeros(3), x, 6) @ w for x in coords])


def test_aux_matrix_kernel_and_energy():
    p = make_problem(4)
    lev = _random_level(p)
    lev.M[:] = 0.0
    A = assemble_aux_dense(lev)
    assert np.allclose(A, A.T, atol=1e-12)
    for _ in range(3):
        u = _global_rbm6(lev.coords, rng.standard_normal(6))
        assert np.abs(A @ u).max() < 1e-11 * np.abs(A).max() * np.abs(u).max()
    # energy of eq. deng (each edge once) equals u^T Ahat u
    lev2 = _random_level(p)
    A2 = assemble_aux_dense(lev2)
    u = rng.standard_normal(A2.shape[0])
    U = u.reshape(-1, 6)
    energy = sum(U[i] @ lev2.M[i] @ U[i] for i in range(lev2.n))
    for e, (i, j) in enumerate(lev2.edges):
        d = q_half(lev2.coords[i], lev2.coords[j], 6) @ U[i] - q_half(lev2.coords[j],
                                                                       lev2.coords[i], 6) @ U[j]
        energy += d @ lev2.E[e] @ d
    assert abs(energy - u @ A2 @ u) < 1e-11 * abs(energy)


def test_finest_elasticity_edge_matrices_reduce_to_truss():
    # Thm thm:deng_elast: E^T Ahat E equals the 3x3 form with E^ij = c t t^T and Q = I
    p = make_problem(4)
    lev = finest_aux(3, p.coords, p.row_ptr, p.col_idx, p.vals)
    A6 = assemble_aux_dense(lev)
    n = lev.n
    Emb = np.zeros((6 * n, 3 * n))
    for i in range(n):
        Emb[6 * i:6 * i + 3, 3 * i:3 * i + 3] = np.eye(3)
    At = np.zeros((3 * n, 3 * n))
    for e, (i, j) in enumerate(lev.edges):
        Ee = lev.E[e][:3, :3]
        for a, b, s in ((i, i, 1), (j, j, 1), (i, j, -1), (j, i, -1)):
            At[3 * a:3 * a + 3, 3 * b:3 * b + 3] += s * Ee
    assert np.allclose(Emb.T @ A6 @ Emb, At, atol=1e-13)
    # c^ij is the mean absolute entry of (A_N)_ij and tr E^ij = c^ij (unit direction)
    e = 7
    i, j = lev.edges[e]
    s, t = p.row_ptr[i], p.row_ptr[i + 1]
    blk = p.vals[s + np.nonzero(p.col_idx[s:t] == j)[0][0]]
    assert abs(np.trace(lev.E[e]) - np.abs(blk).mean()) < 1e-15
    assert np.all(lev.M == 0)


def test_scalar_m_matrix_splitting_is_exact():
    # section "deng": for an M-matrix, E^ij = |A_ij|, M^i = A_ii - sum |A_ij| reproduce A
    p = make_problem(5, kind="poisson", clamp="none")
    lev = finest_aux(1, p.coords, p.row_ptr, p.col_idx, p.vals)
    A = _csr(p).toarray()
    assert np.allclose(assemble_aux_dense(lev), A, atol=1e-14)
    # a zero-order term shows up in M (eq. gg with beta > 0)
    A2 = A + 0.3 * np.eye(A.shape[0])
    vals = p.vals.copy()
    rows = np.repeat(np.arange(p.n_vertices), np.diff(p.row_ptr))
    vals[rows == p.col_idx] += 0.3
    lev2 = finest_aux(1, p.coords, p.row_ptr, p.col_idx, vals)
    assert np.allclose(assemble_aux_dense(lev2), A2, atol=1e-14)
    assert np.allclose(lev2.M[:, 0, 0], 0.3)


def _random_agglomerates(n, dfrac=0.15):
    perm = rng.permutation(n)
    nd = int(dfrac * n)
    dmask = np.zeros(n, dtype=bool)
    dmask[perm[:nd]] = True
    rest = perm[nd:]
    aggs, pos = [], 0
    while pos < rest.size:
        s = int(rng.integers(1, 5))
        aggs.append(np.sort(rest[pos:pos + s]))
        pos += s
    return aggs, dmask


def test_coarse_edge_matrices_galerkin_identity():
    # Thm thm:cemats: P^T Ahat P == Ahat_c assembled from E^IJ, M^I (incl. D absorption)
    p = make_problem(4)
    lev = _random_level(p)
    aggs, dmask = _random_agglomerates(lev.n)
    cc = rng.standard_normal((len(aggs), 3))     # any coarse positions
    clev = coarse_aux(lev, aggs, dmask, cc)
    agg_of = np.full(lev.n, -1)
    for I, mem in enumerate(aggs):
        agg_of[mem] = I
    P = tentative_prolongation(lev.n, 6, 6, lev.coords, agg_of, cc).to_scipy().toarray()
    lhs = P.T @ assemble_aux_dense(lev) @ P
    rhs = assemble_aux_dense(clev)
    assert np.abs(lhs - rhs).max() < 1e-11 * np.abs(lhs).max()


def test_coarse_edge_matrices_galerkin_identity_finest_elasticity():
    p = make_problem(5)
    lev = finest_aux(3, p.coords, p.row_ptr, p.col_idx, p.vals)
    aggs, dmask = _random_agglomerates(lev.n, 0.2)
    cc = np.array([lev.coords[a].mean(axis=0) for a in aggs])
    clev = coarse_aux(lev, aggs, dmask, cc)
    agg_of = np.full(lev.n, -1)
    for I, mem in enumerate(aggs):
        agg_of[mem] = I
    P = tentative_prolongation(lev.n, 6, 6, lev.coords, agg_of, cc).to_scipy().toarray()
    lhs = P.T @ assemble_aux_dense(lev) @ P
    assert np.abs(lhs - assemble_aux_dense(clev)).max() < 1e-12 * np.abs(lhs).max()
