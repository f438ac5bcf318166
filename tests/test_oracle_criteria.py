"""Pins of the coarsening measures: mu_b = mu_g on pairs when M = 0 and mu_g <= mu_b otherwise
(Lemma thm:mu2 and the remark after it), the two-grid bound K_TG <= max{mu_D, mu_g} (Thm
thm:mu1 with eq. ktg_generic of Lemma thm:ktg_generic) and the resulting convergence factor
bound (eq. tgc_generic), dense on tiny meshes, for elasticity and for the scalar M-matrix case
where Ahat = A exactly."""
import numpy as np
import pytest
import scipy.linalg as sla
import scipy.sparse as sp

from gen import make_problem
from oracle.auxtop import AuxLevel, assemble_aux_dense, dhat_all, finest_aux
from oracle.coarsen import successive_matching
from oracle.criteria import mu_D, mu_b, mu_g, mu_s, trace_strength
from oracle.dense import pinv_tau
from oracle.prolong import tentative_prolongation

rng = np.random.default_rng(9)


def _psd(n, rank=None):
    X = rng.standard_normal((n, n if rank is None else rank))
    return X @ X.T


def _rand_level(n_v=4, rankE=6, withM=False):
    p = make_problem(n_v)
    base = finest_aux(3, p.coords, p.row_ptr, p.col_idx, p.vals)
    E = np.array([_psd(6, rankE) for _ in range(base.edges.shape[0])])
    M = np.array([_psd(6, 2) for _ in range(base.n)]) if withM else np.zeros((base.n, 6, 6))
    return AuxLevel(6, p.coords.copy(), base.edges, E, M)


def test_mu_b_equals_mu_g_on_pairs_without_vertex_weights():
    lev = _rand_level()
    D = dhat_all(lev)
    for e in rng.choice(lev.edges.shape[0], 8, replace=False):
        i, j = lev.edges[e]
        b, g = mu_b(lev, i, j, D), mu_g(lev, [i, j], D)
        assert abs(b - g) < 1e-8 * b


def test_mu_b_equals_mu_g_finest_elasticity():
    p = make_problem(5)
    lev = finest_aux(3, p.coords, p.row_ptr, p.col_idx, p.vals)
    D = dhat_all(lev)
    for e in rng.choice(lev.edges.shape[0], 10, replace=False):
        i, j = lev.edges[e]
        b, g = mu_b(lev, i, j, D), mu_g(lev, [i, j], D)
        assert np.isfinite(b) and abs(b - g) < 1e-7 * b


def test_mu_g_bounded_by_mu_b_with_vertex_weights():
    lev = _rand_level(withM=True)
    D = dhat_all(lev)
    for e in rng.choice(lev.edges.shape[0], 8, replace=False):
        i, j = lev.edges[e]
        assert mu_g(lev, [i, j], D) <= mu_b(lev, i, j, D) * (1 + 1e-9)


def test_mu_s_and_mu_D_closed_forms():
    # two vertices joined by one edge: mu_s = sqrt(tr E tr E) / tr E = 1
    x = np.array([[0.0, 0, 0], [1.0, 0, 0]])
    E = _psd(6)[None]
    lev = AuxLevel(6, x, np.array([[0, 1]]), E, np.zeros((2, 6, 6)))
    assert abs(mu_s(lev, 0, 1, trace_strength(lev)) - 1.0) < 1e-15
    # mu_D = 1 when the whole diagonal is vertex weight; +inf when M = 0
    lev2 = AuxLevel(6, x, np.array([[0, 1]]), 0 * E, np.array([_psd(6), np.zeros((6, 6))]))
    D = dhat_all(lev2)
    assert abs(mu_D(lev2, 0, D) - 1.0) < 1e-12
    lev3 = AuxLevel(6, x, np.array([[0, 1]]), E, np.zeros((2, 6, 6)))
    assert mu_D(lev3, 0, dhat_all(lev3)) == float("inf")
    # dominance: M = D/3 -> mu_D = 3 when the edge weight equals 2 M
    M0 = _psd(6)
    lev4 = AuxLevel(6, np.array([[0.0, 0, 0], [0.0, 0, 0]]), np.array([[0, 1]]),
                    (2 * M0)[None], np.array([M0, M0]))
    assert abs(mu_D(lev4, 0, dhat_all(lev4)) - 3.0) < 1e-10


def _range_basis(X, tau=1e-10):
    lam, U = np.linalg.eigh(0.5 * (X + X.T))
    keep = lam > tau * lam.max()
    return U[:, keep], lam[keep]


def _ktg(Ahat, P, tau=1e-10):
    """eq. ktg_generic: sup over ker(Ahat)^perp of v^T Dh (I - P (P^T Dh P)^+ P^T Dh) v / v^T Ahat v."""
    k = 6 if Ahat.shape[0] % 6 == 0 and P.shape[1] % 6 == 0 else 1
    n = Ahat.shape[0] // k
    Dh = np.zeros_like(Ahat)
    for i in range(n):
        Dh[i * k:(i + 1) * k, i * k:(i + 1) * k] = Ahat[i * k:(i + 1) * k, i * k:(i + 1) * k]
    N = Dh - Dh @ P @ pinv_tau(P.T @ Dh @ P, tau) @ P.T @ Dh
    U, lam = _range_basis(Ahat, tau)
    W = U / np.sqrt(lam)
    return np.linalg.eigvalsh(W.T @ N @ W).max()


def _two_grid_factor(A, P, bs):
    """rho(E_TG) for block Gauss-Seidel (natural order) pre / post smoothing."""
    n = A.shape[0]
    Mgs = np.tril(A)
    for i in range(0, n, bs):
        Mgs[i:i + bs, i:i + bs] = A[i:i + bs, i:i + bs]
    Ac = P.T @ A @ P
    C = np.eye(n) - P @ pinv_tau(Ac, 1e-12) @ P.T @ A
    S1 = np.eye(n) - np.linalg.solve(Mgs, A)
    S2 = np.eye(n) - np.linalg.solve(Mgs.T, A)
    E = S2 @ C @ S1
    return np.abs(np.linalg.eigvals(E)).max(), Mgs


@pytest.mark.parametrize("kind", ["elasticity", "poisson"])
def test_two_grid_bound(kind):
    if kind == "elasticity":
        p = make_problem(4, E=1.0, nu=0.3, seed=0)
        dim, k = 3, 6
    else:
        p = make_problem(6, kind="poisson", clamp="all", seed=0)
        dim, k = 1, 1
    lev = finest_aux(dim, p.coords, p.row_ptr, p.col_idx, p.vals)
    vd = p.dirichlet.astype(bool)
    res = successive_matching(lev, vd, sigma=20.0, rounds=2)
    free = ~res.dmask
    fidx = np.nonzero(free)[0]
    n = lev.n
    # aux matrix on the free vertices (Dirichlet vertices eliminated)
    Ahat_full = assemble_aux_dense(lev)
    sel = (fidx[:, None] * k + np.arange(k)).ravel()
    Ahat = Ahat_full[np.ix_(sel, sel)]
    agg_of = np.full(n, -1)
    for I, mem in enumerate(res.aggs):
        agg_of[mem] = I
    P6 = tentative_prolongation(n, k, k, lev.coords, agg_of, res.coarse_coords)
    P6 = P6.to_scipy().toarray()[sel]
    K = _ktg(Ahat, P6)
    Dh = dhat_all(lev)
    mug = max([mu_g(lev, a, Dh) for a in res.aggs if len(a) > 1], default=0.0)
    assert K <= mug * (1 + 1e-8) + 1e-10
    assert mug < 20.0
    # FE matrix on free dofs and the restricted (real-dof) prolongation
    A = sp.bsr_matrix((p.vals, p.col_idx, p.row_ptr), shape=(p.n_dofs,) * 2).toarray()
    fd = (fidx[:, None] * dim + np.arange(dim)).ravel()
    A = A[np.ix_(fd, fd)]
    Pr = tentative_prolongation(n, k, dim, lev.coords, agg_of, res.coarse_coords)
    Pr = Pr.to_scipy().toarray()[fd]
    # c1 At <= A <= c2 At with At = E^T Ahat E (E = displacement embedding)
    Emb = np.zeros((Ahat.shape[0], A.shape[0]))
    for a in range(fidx.size):
        Emb[a * k:a * k + dim, a * dim:(a + 1) * dim] = np.eye(dim)
    At = Emb.T @ Ahat @ Emb
    lam = sla.eigh(A, At, eigvals_only=True)
    c1, c2 = lam.min(), lam.max()
    if kind == "poisson":
        assert abs(c1 - 1) < 1e-10 and abs(c2 - 1) < 1e-10    # Ahat = A exactly
    rho, Mgs = _two_grid_factor(A, Pr, dim)
    Dg = np.zeros_like(A)
    for i in range(0, A.shape[0], dim):
        Dg[i:i + dim, i:i + dim] = A[i:i + dim, i:i + dim]
    Mt = Mgs @ np.linalg.solve(Mgs + Mgs.T - A, Mgs.T)
    d2 = sla.eigh(Dg, Mt, eigvals_only=True).max()
    bound = 1.0 - c1 / (c2 * d2 * K)
    assert rho <= bound + 1e-10
    assert rho < 1.0
