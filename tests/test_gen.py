"""Pins of the generated problems (paper section "fem"): the rigid body modes (section "amg")
lie in the kernel of the BC-free elasticity matrix, the matrix is symmetric, and a linear
displacement field has exactly the energy of the continuous bilinear form."""
import numpy as np
import scipy.sparse as sp

from gen import kuhn_mesh, lame_from_young, make_problem
from gen.kuhn import _p1_gradients, _tet_offsets


def _csr(p):
    n = p.n_dofs
    return sp.bsr_matrix((p.vals, p.col_idx, p.row_ptr), shape=(n, n)).tocsr()


def _rbm(coords):
    n = coords.shape[0]
    R = np.zeros((3 * n, 6))
    for m in range(3):
        R[m::3, m] = 1.0
        e = np.zeros(3)
        e[m] = 1.0
        R[:, 3 + m] = np.cross(coords, e).ravel()   # x cross e_m
    return R


def test_exact_block_counts():
    # 14 neighbours per interior vertex of the Kuhn mesh
    p = make_problem(17)
    assert p.nnzb == 66961 and p.n_dofs == 14739 and p.n_free_dofs == 13872
    interior = np.diff(p.row_ptr).max()
    assert interior == 15


def test_symmetric_and_rbm_kernel():
    p = make_problem(6, nu=0.37)
    A = _csr(p)
    assert abs(A - A.T).max() < 1e-15
    R = _rbm(p.coords)
    assert np.abs(A @ R).max() < 1e-13 * abs(A).max()


def test_patch_test_linear_field_energy():
    # u(x) = G x: u^T A_N u = |Omega| (2 mu eps:eps + lambda tr(eps)^2)
    rng = np.random.default_rng(7)
    G = rng.standard_normal((3, 3))
    E, nu = 2.5, 0.31
    p = make_problem(5, E=E, nu=nu)
    mu, lam = lame_from_young(E, nu)
    u = (p.coords @ G.T).ravel()
    eps = 0.5 * (G + G.T)
    expect = 2 * mu * np.sum(eps * eps) + lam * np.trace(eps) ** 2
    assert abs(u @ (_csr(p) @ u) - expect) < 1e-12 * abs(expect)


def test_tet_volumes_fill_cube():
    offs = _tet_offsets()
    vols = [_p1_gradients(offs[t].astype(float))[1] for t in range(6)]
    assert abs(sum(vols) - 1.0) < 1e-15
    g, _ = _p1_gradients(offs[0].astype(float))
    assert np.abs(g.sum(axis=0)).max() < 1e-15      # partition of unity


def test_poisson_kuhn_laplacian_is_m_matrix():
    # The Kuhn triangulation gives the 7-point finite difference Laplacian (times h) at
    # interior vertices, and an M-matrix with zero row sums without boundary conditions.
    n = 6
    p = make_problem(n, kind="poisson", clamp="none")
    A = _csr(p).toarray()
    h = kuhn_mesh(n).h
    v = 3 + n * (3 + n * 3)
    row = A[v][A[v] != 0] / h
    assert sorted(np.round(row, 12).tolist()) == [-1.0] * 6 + [6.0]
    off = A - np.diag(np.diag(A))
    assert off.max() <= 0.0
    assert np.abs(A.sum(axis=1)).max() < 1e-14


def test_rhs_seeded_and_clamped():
    p = make_problem(5, seed=3)
    b = np.random.default_rng(3).uniform(-1, 1, p.n_dofs)
    mask = np.repeat(p.dirichlet.astype(bool), 3)
    assert np.array_equal(p.b[~mask], b[~mask]) and np.all(p.b[mask] == 0)
    assert p.dirichlet.sum() == 25
