"""Pins of the hierarchy and the solver: rigid-body-mode reproduction by the tentative and the
auxiliary smoothed prolongations (Defs. def:pwp, def:pwp_el, def:aux_sp), symmetric coarse
operators with the modes in their kernel (section "prol"), the 3x3 reduced form of finest
level edge-matrix rows, invariants of the successive matching (Algorithm alg:pwagg), the
smoother as a block triangular solve, the coarsest level regularization (section "sing2"),
and PCG against direct solves and the Krylov minimizer (section "res")."""
import numpy as np
import pytest
import scipy.linalg as sla
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from gen import make_problem
from oracle import hierarchy as H
from oracle.auxtop import dhat_all, finest_aux
from oracle.criteria import mu_b, mu_g, mu_s, trace_strength
from oracle.dense import kernel_basis, pinv_tau, q_transport
from oracle.prolong import ROW_A, smoothed_prolongation, tentative_prolongation
from oracle.solve import _ops, gs_sweep, pcg, vcycle


def _setup(p, **kw):
    return H.setup(p.dim, p.coords, p.row_ptr, p.col_idx, p.vals, p.dirichlet,
                   H.SetupParams(**kw) if kw else None)


@pytest.fixture(scope="module")
def neumann():
    p = make_problem(7, clamp="none", nu=0.25)
    h = H.setup(p.dim, p.coords, p.row_ptr, p.col_idx, p.vals, p.dirichlet,
                factor_coarsest=False)
    return p, h


@pytest.fixture(scope="module")
def clamped():
    p = make_problem(7, seed=2)
    return p, _setup(p)


def _rbm_coarse(coords, d, r, k):
    if k == 1:
        return np.ones(coords.shape[0]) * d[0]
    return np.concatenate([np.concatenate([d + np.cross(x, r), r]) for x in coords])


@pytest.fixture(scope="module", params=["paper caps", "caps 6/4/3", "caps 6/4/4 sigma 18"])
def neumann_caps(request, neumann):
    # the P_s row caps and sigma are free parameters: rigid body modes must be reproduced for any
    # of them
    if request.param == "paper caps":
        return neumann
    p = neumann[0]
    prm = (H.SetupParams(cap_std_l0=6, cap_std=4, cap_aux=3) if request.param == "caps 6/4/3"
           else H.SetupParams(cap_std_l0=6, cap_std=4, cap_aux=4, sigma=18.0))
    h = H.setup(p.dim, p.coords, p.row_ptr, p.col_idx, p.vals, p.dirichlet, prm,
                factor_coarsest=False)
    return p, h


def test_kernel_reproduction_all_levels(neumann_caps):
    p, h = neumann_caps
    rng = np.random.default_rng(1)
    d, r = rng.standard_normal(3), rng.standard_normal(3)
    uf = np.concatenate([d + np.cross(x, r) for x in p.coords])
    assert all(not lv.match.dmask.any() for lv in h.levels[:-1])
    for lvl, lv in enumerate(h.levels[:-1]):
        cc = lv.match.coarse_coords
        uc = _rbm_coarse(cc, d, r, 6)
        fine = lv.aux.coords
        target = uf if lvl == 0 else _rbm_coarse(fine, d, r, 6)
        Pt = tentative_prolongation(lv.n, 6, lv.bs, fine, lv.agg_of, cc).to_scipy()
        assert np.abs(Pt @ uc - target).max() < 1e-13
        assert np.abs(lv.P.to_scipy() @ uc - target).max() < 1e-12
    # composite prolongation from the coarsest level
    u = _rbm_coarse(h.levels[-1].aux.coords, d, r, 6)
    for lv in reversed(h.levels[:-1]):
        u = lv.P.to_scipy() @ u
    assert np.abs(u - uf).max() < 1e-11


@pytest.mark.parametrize("omega", [0.3, 2.0 / 3.0, 1.7])
def test_smoothed_rows_preserve_modes_away_from_D(clamped, omega):
    p, h = clamped
    lv = h.levels[0]
    cc = lv.match.coarse_coords
    Ps, types = smoothed_prolongation(lv.A, lv.aux, lv.agg_of, lv.match.dmask, cc, 8, 4, omega)
    rng = np.random.default_rng(2)
    d, r = rng.standard_normal(3), rng.standard_normal(3)
    uc = _rbm_coarse(cc, d, r, 6)
    uf = np.concatenate([d + np.cross(x, r) for x in p.coords]).reshape(-1, 3)
    out = (Ps.to_scipy() @ uc).reshape(-1, 3)
    dm = lv.match.dmask
    A = lv.A
    for i in range(lv.n):
        if dm[i]:
            continue
        stencil = A.col[A.row_ptr[i]:A.row_ptr[i + 1]]
        if dm[stencil].any():
            continue
        assert np.abs(out[i] - uf[i]).max() < 1e-12


def test_coarse_operators_symmetric_with_modes_in_kernel(neumann):
    p, h = neumann
    rng = np.random.default_rng(3)
    for lv in h.levels[1:]:
        A = lv.A.to_scipy()
        assert abs(A - A.T).max() <= 1e-13 * abs(A).max()
        u = _rbm_coarse(lv.aux.coords, rng.standard_normal(3), rng.standard_normal(3), 6)
        assert np.abs(A @ u).max() < 1e-11 * abs(A).max() * np.abs(u).max()


def test_finest_edge_rows_equal_reduced_3x3_form():
    p = make_problem(6, seed=4)
    lv = _setup(p).levels[0]
    cc = lv.match.coarse_coords
    omega = 2.0 / 3.0
    Ps, types = smoothed_prolongation(lv.A, lv.aux, lv.agg_of, lv.match.dmask, cc, 0, 4, omega)
    assert (types == ROW_A).sum() == (~lv.match.dmask).sum()
    x = lv.aux.coords
    from oracle.prolong import filtered_neighbors
    for i in np.nonzero(types == ROW_A)[0][::7]:
        F, cols = filtered_neighbors(lv.aux, i, lv.agg_of, lv.match.dmask, 4)
        def Pf(v):   # [I, Skew(x_v - x_J)] with Skew(t) r = t x r
            t = x[v] - cc[lv.agg_of[v]]
            return np.hstack([np.eye(3), np.stack([np.cross(t, e) for e in np.eye(3)], axis=1)])

        Dr = np.zeros((3, 3))
        acc = {J: np.zeros((3, 6)) for J in cols}
        for l, e in F:
            t = (x[l] - x[i]) / np.linalg.norm(x[l] - x[i])
            c = np.trace(lv.aux.E[e])
            Dr += c * np.outer(t, t)
            acc[lv.agg_of[l]] -= c * np.outer(t, t) @ Pf(l)
        acc[lv.agg_of[i]] += Dr @ Pf(i)
        Dp = pinv_tau(Dr)
        for J in cols:
            expect = -omega * Dp @ acc[J] + (Pf(i) if J == lv.agg_of[i] else 0)
            assert np.abs(Ps.block(i, J) - expect).max() < 1e-12


def test_successive_matching_invariants(clamped):
    p, h = clamped
    sigma = h.params.sigma
    for lv in h.levels[:-1]:
        m = lv.match
        seen = np.zeros(lv.n, dtype=int)
        for a in m.aggs:
            seen[a] += 1
            assert 1 <= len(a) <= 2 ** h.params.rounds
        assert np.all(seen[~m.dmask] == 1) and np.all(seen[m.dmask] == 0)
        Dh = dhat_all(lv.aux)
        for a in m.aggs:
            # connected in the aux graph
            comp, stack = {int(a[0])}, [int(a[0])]
            while stack:
                v = stack.pop()
                for u in lv.aux.neighbors(v)[0]:
                    if int(u) in set(a.tolist()) and int(u) not in comp:
                        comp.add(int(u))
                        stack.append(int(u))
            assert len(comp) == len(a)
            if len(a) > 2:
                assert mu_g(lv.aux, a, Dh) < sigma
        mtr = trace_strength(lv.aux)
        for pair in m.pass_lists[0]:
            if len(pair) == 2:
                i, j = pair
                assert mu_s(lv.aux, i, j, mtr) < sigma and mu_b(lv.aux, i, j, Dh) < sigma


def test_multicolor_gs_is_block_triangular_solve(clamped):
    p, h = clamped
    for lvl in (0,):
        lv = h.levels[lvl]
        o = _ops(h)[lvl]
        rng = np.random.default_rng(5)
        b = rng.standard_normal(lv.n * lv.bs)
        x = gs_sweep(o, b, np.zeros_like(b), range(len(o.rows)))
        perm = np.argsort(lv.colors, kind="stable")
        dofs = (perm[:, None] * lv.bs + np.arange(lv.bs)).ravel()
        A = lv.A.to_scipy().toarray()[np.ix_(dofs, dofs)]
        col = np.repeat(lv.colors[perm], lv.bs)
        Lw = np.where(col[:, None] > col[None, :], A, 0.0)
        for a in range(lv.n):
            s = slice(a * lv.bs, (a + 1) * lv.bs)
            Lw[s, s] = A[s, s]
        y = np.linalg.solve(Lw, b[dofs])   # (D + L) y = b in colour-permuted order
        assert np.allclose(x[dofs], y, rtol=1e-11, atol=1e-12 * np.abs(y).max())


def test_coarsest_regularization_keeps_coarse_correction():
    # section "sing2": (E Atilde E^T + I - E E^T)^{-1} restricted by the prolongation equals the
    # restricted inverse; with the tentative 3x6 finest prolongation of collinear pairs.
    p = make_problem(6, seed=1)
    lv = _setup(p).levels[0]
    cc = lv.match.coarse_coords
    fd = np.nonzero(np.repeat(~lv.match.dmask, 3))[0]
    A = lv.A.to_scipy().toarray()[np.ix_(fd, fd)]
    P = tentative_prolongation(lv.n, 6, 3, lv.aux.coords, lv.agg_of, cc).to_scipy().toarray()[fd]
    Ac = P.T @ A @ P
    reg = Ac.copy()
    for I in range(Ac.shape[0] // 6):
        s = slice(6 * I, 6 * I + 6)
        U0 = kernel_basis(Ac[s, s])
        reg[s, s] += U0 @ U0.T
    C1 = P @ np.linalg.solve(reg, P.T)
    C2 = P @ np.linalg.pinv(Ac, rcond=1e-10, hermitian=True) @ P.T
    assert np.abs(C1 - C2).max() < 1e-8 * np.abs(C2).max()
    assert np.linalg.eigvalsh(reg).min() > 0


def test_coarsest_cholesky_is_lapack(clamped):
    p, h = clamped
    L = h.coarse_chol
    assert np.allclose(L @ L.T, h.coarse_dense, atol=1e-12 * np.abs(h.coarse_dense).max())
    assert np.allclose(L, np.linalg.cholesky(h.coarse_dense))


def test_vcycle_is_symmetric_positive(clamped):
    p, h = clamped
    rng = np.random.default_rng(6)
    r1, r2 = rng.standard_normal((2, p.n_dofs))
    m = np.repeat(p.dirichlet.astype(bool), 3)
    r1[m] = r2[m] = 0
    a, b = vcycle(h, r1) @ r2, r1 @ vcycle(h, r2)
    assert abs(a - b) < 1e-10 * abs(a)
    assert vcycle(h, r1) @ r1 > 0


def test_pcg_matches_direct_solve(clamped):
    p, h = clamped
    x, it, rel, rel_true, conv = pcg(h, p.b, rtol=1e-13)
    A = h.levels[0].A.to_scipy()
    xd = spla.spsolve(A.tocsc(), p.b)
    assert conv and np.linalg.norm(x - xd) <= 1e-9 * np.linalg.norm(xd)
    assert rel_true < 1e-12


def test_unpreconditioned_cg_is_krylov_minimizer():
    p = make_problem(6, seed=8)
    h = _setup(p)
    A = h.levels[0].A.to_scipy().toarray()
    b = p.b
    xs = np.linalg.solve(A, b)
    for k in (1, 3, 6):
        x, it, *_ = pcg(h, b, rtol=0.0, max_it=k, precond=False)
        assert it == k
        K = np.empty((b.size, k))
        v = b / np.linalg.norm(b)
        for j in range(k):       # Krylov basis with full re-orthogonalization
            K[:, j] = v
            v = A @ v
            v -= K[:, :j + 1] @ (K[:, :j + 1].T @ v)
            v /= np.linalg.norm(v)
        y = np.linalg.solve(K.T @ A @ K, K.T @ b)
        xk = K @ y
        assert np.sqrt((x - xs) @ A @ (x - xs)) <= np.sqrt((xk - xs) @ A @ (xk - xs)) * (1 + 1e-8)
        assert np.linalg.norm(x - xk) <= 1e-8 * np.linalg.norm(xk)
