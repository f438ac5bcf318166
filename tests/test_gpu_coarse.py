"""GPU parity of the coarsest-level direct solve for coarsest levels of thousands of dofs.

The regularized coarsest matrix (section on singular coarse levels) is inverted on the device by
blocked Gauss-Jordan elimination and applied as a dense product; the oracle solves with its own
Cholesky factor.  Checked here:

* one level (the whole problem is the coarsest): the V-cycle is A^{-1} r, compared with a dense
  LAPACK solve of the assembled matrix, for a ragged size (3993 dofs, leading dimension 4096);
  PCG then converges in one iteration; the FP32 V-cycle (FP64 inverse, FP32 vectors) within
  FP32 round-off;
* two levels with a 7000-dof coarsest: hierarchy, V-cycle and the PCG iterate at the oracle's
  iteration count within 1e-10 relative of the oracle run with the same parameters;
* the panel product for 5 and 40 right-hand sides (panel widths 8 and 64) against the dense
  solve per column (FP64 1e-10; FP32 vectors: true residual 1e-9, error 1e-6);
* the Gauss-Jordan inverse against a Cholesky solve (the oracle's factorization) on a
  nu = 0.45 level of 6591 dofs, within the FP64 bar (the measured error and cond(A) printed);
* the limit on coarsest_max_dofs, and an indefinite matrix reported as not SPD.
"""
import numpy as np
import pytest
import scipy.sparse as sp

import oracle
import paper_2011_13325_amd as E
from gen import make_problem

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

X_TOL = 1e-10
BIG = 8192


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _dev(a):
    return torch.tensor(np.asarray(a, dtype=np.float64), device="cuda")


def _bound_dense(p):
    A = sp.bsr_matrix((p.vals, p.col_idx, p.row_ptr), shape=(p.n_dofs,) * 2).tocsr()
    dm = np.repeat(p.dirichlet.astype(bool), p.dim)
    Dm = sp.diags((~dm).astype(float))
    return (Dm @ A @ Dm + sp.diags(dm.astype(float))).toarray(), dm


def _lib(p, **prm):
    return E.Hierarchy(p.dim, p.coords, p.row_ptr, p.col_idx, p.vals, p.dirichlet,
                       E.eamg_default_setup_params(**prm))


def test_single_level_dense_inverse():
    p = make_problem(11, seed=6)                   # 3993 dofs: one level, ld 4096
    hl = _lib(p, coarsest_max_dofs=BIG, vcycle_fp32=1)
    assert hl.stats()["n_levels"] == 1
    Ad, dm = _bound_dense(p)
    r = np.random.default_rng(1).standard_normal(p.n_dofs)
    r[dm] = 0.0
    zs = np.linalg.solve(Ad, r)
    z = torch.empty(p.n_dofs, dtype=torch.float64, device="cuda")
    E.eamg_vcycle(hl.h, _dev(r), z)
    torch.cuda.synchronize()
    err = np.linalg.norm(z.cpu().numpy() - zs) / np.linalg.norm(zs)
    z32 = torch.empty_like(z)
    E.eamg_vcycle(hl.h, _dev(r), z32, precision=E.EAMG_PRECOND_VCYCLE_FP32)
    torch.cuda.synchronize()
    err32 = np.linalg.norm(z32.cpu().numpy() - zs) / np.linalg.norm(zs)
    print(f"\n[dense 3993] V-cycle rel err FP64 {err:.2e} FP32 vectors {err32:.2e}", flush=True)
    assert err <= X_TOL
    assert err32 <= 1e-5
    x, info = hl.solve(_dev(p.b), rtol=1e-8)
    assert info["status"] == E.EAMG_OK and info["iterations"] <= 2
    xs = np.linalg.solve(Ad, p.b)
    assert np.linalg.norm(x.cpu().numpy() - xs) <= 1e-10 * np.linalg.norm(xs)
    hl.close()


def test_gauss_jordan_inverse_against_cholesky_nu045():
    # the oracle factors the coarsest matrix by Cholesky, the library inverts it by Gauss-Jordan
    # elimination without pivoting (on an SPD matrix both are backward stable; the applied
    # inverse's forward error is bounded by a small multiple of cond(A) * eps): one level of
    # 6591 dofs at nu = 0.45 (ld 6656), the apply against a LAPACK Cholesky solve
    import scipy.linalg as sl
    p = make_problem(13, nu=0.45, seed=7)
    hl = _lib(p, coarsest_max_dofs=16384)
    assert hl.stats()["n_levels"] == 1
    Ad, dm = _bound_dense(p)
    cond = np.linalg.cond(Ad)
    r = np.random.default_rng(2).standard_normal(p.n_dofs)
    r[dm] = 0.0
    zc = sl.cho_solve(sl.cho_factor(Ad), r)
    z = torch.empty(p.n_dofs, dtype=torch.float64, device="cuda")
    E.eamg_vcycle(hl.h, _dev(r), z)
    torch.cuda.synchronize()
    err = np.linalg.norm(z.cpu().numpy() - zc) / np.linalg.norm(zc)
    print(f"\n[GJ vs Cholesky, 6591 dofs, nu=0.45] cond {cond:.2e} rel err {err:.2e} "
          f"(cond * eps = {cond * 2.2e-16:.2e})", flush=True)
    assert err <= max(X_TOL, 100 * cond * 2.2e-16)
    hl.close()


def test_two_levels_large_coarsest_match_oracle():
    p = make_problem(17)
    ho = oracle.setup(p.dim, p.coords, p.row_ptr, p.col_idx, p.vals, p.dirichlet,
                      oracle.SetupParams(coarsest_max_dofs=BIG))
    hl = _lib(p, coarsest_max_dofs=BIG)
    st = hl.stats()
    print(f"\n[cube17 coarsest<{BIG}] levels={st['n_levels']} n={st['n']}", flush=True)
    assert st["n_levels"] == ho.n_levels == 2
    assert 6 * st["n"][-1] > 4000                      # beyond the former host-side limit
    r = np.random.default_rng(3).standard_normal(p.n_dofs)
    r[np.repeat(p.dirichlet.astype(bool), p.dim)] = 0.0
    zo = oracle.vcycle(ho, r)
    z = torch.empty(p.n_dofs, dtype=torch.float64, device="cuda")
    E.eamg_vcycle(hl.h, _dev(r), z)
    torch.cuda.synchronize()
    verr = np.linalg.norm(z.cpu().numpy() - zo) / np.linalg.norm(zo)
    xo, it, _, _, conv = oracle.pcg(ho, p.b, rtol=1e-8)
    assert conv
    xk, infok = hl.solve(_dev(p.b), rtol=0.0, max_it=it)
    xerr = np.linalg.norm(xk.cpu().numpy() - xo) / np.linalg.norm(xo)
    _, info = hl.solve(_dev(p.b), rtol=1e-8)
    print(f"[cube17 coarsest<{BIG}] V-cycle rel err {verr:.2e}; its oracle={it} "
          f"lib={info['iterations']}; x rel err at k*={xerr:.2e}", flush=True)
    assert verr <= X_TOL and xerr <= X_TOL
    assert info["status"] == E.EAMG_OK and abs(info["iterations"] - it) <= 1
    hl.close()


@pytest.mark.parametrize("m", [5, 40])
def test_dense_panel_product(m):
    p = make_problem(9, seed=8)                    # 2187 dofs: one level, ld 2304
    hl = _lib(p, coarsest_max_dofs=BIG, vcycle_fp32=1)
    assert hl.stats()["n_levels"] == 1
    Ad, dm = _bound_dense(p)
    B = np.random.default_rng([9, m]).uniform(-1.0, 1.0, size=(m, p.n_dofs))
    B[:, dm] = 0.0
    Xs = np.linalg.solve(Ad, B.T).T
    # FP64: one iteration with the exact inverse; FP32 vectors: about 1e-7 per iteration
    for prec, tol in ((E.EAMG_PRECOND_VCYCLE, 1e-10), (E.EAMG_PRECOND_VCYCLE_FP32, 1e-6)):
        X, st, inf = hl.solve_batch(_dev(B), rtol=1e-9, precond=prec)
        assert st == E.EAMG_OK and all(i["iterations"] <= 3 for i in inf)
        assert all(i["rel_res_true"] <= 1e-9 for i in inf)
        err = max(np.linalg.norm(X[c].cpu().numpy() - Xs[c]) / np.linalg.norm(Xs[c])
                  for c in range(m))
        print(f"\n[dense panel m={m} precond={prec}] max col rel err {err:.2e}", flush=True)
        assert err <= tol
    hl.close()


def test_coarsest_limit_and_not_spd():
    p = make_problem(4)
    with pytest.raises(E.EamgError) as ei:
        _lib(p, coarsest_max_dofs=16385)
    assert ei.value.status == E.EAMG_ERR_INVALID_ARG
    hl = _lib(p, coarsest_max_dofs=16384)
    hl.close()
    # an indefinite matrix whose coarsest level is the finest one (the dense path)
    vals = p.vals.copy()
    rows = np.repeat(np.arange(p.n_vertices), np.diff(p.row_ptr))
    diag = np.nonzero((rows == p.col_idx) & (p.dirichlet[rows] == 0))[0]
    vals[diag[5]] *= -3.0
    with pytest.raises(E.EamgError) as ei:
        E.Hierarchy(3, p.coords, p.row_ptr, p.col_idx, vals, p.dirichlet,
                    E.eamg_default_setup_params(coarsest_max_dofs=BIG))
    assert ei.value.status == E.EAMG_ERR_NOT_SPD
