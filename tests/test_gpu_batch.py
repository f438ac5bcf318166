"""GPU parity of the batched block-panel solve (eamg_solve_batch) against the FP64 CPU oracle.

Each column of a batch runs its own PCG recurrence with the same V-cycle as the single-vector
solve, so every column must match the oracle's single-vector PCG on that right-hand side:

* at the oracle's iteration count, each column's iterate within X_TOL = 1e-10 relative (the
  FP64 parity bar; the panel kernels sum in a different order than the single-vector ones);
* run to rtol = 1e-8, each column reaches ||b - A x|| <= 1e-8 ||b|| (checked on the CPU with
  the assembled matrix) within one iteration of the oracle's count;
* ragged batches (padding to the panel width), more than one panel, a zero column, a
  non-finite column, the iteration limit, an initial guess and a strided leading dimension;
* the FP32 V-cycle inside the FP64 CG per column (true residual 1e-8, iterations at most
  three above the FP64 V-cycle's);
* full size (64^3 vertices, 32 right-hand sides): every column converges, and sampled columns'
  true residuals are checked on the CPU.
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


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _bound_matrix(p):
    A = sp.bsr_matrix((p.vals, p.col_idx, p.row_ptr), shape=(p.n_dofs,) * 2).tocsr()
    dm = np.repeat(p.dirichlet.astype(bool), p.dim)
    Dm = sp.diags((~dm).astype(float))
    return Dm @ A @ Dm + sp.diags(dm.astype(float))


def _rhs(p, m, seed):
    """m seeded load cases: uniform[-1, 1] like the problem's own right-hand side."""
    rng = np.random.default_rng([seed, m])
    B = rng.uniform(-1.0, 1.0, size=(m, p.n_dofs))
    B[:, np.repeat(p.dirichlet.astype(bool), p.dim)] = 0.0
    return B


CASES = {
    "cube13": dict(n=13, seed=7),
    "box_ragged": dict(n=11, ny=7, nz=5, h=0.1, nu=0.35, seed=4),
    "poisson10": dict(n=10, kind="poisson", clamp="all", seed=2),
}


@pytest.fixture(scope="module", params=list(CASES))
def case(request):
    name = request.param
    p = make_problem(**CASES[name])
    print(f"\n[batch case {name}] dofs={p.n_dofs}", flush=True)
    ho = oracle.setup(p.dim, p.coords, p.row_ptr, p.col_idx, p.vals, p.dirichlet)
    hl = E.Hierarchy(p.dim, p.coords, p.row_ptr, p.col_idx, p.vals, p.dirichlet,
                     E.eamg_default_setup_params(vcycle_fp32=1))
    yield name, p, ho, hl
    hl.close()


def test_batch_columns_match_oracle(case):
    name, p, ho, hl = case
    m = 5                                    # panel width 8: three padded columns
    B = _rhs(p, m, 11)
    Bd = torch.tensor(B, device="cuda")
    ref = [oracle.pcg(ho, B[c], rtol=1e-8) for c in range(m)]
    its = max(r[1] for r in ref)
    # fixed iteration count: every column runs exactly `its` iterations
    Xk, st, infk = hl.solve_batch(Bd, rtol=0.0, max_it=its)
    assert st == E.EAMG_NOT_CONVERGED and all(i["iterations"] == its for i in infk)
    worst = 0.0
    for c in range(m):
        xo, _, _, _, _ = oracle.pcg(ho, B[c], rtol=0.0, max_it=its)
        worst = max(worst, np.linalg.norm(Xk[c].cpu().numpy() - xo) / np.linalg.norm(xo))
    # to tolerance: each column stops on its own
    X, st, inf = hl.solve_batch(Bd, rtol=1e-8)
    assert st == E.EAMG_OK
    Ab = _bound_matrix(p)
    Xh = X.cpu().numpy()
    for c in range(m):
        assert inf[c]["status"] == E.EAMG_OK
        assert abs(inf[c]["iterations"] - ref[c][1]) <= 1
        res = np.linalg.norm(B[c] - Ab @ Xh[c]) / np.linalg.norm(B[c])
        assert res <= 1e-8 and abs(res - inf[c]["rel_res_true"]) <= 1e-3 * res + 1e-15
    print(f"[{name}] its oracle={[r[1] for r in ref]} batch={[i['iterations'] for i in inf]} "
          f"max x rel err at {its} its={worst:.2e}", flush=True)
    assert worst <= X_TOL
    # run-to-run reproducible
    X2, _, _ = hl.solve_batch(Bd, rtol=1e-8)
    assert torch.equal(X, X2)


def test_batch_fp32_vcycle(case):
    name, p, ho, hl = case
    m = 6
    B = _rhs(p, m, 12)
    Bd = torch.tensor(B, device="cuda")
    X64, st64, i64 = hl.solve_batch(Bd, rtol=1e-8)
    X32, st32, i32 = hl.solve_batch(Bd, rtol=1e-8, precond=E.EAMG_PRECOND_VCYCLE_FP32)
    assert st64 == E.EAMG_OK and st32 == E.EAMG_OK
    Ab = _bound_matrix(p)
    X32h = X32.cpu().numpy()
    for c in range(m):
        res = np.linalg.norm(B[c] - Ab @ X32h[c]) / np.linalg.norm(B[c])
        assert res <= 1e-8
        assert i32[c]["iterations"] <= i64[c]["iterations"] + 3
    err = max(np.linalg.norm(X32h[c] - X64[c].cpu().numpy()) / np.linalg.norm(X64[c].cpu().numpy())
              for c in range(m))
    print(f"[{name}] fp32 its={[i['iterations'] for i in i32]} fp64 its="
          f"{[i['iterations'] for i in i64]} max |x32 - x64| / |x64| = {err:.2e}", flush=True)


def test_batch_matches_single_solve(case):
    name, p, ho, hl = case
    B = _rhs(p, 1, 13)
    Bd = torch.tensor(B, device="cuda")
    X, st, inf = hl.solve_batch(Bd, rtol=1e-8)
    x1, info1 = hl.solve(Bd[0].contiguous(), rtol=1e-8)
    assert st == E.EAMG_OK and inf[0]["iterations"] == info1["iterations"]
    err = float((X[0] - x1).norm() / x1.norm())
    assert err <= X_TOL, err


def test_batch_edge_columns():
    p = make_problem(9, seed=5)
    hl = E.Hierarchy(p.dim, p.coords, p.row_ptr, p.col_idx, p.vals, p.dirichlet)
    B = _rhs(p, 4, 21)
    B[1] = 0.0
    Bd = torch.tensor(B, device="cuda")
    free = np.nonzero(~np.repeat(p.dirichlet.astype(bool), p.dim))[0]
    Bd[2, int(free[3])] = float("nan")
    X, st, inf = hl.solve_batch(Bd, rtol=1e-8)
    assert st == E.EAMG_NOT_CONVERGED
    assert [i["status"] for i in inf] == [E.EAMG_OK, E.EAMG_OK, E.EAMG_ERR_BREAKDOWN, E.EAMG_OK]
    assert inf[1]["iterations"] == 0 and float(X[1].abs().max()) == 0.0
    assert float(X[2].abs().max()) == 0.0
    # the healthy columns equal their single-vector solves
    for c in (0, 3):
        xs, info = hl.solve(Bd[c].contiguous(), rtol=1e-8)
        assert inf[c]["iterations"] == info["iterations"]
        assert float((X[c] - xs).norm() / xs.norm()) <= X_TOL
    # iteration limit
    _, st, inf = hl.solve_batch(Bd[[0, 3]].contiguous(), rtol=1e-12, max_it=2)
    assert st == E.EAMG_NOT_CONVERGED
    assert all(i["status"] == E.EAMG_NOT_CONVERGED and i["iterations"] == 2 for i in inf)
    # initial guess: converged solutions as x0 finish at once
    B0 = Bd[[0, 3]].contiguous()
    X0, _, _ = hl.solve_batch(B0, rtol=1e-8)
    X1, st, inf = hl.solve_batch(B0, X0.clone(), rtol=1e-6, use_x0=True)
    assert st == E.EAMG_OK and all(i["iterations"] <= 1 for i in inf)
    # strided leading dimension: a view into a wider buffer
    wide = torch.zeros(2, p.n_dofs + 40, dtype=torch.float64, device="cuda")
    wide[:, :p.n_dofs] = B0
    Xw = torch.full_like(wide, 7.0)
    st, inf = E.eamg_solve_batch(hl.h, wide[:, :p.n_dofs], Xw[:, :p.n_dofs], rtol=1e-8)
    assert st == E.EAMG_OK
    assert torch.equal(Xw[:, :p.n_dofs], X0) and float((Xw[:, p.n_dofs:] - 7.0).abs().max()) == 0.0
    hl.close()


def test_batch_many_panels():
    """70 right-hand sides: one 64-wide panel and one 8-wide panel (6 live columns)."""
    p = make_problem(7, seed=8)
    hl = E.Hierarchy(p.dim, p.coords, p.row_ptr, p.col_idx, p.vals, p.dirichlet)
    B = _rhs(p, 70, 22)
    Bd = torch.tensor(B, device="cuda")
    X, st, inf = hl.solve_batch(Bd, rtol=1e-8)
    assert st == E.EAMG_OK
    Ab = _bound_matrix(p)
    Xh = X.cpu().numpy()
    for c in (0, 31, 63, 64, 69):
        xs, info = hl.solve(Bd[c].contiguous(), rtol=1e-8)
        assert inf[c]["iterations"] == info["iterations"]
        assert float((X[c] - xs).norm() / xs.norm()) <= X_TOL
    res = np.linalg.norm(B - (Ab @ Xh.T).T, axis=1) / np.linalg.norm(B, axis=1)
    assert res.max() <= 1e-8
    hl.close()


def test_batch_rejects_bad_arguments():
    p = make_problem(6)
    hl = E.Hierarchy(p.dim, p.coords, p.row_ptr, p.col_idx, p.vals, p.dirichlet)
    Bd = torch.tensor(_rhs(p, 2, 1), device="cuda")
    with pytest.raises(E.EamgError) as ei:
        hl.solve_batch(Bd, precond=E.EAMG_PRECOND_VCYCLE_FP32)
    assert ei.value.status == E.EAMG_ERR_INVALID_ARG
    with pytest.raises(E.EamgError) as ei:
        E.eamg_solve_batch(hl.h, Bd, Bd)
    assert ei.value.status == E.EAMG_ERR_INVALID_ARG
    hl.close()


def test_batch_full_size_cube64_32rhs():
    p = make_problem(64, seed=1)
    print(f"\n[cube64 x 32] dofs={p.n_dofs}", flush=True)
    # the bench's 64^3 configuration (caps 6 / 4 / 4, sigma 18, dense V-cycle tail)
    hl = E.Hierarchy(p.dim, p.coords, p.row_ptr, p.col_idx, p.vals, p.dirichlet,
                     E.eamg_default_setup_params(vcycle_fp32=1, coarsest_max_dofs=500,
                                                 dense_tail_dofs=16384, cap_std_l0=6, cap_std=4,
                                                 cap_aux=4, sigma=18.0))
    E.eamg_autotune(hl.h, panel_width=32)
    B = _rhs(p, 32, 4)
    Bd = torch.tensor(B, device="cuda")
    Ab = _bound_matrix(p)
    for prec in (E.EAMG_PRECOND_VCYCLE, E.EAMG_PRECOND_VCYCLE_FP32):
        X, st, inf = hl.solve_batch(Bd, rtol=1e-8, precond=prec)
        print(f"[cube64 x 32] precond={prec} its={sorted(set(i['iterations'] for i in inf))} "
              f"ms={inf[0]['ms']:.1f}", flush=True)
        assert st == E.EAMG_OK
        for c in (0, 17, 31):
            xh = X[c].cpu().numpy()
            assert np.linalg.norm(B[c] - Ab @ xh) <= 1e-8 * np.linalg.norm(B[c])
    hl.close()
