"""Full-size properties of the 128^3 elasticity workload (6,291,456 dofs, nu = 0.45, RHS seed 3):
the FP32 V-cycle inside FP64 CG, with the bench's headline settings (coarsening to < 500 dofs,
dense V-cycle tail <= 16384 dofs, P_s row caps 6 / 4 / 4, sigma 18).

The oracle cannot set up a problem of this size, so this checks what holds at any size, on the
library's own hierarchy:

* both preconditioners (FP64 V-cycle, FP32 V-cycle) reach a true relative residual of 1e-8, the
  residual recomputed here on the host from the input matrix (scipy BSR product, FP64);
* level 0: the agglomerates partition the free vertices into groups of at most four (two
  matching passes), Dirichlet vertices are dropped;
* P_s reproduces the rigid body modes exactly (1e-10) on rows whose stencil avoids the clamped
  face (Thm thm:deng_elast: the kernel vectors are in the range of the prolongation);
* A_1 equals P_s^T A_0 P_s on sampled columns (1e-11), and its sampled rows equal its columns
  (symmetry, 1e-12).
"""
import time

import numpy as np
import pytest
import scipy.sparse as sp

import paper_2011_13325_amd as E
from gen import make_problem

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

N = 128
HEADLINE = dict(vcycle_fp32=1, coarsest_max_dofs=500, dense_tail_dofs=16384, cap_std_l0=6,
                cap_std=4, cap_aux=4, sigma=18.0)


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


@pytest.fixture(scope="module")
def big():
    t0 = time.perf_counter()
    p = make_problem(N, nu=0.45, seed=3)
    print(f"\n[cube128] dofs={p.n_dofs} nnzb={p.col_idx.size} generated in "
          f"{time.perf_counter() - t0:.1f} s", flush=True)
    t0 = time.perf_counter()
    h = E.Hierarchy(p.dim, p.coords, p.row_ptr, p.col_idx, p.vals, p.dirichlet,
                    E.eamg_default_setup_params(**HEADLINE))
    st = h.stats()
    print(f"[cube128] setup {time.perf_counter() - t0:.1f} s levels={st['n_levels']} n={st['n']} "
          f"vc={st['vc']:.3f} oc={st['oc']:.3f}", flush=True)
    yield p, h
    h.close()


def _true_rel_residual(p, x):
    A = sp.bsr_matrix((p.vals.reshape(-1, 3, 3), p.col_idx, p.row_ptr), shape=(p.n_dofs,) * 2)
    dm = np.repeat(p.dirichlet.astype(bool), 3)
    xf = np.where(dm, 0.0, x)
    r = p.b - np.where(dm, 0.0, A @ xf) - np.where(dm, x, 0.0)
    return np.linalg.norm(r) / np.linalg.norm(p.b)


def test_full_size_cube128_solves(big):
    p, h = big
    b = torch.tensor(p.b, dtype=torch.float64, device="cuda")
    xs = {}
    for name, prec in (("fp64", E.EAMG_PRECOND_VCYCLE), ("fp32", E.EAMG_PRECOND_VCYCLE_FP32)):
        x, info = h.solve(b, rtol=1e-8, precond=prec)
        xh = x.cpu().numpy()
        rel = _true_rel_residual(p, xh)
        print(f"[cube128 {name} V-cycle] its={info['iterations']} ms={info['ms']:.1f} "
              f"rel_res_true(lib)={info['rel_res_true']:.2e} host={rel:.2e}", flush=True)
        assert info["status"] == E.EAMG_OK
        assert rel <= 1e-8 and info["rel_res_true"] <= 1e-8
        xs[name] = xh
    d = np.linalg.norm(xs["fp32"] - xs["fp64"]) / np.linalg.norm(xs["fp64"])
    print(f"[cube128] |x_fp32vc - x_fp64vc| / |x_fp64vc| = {d:.2e}", flush=True)


def test_full_size_cube128_hierarchy(big):
    p, h = big
    ex = h.export(0)
    agg = ex["agg"]
    free = p.dirichlet == 0
    assert np.all(agg[free] >= 0) and np.all(agg[~free] == -1)
    assert np.bincount(agg[free]).max() <= 4
    ex1 = h.export(1)
    nc = ex1["info"]["n"]
    cc = np.zeros((nc, 3))
    np.add.at(cc, agg[free], p.coords[free])
    cc /= np.bincount(agg[free])[:, None]
    rng = np.random.default_rng(0)
    d, r = rng.standard_normal(3), rng.standard_normal(3)
    uc = np.concatenate([d + np.cross(cc, r), np.broadcast_to(r, (nc, 3))], axis=1).ravel()
    Pm = sp.bsr_matrix((ex["P_val"], ex["P_col"], ex["P_rowptr"]), shape=(p.n_dofs, 6 * nc))
    uf = (Pm @ uc).reshape(-1, 3)
    ref = d + np.cross(p.coords, r)
    nearD = np.zeros(p.n_vertices, bool)
    rows = np.repeat(np.arange(p.n_vertices), np.diff(p.row_ptr))
    nearD[rows[p.dirichlet[p.col_idx] == 1]] = True
    ok = ~nearD & free
    err = np.abs(uf[ok] - ref[ok]).max() / np.abs(ref).max()
    A = sp.bsr_matrix((p.vals.reshape(-1, 3, 3), p.col_idx, p.row_ptr), shape=(p.n_dofs,) * 2)
    dm = np.repeat(p.dirichlet.astype(bool), 3)
    A1 = sp.bsr_matrix((ex1["A_val"], ex1["A_col"], ex1["A_rowptr"]), shape=(6 * nc,) * 2)
    worst = 0.0
    for c in rng.choice(6 * nc, 6, replace=False):
        e = np.zeros(6 * nc)
        e[c] = 1.0
        v = Pm @ e
        v[dm] = 0.0
        Av = A @ v
        Av[dm] = 0.0
        ref_col = Pm.T @ Av
        worst = max(worst, np.abs(A1 @ e - ref_col).max() / np.abs(ref_col).max())
    # symmetry on sampled rows: row c read from the block arrays against column c = A_1 e_c
    asym = 0.0
    vals1 = ex1["A_val"]
    for c in rng.choice(6 * nc, 6, replace=False):
        e = np.zeros(6 * nc)
        e[c] = 1.0
        col_c = A1 @ e
        I, ci = divmod(int(c), 6)
        lo, hi = ex1["A_rowptr"][I], ex1["A_rowptr"][I + 1]
        row_c = np.zeros(6 * nc)
        idx = (6 * ex1["A_col"][lo:hi, None] + np.arange(6)).ravel()
        row_c[idx] = vals1[lo:hi, ci, :].ravel()
        asym = max(asym, np.abs(row_c - col_c).max() / np.abs(col_c).max())
    print(f"[cube128] rigid body modes through P_s: {err:.1e}; A_1 vs P^T A P: {worst:.1e}; "
          f"asymmetry {asym:.1e}", flush=True)
    assert err <= 1e-10
    assert worst <= 1e-11
    assert asym <= 1e-12
