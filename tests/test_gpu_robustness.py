"""GPU: the coefficient-jump example (the paper's eleven-box geometry) through the library.

* Scalar-only pairing (mu_s_only = 1) keeps parity with the oracle: agglomerates and patterns
  bit-exact, V-cycle within 1e-10 (12^3 vertices, one cell per box).
* On the 22-cell cube (23^3 vertices, 36,501 dofs, two cells per box) the robust criteria need
  far fewer PCG iterations to 1e-8 than scalar-only pairing (the trend of the paper's figures
  fig:2dc_rob / fig:2dc_norob), both in FP64 and with the FP32 V-cycle.
"""
import numpy as np
import pytest

import oracle
import paper_2011_13325_amd as E
from gen import make_problem

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _lib(p, **prm):
    return E.Hierarchy(p.dim, p.coords, p.row_ptr, p.col_idx, p.vals, p.dirichlet,
                       E.eamg_default_setup_params(**prm))


def test_scalar_only_pairing_matches_oracle():
    p = make_problem(12, boxes=True, seed=14)
    ho = oracle.setup(p.dim, p.coords, p.row_ptr, p.col_idx, p.vals, p.dirichlet,
                      oracle.SetupParams(mu_s_only=True))
    hl = _lib(p, mu_s_only=1)
    assert hl.stats()["n_levels"] == ho.n_levels
    for l, lev in enumerate(ho.levels[:-1]):
        ex = hl.export(l)
        assert np.array_equal(ex["agg"], lev.agg_of)
        assert np.array_equal(ex["A_col"], lev.A.col)
    r = np.random.default_rng(3).standard_normal(p.n_dofs)
    r[np.repeat(p.dirichlet.astype(bool), p.dim)] = 0.0
    zo = oracle.vcycle(ho, r)
    z = torch.empty(p.n_dofs, dtype=torch.float64, device="cuda")
    E.eamg_vcycle(hl.h, torch.tensor(r, device="cuda"), z)
    torch.cuda.synchronize()
    err = np.linalg.norm(z.cpu().numpy() - zo) / np.linalg.norm(zo)
    print(f"\n[eleven boxes 12^3, mu_s only] levels {ho.n_levels}, V-cycle rel err {err:.2e}", flush=True)
    assert err <= 1e-10
    hl.close()


def test_robust_criteria_need_fewer_iterations():
    p = make_problem(23, boxes=True, seed=14)
    b = torch.tensor(p.b, device="cuda")
    its = {}
    for mso in (0, 1):
        h = _lib(p, mu_s_only=mso, vcycle_fp32=1)
        _, i64 = h.solve(b, rtol=1e-8, max_it=400)
        _, i32 = h.solve(b, rtol=1e-8, max_it=400, precond=E.EAMG_PRECOND_VCYCLE_FP32)
        its[mso] = (i64["iterations"], i32["iterations"], i64["status"], h.stats()["n"])
        h.close()
    print(f"\n[eleven boxes 23^3] robust: its {its[0][:2]}, levels {its[0][3]}; "
          f"mu_s only: its {its[1][:2]}, levels {its[1][3]}", flush=True)
    assert its[0][2] == E.EAMG_OK
    assert its[0][0] <= 25
    assert its[1][0] >= 3 * its[0][0]
    assert its[1][1] >= 3 * its[0][1]
