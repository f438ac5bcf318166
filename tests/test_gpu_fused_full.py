"""The multi-mesh workload at full size, in the bench's configuration: 16 cubes with sides
uniform in [8, 48] and Poisson ratios uniform in [0.2, 0.45] (2.25 M free dofs), each with its
own hierarchy (caps 6 / 4 / 3, sigma 20, coarsening to < 500 dofs, dense tail <= 16384 dofs),
fused into one block-diagonal hierarchy with V-cycles ending at 4096-dof tails it builds,
autotuned, solved with the FP32 V-cycle in FP64 CG (section "res" per system).

This checks what holds at any size for the FP32 V-cycle the bench times: every system reaches a
true relative residual of 1e-8 recomputed on the host, with the iteration count of its own
single-system solve (within one) and the same solution up to the solver's accuracy.  The same
workload with the FP64 V-cycle is compared with the oracle's hierarchies and solves in
test_gpu_multi16_oracle.py."""
import numpy as np
import pytest
import scipy.sparse as sp

import paper_2011_13325_amd as E
from gen import make_problem

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

PRM = dict(vcycle_fp32=1, coarsest_max_dofs=500, dense_tail_dofs=16384, cap_std_l0=6, cap_std=4,
           cap_aux=3, sigma=20.0)


def _true_res(p, x):
    A = sp.bsr_matrix((p.vals.reshape(-1, 3, 3), p.col_idx, p.row_ptr), shape=(p.n_dofs,) * 2)
    dm = np.repeat(p.dirichlet.astype(bool), 3)
    xf = np.where(dm, 0.0, x)
    r = p.b - np.where(dm, 0.0, A @ xf) - np.where(dm, x, 0.0)
    return np.linalg.norm(r) / np.linalg.norm(p.b)


def test_sixteen_cubes_fused_at_full_size():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    rng = np.random.default_rng(4)
    sides = rng.integers(8, 49, size=16)
    nus = rng.uniform(0.2, 0.45, size=16)
    sysm = []
    f = None
    try:
        for c, (n, nu) in enumerate(zip(sides, nus)):
            p = make_problem(int(n), nu=float(nu), seed=100 + c)
            sysm.append((p, E.Hierarchy(p.dim, p.coords, p.row_ptr, p.col_idx, p.vals, p.dirichlet,
                                        E.eamg_default_setup_params(**PRM))))
        print(f"\n[16 cubes] sides {sides.tolist()} free dofs {sum(p.n_free_dofs for p, _ in sysm)}",
              flush=True)
        f = E.Fused([h for _, h in sysm], dense_tail_dofs=4096)
        E.eamg_autotune(f.h, 0)
        bs = [torch.tensor(p.b, device="cuda") for p, _ in sysm]
        xs, st, infos = f.solve(bs, rtol=1e-8, precond=E.EAMG_PRECOND_VCYCLE_FP32)
        assert st == E.EAMG_OK
        worst_r, worst_d = 0.0, 0.0
        for m, ((p, h), b, x, inf) in enumerate(zip(sysm, bs, xs, infos)):
            xo, io = h.solve(b, rtol=1e-8, precond=E.EAMG_PRECOND_VCYCLE_FP32)
            r = _true_res(p, x.cpu().numpy())
            d = float((x - xo).norm() / xo.norm())
            worst_r, worst_d = max(worst_r, r), max(worst_d, d)
            assert inf["status"] == E.EAMG_OK and r <= 1e-8, (m, r, inf)
            assert abs(inf["iterations"] - io["iterations"]) <= 1, (m, inf, io)
            assert d <= 1e-5, (m, d)
        print(f"[16 cubes] iterations {[i['iterations'] for i in infos]}, worst true residual "
              f"{worst_r:.2e}, worst distance to the own solves {worst_d:.1e}", flush=True)
    finally:
        if f is not None:
            f.close()
        for _, h in sysm:
            h.close()
