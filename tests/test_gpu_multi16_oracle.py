"""The 16-cube multi-mesh workload at full size against the oracle: each cube's hierarchy and
PCG solve as the oracle computes them (tests/golden/multi16_oracle.txt, written by
tests/golden/make_multi16_oracle.py, which calls only oracle/ and gen/).

The library builds each cube's hierarchy with the workload's settings (P_s row caps 6 / 4 / 3,
sigma 20, two matching passes per level, coarsening to < 500 dofs; its own dense tail of at most
16384 dofs), fuses the 16 into one block-diagonal hierarchy with 4096-dof tails (the bench's
configuration) and solves all of them together with the FP64 V-cycle:

* every cube, every level: vertex count, block size, agglomerates (Algorithm alg:pwagg),
  smoother colours and the patterns of A_l and P_s (Def. def:aux_sp) equal the oracle's bit for
  bit (SHA-256 of each array);
* the fused PCG (section "res" per system) stops every cube at the oracle's iteration count k*
  for relative residual 1e-8, and each iterate equals the oracle's at 32 seeded positions and in
  its 2-norm within 1e-10 relative (the FP64 parity bar).
"""
import hashlib
import os
from collections import defaultdict

import numpy as np
import pytest

from gen import make_problem

GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "multi16_oracle.txt")
PRM = dict(vcycle_fp32=1, coarsest_max_dofs=500, dense_tail_dofs=16384, cap_std_l0=6, cap_std=4,
           cap_aux=3, sigma=20.0)
X_TOL = 1e-10


def _digest(a):
    return hashlib.sha256(np.ascontiguousarray(np.asarray(a, dtype="<i8")).tobytes()).hexdigest()


def _workload():
    rng = np.random.default_rng(4)
    sides = rng.integers(8, 49, size=16)
    nus = rng.uniform(0.2, 0.45, size=16)
    return [(m, int(n), float(nu)) for m, (n, nu) in enumerate(zip(sides, nus))]


def _read():
    g = defaultdict(lambda: {"levels": [], "idx": [], "x": []})
    with open(GOLD) as fh:
        for line in fh:
            f = line.split()
            if not f or f[0].startswith("#"):
                continue
            if f[0] == "system":
                g[int(f[1])]["side"] = int(f[3])
            elif f[0] == "level":
                g[int(f[1])]["levels"].append(dict(n=int(f[3]), bs=int(f[4]), agg=f[5], colors=f[6],
                                                   A_rp=f[7], A_col=f[8], P_rp=f[9], P_col=f[10]))
            elif f[0] == "iterations":
                g[int(f[1])]["its"] = int(f[2])
            elif f[0] == "rel_res_true_last_two":
                g[int(f[1])]["res"] = (float(f[2]), float(f[3]))
            elif f[0] == "norm_x":
                g[int(f[1])]["norm"] = float(f[2])
            elif f[0] == "x":
                g[int(f[1])]["idx"].append(int(f[2]))
                g[int(f[1])]["x"].append(float(f[3]))
    return [g[m] for m in range(16)]


def test_fixture_is_the_multi_mesh_workload():
    """CPU: each cube's side and level-0 pattern are those of the generated workload, and each
    stopping test has a margin on both sides of 1e-8."""
    import oracle
    g = _read()
    for (m, n, nu), rec in zip(_workload(), g):
        p = make_problem(n, nu=nu, seed=100 + m)
        A = oracle.hierarchy.apply_dirichlet(p.n_vertices, p.row_ptr, p.col_idx,
                                             np.asarray(p.vals).reshape(-1, 3, 3), p.dirichlet)
        lv0 = rec["levels"][0]
        assert rec["side"] == n and lv0["n"] == p.n_vertices and lv0["bs"] == 3
        assert lv0["A_rp"] == _digest(A.row_ptr) and lv0["A_col"] == _digest(A.col)
        assert rec["res"][1] < 1e-8 < rec["res"][0], m
        assert len(rec["idx"]) == 32


@pytest.mark.gpu
def test_sixteen_cubes_equal_the_oracle():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2011_13325_amd as E
    g = _read()
    sysm, f = [], None
    try:
        for m, n, nu in _workload():
            p = make_problem(n, nu=nu, seed=100 + m)
            h = E.Hierarchy(p.dim, p.coords, p.row_ptr, p.col_idx, p.vals, p.dirichlet,
                            E.eamg_default_setup_params(**PRM))
            sysm.append((p, h))
            rec = g[m]
            assert h.stats()["n_levels"] == len(rec["levels"]), m
            for l, lv in enumerate(rec["levels"]):
                ex = h.export(l)
                assert ex["info"]["n"] == lv["n"] and ex["info"]["bs"] == lv["bs"], (m, l)
                assert _digest(ex["A_rowptr"]) == lv["A_rp"] and _digest(ex["A_col"]) == lv["A_col"], (m, l)
                if lv["agg"] != "-":
                    assert _digest(ex["agg"]) == lv["agg"], (m, l)
                    assert _digest(ex["color"]) == lv["colors"], (m, l)
                    assert _digest(ex["P_rowptr"]) == lv["P_rp"], (m, l)
                    assert _digest(ex["P_col"]) == lv["P_col"], (m, l)
        print(f"\n[16 cubes vs oracle] hierarchies equal; k* = {[r['its'] for r in g]}", flush=True)
        f = E.Fused([h for _, h in sysm], dense_tail_dofs=4096)
        E.eamg_autotune(f.h, 0)
        bs = [torch.tensor(p.b, device="cuda") for p, _ in sysm]
        xs, st, infos = f.solve(bs, rtol=1e-8, precond=E.EAMG_PRECOND_VCYCLE)
        assert st == E.EAMG_OK
        worst = 0.0
        for m, (x, inf, rec) in enumerate(zip(xs, infos, g)):
            xh = x.cpu().numpy()
            ref = np.array(rec["x"])
            err = np.abs(xh[np.array(rec["idx"])] - ref).max() / np.abs(ref).max()
            nerr = abs(np.linalg.norm(xh) - rec["norm"]) / rec["norm"]
            worst = max(worst, err, nerr)
            assert inf["status"] == E.EAMG_OK and inf["iterations"] == rec["its"], (m, inf, rec["its"])
            assert err <= X_TOL and nerr <= X_TOL, (m, err, nerr)
        print(f"[16 cubes vs oracle] fused FP64 iterations = k* for all; worst rel err {worst:.2e}",
              flush=True)
    finally:
        if f is not None:
            f.close()
        for _, h in sysm:
            h.close()
