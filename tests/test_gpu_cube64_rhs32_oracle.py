"""Full-size parity of the batched block-panel solve: the 64^3 cube's 32 load cases solved as one
panel against the oracle's single-vector PCG solves of each case
(tests/golden/cube64_rhs32_oracle.txt, written by tests/golden/make_cube64_rhs32_oracle.py,
which calls only oracle/ and gen/).

The library runs the benchmark's configuration of this workload: the 64^3 hierarchy of
test_gpu_cube64_oracle.py (whose levels equal the oracle's bit for bit), its dense V-cycle tail,
launch shapes autotuned for 32-column panels, and the 32 load cases as one batch with the FP64
V-cycle.  Every column runs its own PCG recurrence (section "res" per column): each must stop at
the oracle's iteration count k* for relative residual 1e-8, and its iterate must equal the
oracle's at 16 seeded positions and in its 2-norm within 1e-10 relative (the FP64 parity bar).
"""
import os
from collections import defaultdict

import numpy as np
import pytest

from gen import make_problem

GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "cube64_rhs32_oracle.txt")
BENCH64 = dict(vcycle_fp32=1, coarsest_max_dofs=500, dense_tail_dofs=16384, cap_std_l0=6,
               cap_std=4, cap_aux=4, sigma=18.0)
CASES = 32
X_TOL = 1e-10


def _read():
    g = defaultdict(lambda: {"idx": [], "x": []})
    with open(GOLD) as fh:
        for line in fh:
            f = line.split()
            if not f or f[0].startswith("#"):
                continue
            c = int(f[1])
            if f[0] == "iterations":
                g[c]["its"] = int(f[2])
            elif f[0] == "rel_res_true_last_two":
                g[c]["res"] = (float(f[2]), float(f[3]))
            elif f[0] == "norm_x":
                g[c]["norm"] = float(f[2])
            elif f[0] == "x":
                g[c]["idx"].append(int(f[2]))
                g[c]["x"].append(float(f[3]))
    return [g[c] for c in range(CASES)]


def _load_cases(p):
    B = np.stack([np.random.default_rng([4, c]).uniform(-1.0, 1.0, p.n_dofs) for c in range(CASES)])
    B[:, np.repeat(p.dirichlet.astype(bool), p.dim)] = 0.0
    return B


def test_fixture_has_every_load_case():
    """CPU: 32 cases, each with 16 samples and a stopping-test margin on both sides of 1e-8."""
    g = _read()
    assert len(g) == CASES
    for c, rec in enumerate(g):
        assert len(rec["idx"]) == 16 and rec["its"] > 0, c
        assert rec["res"][1] < 1e-8 < rec["res"][0], c


@pytest.mark.gpu
def test_cube64_panel_of_32_load_cases_equals_the_oracle():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2011_13325_amd as E
    g = _read()
    p = make_problem(64, seed=1)
    h = E.Hierarchy(p.dim, p.coords, p.row_ptr, p.col_idx, p.vals, p.dirichlet,
                    E.eamg_default_setup_params(**BENCH64))
    try:
        E.eamg_autotune(h.h, panel_width=32)
        Bd = torch.tensor(_load_cases(p), device="cuda")
        X, st, infos = h.solve_batch(Bd, rtol=1e-8, precond=E.EAMG_PRECOND_VCYCLE)
        assert st == E.EAMG_OK
        Xh = X.cpu().numpy()
        worst = 0.0
        for c, (inf, rec) in enumerate(zip(infos, g)):
            ref = np.array(rec["x"])
            err = np.abs(Xh[c][np.array(rec["idx"])] - ref).max() / np.abs(ref).max()
            nerr = abs(np.linalg.norm(Xh[c]) - rec["norm"]) / rec["norm"]
            worst = max(worst, err, nerr)
            assert inf["status"] == E.EAMG_OK and inf["iterations"] == rec["its"], (c, inf, rec["its"])
            assert err <= X_TOL and nerr <= X_TOL, (c, err, nerr)
        print(f"\n[cube64 32 load cases vs oracle] k* = {[r['its'] for r in g]}; "
              f"worst rel err {worst:.2e}", flush=True)
    finally:
        h.close()
