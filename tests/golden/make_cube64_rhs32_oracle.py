"""Write cube64_rhs32_oracle.txt: the oracle's PCG solves of the 32 load cases of the 64^3 cube.

The hierarchy is that of make_cube64_oracle.py (64^3 cube, nu = 0.3, P_s row caps 6 / 4 / 4,
sigma 18, two matching passes per level, coarsening to < 500 dofs).  Load case c is uniform in
[-1, 1] from numpy default_rng([4, c]), zero at the Dirichlet dofs, c = 0..31.  Per case the file
holds the PCG iteration count k* at relative residual 1e-8 (CG with one V-cycle, section "res"),
the relative residuals of the last two iterations, ||x||_2 and x at 16 seeded positions (repr,
round-trip exact).

Only oracle/ and gen/ are called.  The setup runs once (one CPU thread, about 11 minutes), then
four forked worker processes solve the cases.

    python tests/golden/make_cube64_rhs32_oracle.py
"""
import multiprocessing as mp
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from gen import make_problem  # noqa: E402

SETTINGS = dict(sigma=18.0, cap_std_l0=6, cap_std=4, cap_aux=4, coarsest_max_dofs=500)
CASES, SAMPLES = 32, 16
_H = {}


def load_case(p, c):
    b = np.random.default_rng([4, c]).uniform(-1.0, 1.0, p.n_dofs)
    b[np.repeat(p.dirichlet.astype(bool), p.dim)] = 0.0
    return b


def solve(c):
    import scipy.sparse as sp
    from threadpoolctl import threadpool_limits
    p, h = _H["p"], _H["h"]
    b = load_case(p, c)
    with threadpool_limits(limits=1):
        x, its, rel, rel_true, conv = oracle.pcg(h, b, rtol=1e-8)
        x_prev = oracle.pcg(h, b, rtol=0.0, max_it=its - 1)[0]
    assert conv
    A = h.levels[0].A
    M = sp.bsr_matrix((A.val, A.col, A.row_ptr), shape=(A.n_rows * A.r,) * 2)
    r_prev = np.linalg.norm(b - M @ x_prev) / np.linalg.norm(b)
    idx = np.sort(np.random.default_rng(500 + c).choice(p.n_dofs, SAMPLES, replace=False))
    lines = [f"iterations {c} {its}",
             f"rel_res_true_last_two {c} {float(r_prev)!r} {float(rel_true)!r}",
             f"norm_x {c} {float(np.linalg.norm(x))!r}"]
    lines += [f"x {c} {int(i)} {float(x[i])!r}" for i in idx]
    print(f"case {c}: {its} iterations", flush=True)
    return lines


def main():
    from threadpoolctl import threadpool_limits
    p = make_problem(64, seed=1)
    with threadpool_limits(limits=1):
        h = oracle.setup(p.dim, p.coords, p.row_ptr, p.col_idx, p.vals, p.dirichlet,
                         oracle.SetupParams(**SETTINGS))
    print(f"setup done, {h.n_levels} levels", flush=True)
    _H["p"], _H["h"] = p, h
    with mp.get_context("fork").Pool(4) as pool:
        res = pool.map(solve, range(CASES), chunksize=1)
    lines = ["# Oracle PCG solves of 32 load cases of the 64^3 elasticity cube (nu = 0.3).",
             "# Settings: " + ", ".join(f"{k} = {v}" for k, v in SETTINGS.items()) +
             ", two matching passes per level; case c: uniform[-1, 1] from default_rng([4, c]).",
             "# Written by tests/golden/make_cube64_rhs32_oracle.py (oracle/ and gen/ only)."]
    for r in res:
        lines += r
    out = os.path.join(os.path.dirname(os.path.abspath(__file__)), "cube64_rhs32_oracle.txt")
    with open(out, "w") as fh:
        fh.write("\n".join(lines) + "\n")
    print(f"wrote {out}")


if __name__ == "__main__":
    main()
