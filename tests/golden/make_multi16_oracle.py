"""Write multi16_oracle.txt: the oracle's hierarchy and PCG solve of each of the 16 cubes of the
multi-mesh workload.

The workload: 16 elasticity cubes, side s_m uniform in [8, 48] vertices and Poisson ratio nu_m
uniform in [0.2, 0.45] (numpy default_rng(4): integers(8, 49, 16), then uniform(0.2, 0.45, 16)),
cube m generated with RHS seed 100 + m, each set up with its benchmark settings: P_s row caps 6
(level-0 real-matrix rows), 4 (coarser real-matrix rows) and 3 (edge-matrix rows), sigma 20,
two matching passes per level, coarsening to < 500 dofs.  Per system the file holds its side,
then per level the vertex count and SHA-256 digests of the agglomerates, smoother colours and
the patterns of A_l and P_s (as little-endian int64), the PCG iteration count k* at relative
residual 1e-8 (CG with one V-cycle, section "res"), the relative residuals of the last two
iterations, ||x||_2 and x at 32 seeded positions (repr, round-trip exact).

Only oracle/ and gen/ are called.  Four worker processes, one BLAS thread each; about ten
minutes.

    python tests/golden/make_multi16_oracle.py
"""
import hashlib
import multiprocessing as mp
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

SETTINGS = dict(sigma=20.0, cap_std_l0=6, cap_std=4, cap_aux=3, coarsest_max_dofs=500)
SAMPLES = 32


def workload():
    rng = np.random.default_rng(4)
    sides = rng.integers(8, 49, size=16)
    nus = rng.uniform(0.2, 0.45, size=16)
    return [(m, int(n), float(nu)) for m, (n, nu) in enumerate(zip(sides, nus))]


def digest(a):
    return hashlib.sha256(np.ascontiguousarray(np.asarray(a, dtype="<i8")).tobytes()).hexdigest()


def one(args):
    m, n, nu = args
    from threadpoolctl import threadpool_limits
    import scipy.sparse as sp
    import oracle
    from gen import make_problem
    p = make_problem(n, nu=nu, seed=100 + m)
    with threadpool_limits(limits=1):
        h = oracle.setup(p.dim, p.coords, p.row_ptr, p.col_idx, p.vals, p.dirichlet,
                         oracle.SetupParams(**SETTINGS))
        x, its, rel, rel_true, conv = oracle.pcg(h, p.b, rtol=1e-8)
        x_prev = oracle.pcg(h, p.b, rtol=0.0, max_it=its - 1)[0]
    assert conv
    A = h.levels[0].A
    M = sp.bsr_matrix((A.val, A.col, A.row_ptr), shape=(A.n_rows * A.r,) * 2)
    r_prev = np.linalg.norm(p.b - M @ x_prev) / np.linalg.norm(p.b)
    lines = [f"system {m} side {n}"]
    for l, lev in enumerate(h.levels):
        last = l + 1 == h.n_levels
        f = [str(m), str(l), str(lev.n), str(lev.bs),
             "-" if last else digest(lev.agg_of), "-" if last else digest(lev.colors),
             digest(lev.A.row_ptr), digest(lev.A.col),
             "-" if last else digest(lev.P.row_ptr), "-" if last else digest(lev.P.col)]
        lines.append("level " + " ".join(f))
    lines.append(f"iterations {m} {its}")
    lines.append(f"rel_res_true_last_two {m} {float(r_prev)!r} {float(rel_true)!r}")
    lines.append(f"norm_x {m} {float(np.linalg.norm(x))!r}")
    idx = np.sort(np.random.default_rng(1000 + m).choice(p.n_dofs, SAMPLES, replace=False))
    lines += [f"x {m} {int(i)} {float(x[i])!r}" for i in idx]
    print(f"system {m}: side {n}, {h.n_levels} levels, {its} iterations", flush=True)
    return lines


def main():
    work = sorted(workload(), key=lambda w: -w[1])   # largest first
    with mp.Pool(4) as pool:
        res = dict(zip([w[0] for w in work], pool.map(one, work, chunksize=1)))
    lines = ["# Oracle hierarchies and PCG solves of the 16-cube multi-mesh workload.",
             "# Settings: " + ", ".join(f"{k} = {v}" for k, v in SETTINGS.items()) +
             ", two matching passes per level; cube m: RHS seed 100 + m.",
             "# Written by tests/golden/make_multi16_oracle.py (oracle/ and gen/ only).",
             "# level m l n bs sha256(agg) sha256(colors) sha256(A row_ptr) sha256(A col) "
             "sha256(P row_ptr) sha256(P col)   (the coarsest level: '-' for agg, colors and P)"]
    for m in range(16):
        lines += res[m]
    out = os.path.join(os.path.dirname(os.path.abspath(__file__)), "multi16_oracle.txt")
    with open(out, "w") as fh:
        fh.write("\n".join(lines) + "\n")
    print(f"wrote {out}")


if __name__ == "__main__":
    main()
