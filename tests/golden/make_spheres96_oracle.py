"""Write spheres96_oracle.txt: the oracle's hierarchy (exact matching walk) and PCG solve of the
heterogeneous 96^3 elasticity cube.

The workload is the 96^3 cube (884,736 vertices, clamped at x = 0) of E = 1, nu = 0.3 with 200
stiff spherical inclusions (E = 1e4, nu uniform in [0.3, 0.49]; geometry seed 5, RHS seed 5),
with the setup settings its benchmark uses: P_s row caps 6 (level-0 real-matrix rows), 4
(coarser real-matrix rows) and 3 (edge-matrix rows), sigma 20, two matching passes per level,
coarsening to < 500 dofs.  The file holds, per level, the vertex count and SHA-256 digests of
the agglomerates, the smoother colours and the patterns of A_l and P_s (every array as
little-endian int64), then the PCG iteration count k* at relative residual 1e-8 (CG with one
V-cycle, section "res"), the relative residuals of the last two iterations, ||x||_2 and x at
256 seeded positions (repr, round-trip exact).

Only oracle/ and gen/ are called.  One CPU thread; about an hour.

    python tests/golden/make_spheres96_oracle.py
"""
import hashlib
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
from gen import make_problem  # noqa: E402

SETTINGS = dict(sigma=20.0, cap_std_l0=6, cap_std=4, cap_aux=3, coarsest_max_dofs=500)
SAMPLES = 256


def digest(a):
    return hashlib.sha256(np.ascontiguousarray(np.asarray(a, dtype="<i8")).tobytes()).hexdigest()


def main():
    from threadpoolctl import threadpool_limits
    p = make_problem(96, inclusions=200, nu=0.3, geometry_seed=5, seed=5)
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        h = oracle.setup(p.dim, p.coords, p.row_ptr, p.col_idx, p.vals, p.dirichlet,
                         oracle.SetupParams(**SETTINGS))
        t_setup = time.perf_counter() - t0
        t0 = time.perf_counter()
        x, its, rel, rel_true, conv = oracle.pcg(h, p.b, rtol=1e-8)
        t_solve = time.perf_counter() - t0
        # the residuals of the last two iterations, to show the stopping test's margin
        x_prev = oracle.pcg(h, p.b, rtol=0.0, max_it=its - 1)[0]
    assert conv
    A = oracle.hierarchy.apply_dirichlet(p.n_vertices, p.row_ptr, p.col_idx,
                                         np.asarray(p.vals).reshape(-1, 3, 3), p.dirichlet)
    lines = [
        "# Oracle hierarchy (exact walk) and PCG solve: 96^3 elasticity cube, 200 stiff inclusions, "
        "geometry seed 5, RHS seed 5.",
        "# Settings: " + ", ".join(f"{k} = {v}" for k, v in SETTINGS.items()) +
        ", two matching passes per level.",
        "# Written by tests/golden/make_spheres96_oracle.py (oracle/ and gen/ only).",
        "# level n bs sha256(agg) sha256(colors) sha256(A row_ptr) sha256(A col) "
        "sha256(P row_ptr) sha256(P col)   (the coarsest level: '-' for agg, colors and P)",
    ]
    for l, lev in enumerate(h.levels):
        last = l + 1 == h.n_levels
        f = [str(l), str(lev.n), str(lev.bs),
             "-" if last else digest(lev.agg_of), "-" if last else digest(lev.colors),
             digest(lev.A.row_ptr), digest(lev.A.col),
             "-" if last else digest(lev.P.row_ptr), "-" if last else digest(lev.P.col)]
        lines.append("level " + " ".join(f))
    r_prev = np.linalg.norm(p.b - _apply(A, x_prev)) / np.linalg.norm(p.b)
    lines.append(f"iterations {its}")
    lines.append(f"rel_res_true_last_two {float(r_prev)!r} {float(rel_true)!r}")
    lines.append(f"norm_x {float(np.linalg.norm(x))!r}")
    idx = np.sort(np.random.default_rng(96).choice(p.n_dofs, SAMPLES, replace=False))
    for i in idx:
        lines.append(f"x {int(i)} {float(x[i])!r}")
    out = os.path.join(os.path.dirname(os.path.abspath(__file__)), "spheres96_oracle.txt")
    with open(out, "w") as fh:
        fh.write("\n".join(lines) + "\n")
    print(f"setup {t_setup:.1f} s, solve {t_solve:.2f} s, {its} iterations; wrote {out}")


def _apply(A, x):
    import scipy.sparse as sp
    M = sp.bsr_matrix((A.val, A.col, A.row_ptr), shape=(A.n_rows * A.r,) * 2)
    return M @ x


if __name__ == "__main__":
    main()
