"""Pin: robust coarsening criteria on the paper's coefficient-jump example.

The paper's difficult vector problem (its eleven-box geometry: stiff boxes [(i-1)/11, i/11]^3
touching at their corners inside a soft cube, contrast 1e4, paper mu = lambda) is built so that
scalar coarsening merges vertices across the stiff boxes, while the robust criteria mu_b / mu_g
(Lemma thm:mu2, Thm thm:mu1) keep such agglomerates apart.  The paper's 2D version reports a
two-grid condition number of about 2.84 with the robust criteria against about 270 with mu_s
only (figures fig:2dc_rob / fig:2dc_norob).  Here the 3D geometry on an 11-cell Kuhn cube (12^3
vertices, one cell per box) is coarsened both ways by the oracle, and the condition number of
the V-cycle preconditioned operator is estimated by Lanczos from the PCG coefficients: the
robust hierarchy must be far better conditioned (this is the trend, not the paper's values,
which are for a different 2D mesh and a two-grid method).
"""
import numpy as np
import scipy.sparse as sp

import oracle
from gen import make_problem


def _pcg_kappa(h, A, b, its):
    """PCG with the oracle V-cycle; condition number estimate from the Lanczos tridiagonal
    built from the CG coefficients alpha_k, beta_k, and the iterations to 1e-8."""
    x = np.zeros_like(b)
    r = b.copy()
    z = oracle.vcycle(h, r)
    p = z.copy()
    rz = r @ z
    alphas, betas = [], []
    nb = np.linalg.norm(b)
    done = None
    for k in range(its):
        q = A @ p
        a = rz / (p @ q)
        x += a * p
        r -= a * q
        alphas.append(a)
        if done is None and np.linalg.norm(r) <= 1e-8 * nb:
            done = k + 1
        z = oracle.vcycle(h, r)
        rz_new = r @ z
        beta = rz_new / rz
        betas.append(beta)
        rz = rz_new
        p = z + beta * p
    m = len(alphas)
    T = np.zeros((m, m))
    for k in range(m):
        T[k, k] = 1.0 / alphas[k] + (betas[k - 1] / alphas[k - 1] if k > 0 else 0.0)
        if k + 1 < m:
            T[k, k + 1] = T[k + 1, k] = np.sqrt(betas[k]) / alphas[k]
    ev = np.linalg.eigvalsh(T)
    return ev[-1] / ev[0], done


def test_robust_criteria_beat_scalar_coarsening_on_eleven_boxes():
    p = make_problem(12, boxes=True, seed=14)
    A = sp.bsr_matrix((p.vals, p.col_idx, p.row_ptr), shape=(p.n_dofs,) * 2).tocsr()
    dm = np.repeat(p.dirichlet.astype(bool), p.dim)
    Dm = sp.diags((~dm).astype(float))
    Ab = (Dm @ A @ Dm + sp.diags(dm.astype(float))).tocsr()
    out = {}
    for mso in (False, True):
        h = oracle.setup(p.dim, p.coords, p.row_ptr, p.col_idx, p.vals, p.dirichlet,
                         oracle.SetupParams(mu_s_only=mso))
        kappa, its = _pcg_kappa(h, Ab, p.b, 40)
        out[mso] = (kappa, its)
    print(f"\n[eleven boxes 12^3] robust: kappa {out[False][0]:.2f}, its {out[False][1]}; "
          f"mu_s only: kappa {out[True][0]:.1f}, its {out[True][1]}")
    assert out[False][0] < 10.0
    assert out[True][0] > 10.0 * out[False][0]
    assert out[False][1] is not None and out[False][1] <= 20
    assert out[True][1] is None or out[True][1] >= 3 * out[False][1]
