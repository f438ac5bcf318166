"""Learned coarsening (edge-scoring network in the matching walk), on the GPU.

* With a vanishing skip threshold the learned walk is the exact walk: identical agglomerates.
* Recorded samples: labels/weights are 0/1, and the labelled pairs are the walk's evaluations.
* Trained on the GPU (own kernels) on small heterogeneous meshes, the network is applied to a
  held-out heterogeneous mesh.  What it gains over the exact walk: fewer exact criterion
  evaluations (at least 15 % fewer; measured ~30 % on meshes of this kind) at the same
  convergence (PCG iterations at most 2 above the exact hierarchy's, true residual 1e-8).
* Every agglomerate the learned walk forms passes the exact criterion, re-checked with the
  oracle's mu_b / mu_g on the finest level (sampled agglomerates).
"""
import numpy as np
import pytest

import oracle
import paper_2011_13325_amd as E
from gen import make_problem
from oracle.auxtop import dhat_all, finest_aux
from oracle.criteria import mu_b, mu_g

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

SIGMA = 20.0


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _hier(p, **kw):
    return E.Hierarchy(p.dim, p.coords, p.row_ptr, p.col_idx, p.vals, p.dirichlet,
                       E.eamg_default_setup_params(**kw) if kw else None)


@pytest.fixture(scope="module")
def trained():
    graphs = []
    for c, (n, inc, nu) in enumerate([(12, 8, 0.3), (14, 12, 0.4), (16, 16, 0.35), (13, 10, 0.45)]):
        p = make_problem(n, inclusions=inc, nu=nu, geometry_seed=10 + c, seed=c)
        h = _hier(p, gnn_record=1)
        st = E.eamg_coarsening_stats(h.h)
        assert st["sample_passes"] >= 2
        for k in range(st["sample_passes"]):
            X, edges, nn, y, w = E.eamg_gnn_samples(h.h, k)
            assert set(np.unique(y)) <= {0.0, 1.0} and set(np.unique(w)) <= {0.0, 1.0}
            assert np.all(np.isfinite(X))
            if len(y) and w.sum() > 0:
                graphs.append((X, edges, nn, y, w))
        h.close()
    net = E.EdgeNet(seed=3)
    hist = net.train(graphs, epochs=200, lr=3e-3)
    print(f"\n[learned] {len(graphs)} graphs, loss {hist[0]:.3f} -> {hist[-1]:.3f}", flush=True)
    assert hist[-1] < 0.6 * hist[0]
    yield net
    net.close()


def test_vanishing_threshold_is_the_exact_walk(trained):
    p = make_problem(14, inclusions=10, geometry_seed=31, seed=1)
    he = _hier(p)
    hl = _hier(p, gnn=trained.h.value, gnn_skip=1e-30)
    for l in range(he.stats()["n_levels"] - 1):
        assert np.array_equal(he.export(l)["agg"], hl.export(l)["agg"])
    assert E.eamg_coarsening_stats(hl.h)["skipped"] == 0
    he.close()
    hl.close()


def test_learned_walk_gain_and_exactness(trained):
    p = make_problem(22, inclusions=25, nu=0.35, geometry_seed=77, seed=5)
    b = torch.tensor(p.b, device="cuda")
    he = _hier(p)
    hl = _hier(p, gnn=trained.h.value, gnn_skip=0.2)
    se, sl = E.eamg_coarsening_stats(he.h), E.eamg_coarsening_stats(hl.h)
    _, ie = he.solve(b)
    xl, il = hl.solve(b)
    print(f"[learned] evaluations exact {se['evaluated']} (mu_g {se['evaluated_g']}) learned "
          f"{sl['evaluated']} (mu_g {sl['evaluated_g']}, passed over {sl['skipped']}); its "
          f"{ie['iterations']} vs {il['iterations']}; oc {he.stats()['oc']:.3f} vs {hl.stats()['oc']:.3f}",
          flush=True)
    assert sl["evaluated"] <= 0.85 * se["evaluated"]
    assert il["status"] == E.EAMG_OK and il["rel_res_true"] <= 1e-8
    assert il["iterations"] <= ie["iterations"] + 2
    # every level-0 agglomerate passes the exact criterion (oracle, finest level data)
    lev = finest_aux(3, p.coords, p.row_ptr, p.col_idx, p.vals)
    D = dhat_all(lev)
    agg = hl.export(0)["agg"]
    groups = {}
    for i, a in enumerate(agg):
        if a >= 0:
            groups.setdefault(int(a), []).append(i)
    rng = np.random.default_rng(0)
    big = [g for g in groups.values() if len(g) >= 3]
    pairs = [g for g in groups.values() if len(g) == 2]
    for g in [big[i] for i in rng.choice(len(big), min(25, len(big)), replace=False)]:
        assert mu_g(lev, g, D) < SIGMA * (1 + 1e-9)
    for g in [pairs[i] for i in rng.choice(len(pairs), min(25, len(pairs)), replace=False)]:
        assert mu_b(lev, g[0], g[1], D) < SIGMA * (1 + 1e-9)
    he.close()
    hl.close()


def test_learned_walk_at_full_size(trained):
    # the bench's workload: 96^3 with 200 stiff spherical inclusions, in its configuration (FP32
    # V-cycle, caps 6 / 4 / 3, sigma 20, coarsening to < 500 dofs, dense tail); the exact
    # criterion's check of every pair is pinned above on a smaller mesh, here the gain and the
    # convergence at full size
    import scipy.sparse as sp
    p = make_problem(96, inclusions=200, nu=0.3, geometry_seed=5, seed=5)
    prm = dict(vcycle_fp32=1, coarsest_max_dofs=500, dense_tail_dofs=16384, cap_std_l0=6, cap_std=4,
               cap_aux=3, sigma=SIGMA)
    b = torch.tensor(p.b, device="cuda")
    he = _hier(p, **prm)
    hl = _hier(p, gnn=trained.h.value, gnn_skip=0.2, **prm)
    try:
        se, sl = E.eamg_coarsening_stats(he.h), E.eamg_coarsening_stats(hl.h)
        _, ie = he.solve(b, precond=E.EAMG_PRECOND_VCYCLE_FP32)
        xl, il = hl.solve(b, precond=E.EAMG_PRECOND_VCYCLE_FP32)
        print(f"\n[learned 96^3] evaluations exact {se['evaluated']} learned {sl['evaluated']} "
              f"(passed over {sl['skipped']}); its {ie['iterations']} vs {il['iterations']}", flush=True)
        assert sl["evaluated"] <= 0.85 * se["evaluated"]
        assert ie["status"] == E.EAMG_OK and il["status"] == E.EAMG_OK
        assert il["iterations"] <= ie["iterations"] + 2
        A = sp.bsr_matrix((p.vals.reshape(-1, 3, 3), p.col_idx, p.row_ptr), shape=(p.n_dofs,) * 2)
        dm = np.repeat(p.dirichlet.astype(bool), 3)
        x = xl.cpu().numpy()
        xf = np.where(dm, 0.0, x)
        r = p.b - np.where(dm, 0.0, A @ xf) - np.where(dm, x, 0.0)
        assert np.linalg.norm(r) <= 1e-8 * np.linalg.norm(p.b)
        agg = hl.export(0)["agg"]
        free = p.dirichlet == 0
        assert np.all(agg[free] >= 0) and np.all(agg[~free] == -1)
        assert np.bincount(agg[free]).max() <= 4
    finally:
        he.close()
        hl.close()


def test_bad_learned_parameters_are_rejected(trained):
    p = make_problem(5)
    with pytest.raises(E.EamgError) as ei:
        _hier(p, gnn=trained.h.value, gnn_skip=1.5)
    assert ei.value.status == E.EAMG_ERR_INVALID_ARG
