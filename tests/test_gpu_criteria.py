"""Coarsening criteria on the GPU (Lemma thm:mu2, Thm thm:mu1; Algorithm alg:pwagg).

The matching walks hand every pair whose criteria they need to GPU kernels in batches.  Checked:

* mu_b of pairs and mu_g of unions of three and four vertices, device against the library's host
  code through the C ABI, bit for bit (same arithmetic, no contraction), on the finest elasticity
  level (M = 0), on a coarse elasticity level (M != 0, from the oracle's matching) and on a scalar
  level (k = 1); and both against the oracle's independent numpy evaluation (relative 1e-7);
* setups with the criteria (and the coarse weights) on the GPU and on host threads give the same
  hierarchy: agglomerates of every level, the walk's evaluation counts and the matrices bit for
  bit, also with three and four passes per level; with the oracle's agglomerates too (parity
  cases), and on the eleven-box coefficient jump.
"""
import time

import numpy as np
import pytest

import oracle
import paper_2011_13325_amd as E
from gen import make_problem
from oracle.auxtop import dhat_all, finest_aux
from oracle.coarsen import successive_matching
from oracle.criteria import mu_b as o_mu_b
from oracle.criteria import mu_g as o_mu_g

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

O_RTOL = 1e-7


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _unions(lev, count, rng):
    """Connected vertex sets of 3 or 4 vertices (what the second pass unites), ascending."""
    out = []
    while len(out) < count:
        i = int(rng.integers(lev.n))
        mem = [i]
        want = int(rng.integers(3, 5))
        while len(mem) < want:
            a = mem[int(rng.integers(len(mem)))]
            nb, _ = lev.neighbors(a)
            cand = [int(v) for v in nb if int(v) not in mem]
            if not cand:
                break
            mem.append(cand[int(rng.integers(len(cand)))])
        if len(mem) >= 3:
            out.append(sorted(mem) + [-1] * (4 - len(mem)))
    return np.array(out, dtype=np.int32)


def _levels():
    pe = make_problem(11)
    l0 = finest_aux(pe.dim, pe.coords, pe.row_ptr, pe.col_idx, pe.vals)
    res = successive_matching(l0, pe.dirichlet.astype(bool))
    pp = make_problem(9, kind="poisson", clamp="all")
    ls = finest_aux(pp.dim, pp.coords, pp.row_ptr, pp.col_idx, pp.vals)
    return {"elasticity_l0": l0, "elasticity_l1": res.coarse_level, "poisson_l0": ls}


LEVELS = {}


@pytest.fixture(scope="module", params=["elasticity_l0", "elasticity_l1", "poisson_l0"])
def level(request):
    if not LEVELS:
        LEVELS.update(_levels())
    return request.param, LEVELS[request.param]


def _eval(lev, pairs, unions, dev):
    return E.eamg_criteria_eval(lev.k, lev.coords, lev.edges, lev.E, lev.M, pairs, unions,
                                use_device=dev)


def test_device_criteria_equal_host_bit_for_bit(level):
    name, lev = level
    rng = np.random.default_rng(7)
    pairs = np.asarray(lev.edges, dtype=np.int32).copy()
    flip = rng.random(len(pairs)) < 0.5               # both orientations
    pairs[flip] = pairs[flip][:, ::-1]
    unions = _unions(lev, 3000, rng)
    t0 = time.perf_counter()
    bd, gd = _eval(lev, pairs, unions, True)
    t1 = time.perf_counter()
    bh, gh = _eval(lev, pairs, unions, False)
    t2 = time.perf_counter()
    nb = int(np.sum(bd != bh) - np.sum(np.isnan(bd) & np.isnan(bh)))
    ng = int(np.sum(gd != gh) - np.sum(np.isnan(gd) & np.isnan(gh)))
    print(f"\n[criteria {name}] {len(pairs)} pairs, {len(unions)} unions: device {t1 - t0:.3f} s, "
          f"host {t2 - t1:.3f} s; differing mu_b {nb}, mu_g {ng}; finite mu_b "
          f"{np.isfinite(bd).sum()}", flush=True)
    np.testing.assert_array_equal(bd, bh)
    np.testing.assert_array_equal(gd, gh)
    assert not np.any(np.isnan(bd)) and not np.any(np.isnan(gd))


def test_device_criteria_match_oracle(level):
    name, lev = level
    rng = np.random.default_rng(11)
    pairs = np.asarray(lev.edges, dtype=np.int32)[rng.choice(len(lev.edges), 200, replace=False)]
    unions = _unions(lev, 60, rng)
    bd, gd = _eval(lev, pairs, unions, True)
    D = dhat_all(lev)
    bo = np.array([o_mu_b(lev, int(i), int(j), D) for i, j in pairs])
    go = np.array([o_mu_g(lev, [int(v) for v in u if v >= 0], D) for u in unions])
    for got, ref in ((bd, bo), (gd, go)):
        fin = np.isfinite(ref)
        assert np.array_equal(np.isfinite(got), fin)
        err = np.abs(got[fin] - ref[fin]) / np.maximum(np.abs(ref[fin]), 1e-300)
        assert err.max(initial=0.0) <= O_RTOL
    print(f"\n[criteria {name} vs oracle] finite mu_b {np.isfinite(bo).sum()}/{len(bo)}, "
          f"finite mu_g {np.isfinite(go).sum()}/{len(go)}", flush=True)


def test_criteria_eval_rejects_non_edges_and_bad_unions():
    lev = LEVELS.get("poisson_l0") or _levels()["poisson_l0"]
    i, j = (int(v) for v in lev.edges[0])
    far = int(np.setdiff1d(np.arange(lev.n), lev.neighbors(i)[0])[-1])
    for pairs, unions in (([[i, far]], np.zeros((0, 4))), ([[i, lev.n]], np.zeros((0, 4))),
                          ([[i, j]], [[j, i, -1, -1]]), ([[i, j]], [[-1, i, j, -1]]),
                          ([[i, j]], [[i, j, -1, j + 1]])):
        with pytest.raises(E.EamgError) as ei:
            _eval(lev, np.asarray(pairs), np.asarray(unions), True)
        assert ei.value.status == E.EAMG_ERR_INVALID_ARG
    b, g = _eval(lev, np.zeros((0, 2)), np.zeros((0, 4)), True)
    assert b.size == 0 and g.size == 0


def _setup(p, **prm):
    t0 = time.perf_counter()
    h = E.Hierarchy(p.dim, p.coords, p.row_ptr, p.col_idx, p.vals, p.dirichlet,
                    E.eamg_default_setup_params(**prm))
    return h, time.perf_counter() - t0


def _same_hierarchy(ha, hb):
    sa, sb = ha.stats(), hb.stats()
    assert sa["n_levels"] == sb["n_levels"] and list(sa["n"]) == list(sb["n"])
    assert E.eamg_coarsening_stats(ha.h) == E.eamg_coarsening_stats(hb.h)
    for l in range(sa["n_levels"]):
        xa, xb = E.eamg_export_level(ha.h, l), E.eamg_export_level(hb.h, l)
        assert xa["info"] == xb["info"]
        for key in xa:
            if key != "info":
                np.testing.assert_array_equal(xa[key], xb[key], err_msg=f"level {l} {key}")


@pytest.mark.parametrize("case", ["cube20", "boxes16", "poisson24", "cube14_rounds3",
                                  "cube14_rounds4"])
def test_setup_with_gpu_criteria_equals_host_criteria(case):
    extra = {}
    if case == "cube20":
        p = make_problem(20)
    elif case == "boxes16":
        p = make_problem(16, boxes=True)
    elif case == "poisson24":
        p = make_problem(24, kind="poisson", clamp="all")
    else:
        # three and four passes per level: the working level of later passes goes to the device,
        # and unions of more than four vertices are evaluated on the host
        p = make_problem(14)
        extra = dict(rounds=int(case[-1]))
    hd, td = _setup(p, gpu_criteria=2, **extra)     # every batch on the GPU
    hh, th = _setup(p, gpu_criteria=0, **extra)     # host threads only
    hm, tm = _setup(p, gpu_criteria=1, **extra)     # default: large batches on the GPU
    ev = E.eamg_coarsening_stats(hd.h)
    print(f"\n[setup {case}] setup with criteria on the GPU {td:.2f} s, on host threads "
          f"{th:.2f} s, default split {tm:.2f} s; levels {hd.stats()['n_levels']}; "
          f"evaluations {ev}", flush=True)
    _same_hierarchy(hd, hh)
    _same_hierarchy(hm, hh)
    for h in (hd, hh, hm):
        h.close()


def test_gpu_criteria_setup_matches_oracle_agglomerates():
    p = make_problem(9, ny=7, nz=5, h=0.1, nu=0.35, seed=4)
    ho = oracle.setup(p.dim, p.coords, p.row_ptr, p.col_idx, p.vals, p.dirichlet)
    hl, _ = _setup(p, gpu_criteria=2)
    assert hl.stats()["n_levels"] == ho.n_levels
    for l, lev in enumerate(ho.levels[:-1]):
        ex = E.eamg_export_level(hl.h, l)
        assert np.array_equal(ex["agg"], lev.agg_of)
    hl.close()
