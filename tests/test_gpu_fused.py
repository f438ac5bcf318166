"""GPU tests of the fused multi-system solve (eamg_fuse, eamg_solve_fused).

Several independent systems of uneven size are merged into one block-diagonal hierarchy; each
keeps its own V-cycle (Algorithm alg:tg, its own P_s and Galerkin levels) and its own CG
scalars (section "res" per system).  Each system's iterate after K iterations is compared with
the FP64 oracle's PCG after K iterations on its own hierarchy (within 1e-10 relative, the FP64
parity bar), and with the library's own single-system solve.  The systems mix every way a
V-cycle can end: no coarsening (a dense inverse on level 0), the coarsest inverse, and dense
V-cycle tails on different levels.  Covered besides: FP32 V-cycles, graph replay against eager
launches, run-to-run reproducibility, zero, non-finite and iteration-limited systems among
healthy ones, an initial guess, autotuning of the fused hierarchy, the profiler, the lifetime
rule (a component destroyed while fused is freed later), and argument checks; each with the
V-cycles ending at the systems' own dense tails, at their coarsest inverses, and at dense tails
the fused hierarchy builds.
"""
import os

import numpy as np
import pytest
import scipy.sparse as sp

import oracle
import paper_2011_13325_amd as E
from gen import make_problem

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

# (cube side, nu, RHS seed, dense-tail dofs)
SIZES = [(4, 0.30, 1, 0), (6, 0.41, 2, 0), (9, 0.22, 3, 16384), (12, 0.35, 4, 0),
         (7, 0.45, 5, 16384), (14, 0.30, 6, 16384)]


def _hier(n, nu, seed, tail):
    p = make_problem(n, nu=nu, seed=seed)
    h = E.Hierarchy(p.dim, p.coords, p.row_ptr, p.col_idx, p.vals, p.dirichlet,
                    E.eamg_default_setup_params(vcycle_fp32=1, dense_tail_dofs=tail))
    return p, h


@pytest.fixture(scope="module")
def hierarchies():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    out = [_hier(*c) for c in SIZES]
    tails = [E.eamg_dense_tail(h.h) for _, h in out]
    print("\n[fused] levels", [h.stats()["n_levels"] for _, h in out], "tails", tails, flush=True)
    # the mix this file relies on: a single level, coarsest inverses and dense tails
    assert out[0][1].stats()["n_levels"] == 1
    assert any(t[0] >= 1 for t in tails) and any(t[0] < 0 for t in tails)
    yield out
    for _, h in out:
        h.close()


# where the fused V-cycles end: -1 at the systems' own dense tails, 0 at every coarsest inverse,
# 2048 at dense tails the fused hierarchy builds (on level 1 or 2 here, one of them where a
# system's own tail already starts)
@pytest.fixture(scope="module", params=[-1, 0, 2048], ids=["own_tails", "full", "fused_tails"])
def systems(request, hierarchies):
    f = E.Fused([h for _, h in hierarchies], dense_tail_dofs=request.param)
    yield hierarchies, f
    f.close()


def _true_res(p, x):
    A = sp.bsr_matrix((p.vals, p.col_idx, p.row_ptr), shape=(p.n_dofs,) * 2).tocsr()
    dm = np.repeat(p.dirichlet.astype(bool), p.dim)
    Dm = sp.diags((~dm).astype(float))
    Ab = Dm @ A @ Dm + sp.diags(dm.astype(float))
    return np.linalg.norm(p.b - Ab @ x) / np.linalg.norm(p.b)


def _bs(sysl):
    return [torch.tensor(p.b, device="cuda") for p, _ in sysl]


def test_fused_matches_oracle_at_fixed_iteration_count(systems):
    sysl, f = systems
    ors, kstar = [], []
    for p, _ in sysl:
        ho = oracle.setup(p.dim, p.coords, p.row_ptr, p.col_idx, p.vals, p.dirichlet)
        _, it, _, rel_true, conv = oracle.pcg(ho, p.b, rtol=1e-8)
        assert conv and rel_true <= 1e-8
        ors.append(ho)
        kstar.append(it)
    # K: the fewest iterations any coarsened system needs for 1e-8; with rtol = 1e-14 the
    # system without coarsening (a dense inverse on level 0) stops after one iteration and
    # every other one runs exactly K
    K = min(k for k in kstar if k > 2)
    print(f"[fused vs oracle] oracle its {kstar}, K={K}", flush=True)
    bs = _bs(sysl)
    xs, st, infos = f.solve(bs, rtol=1e-14, max_it=K, precond=E.EAMG_PRECOND_VCYCLE)
    worst = 0.0
    for m, ((p, _), ho, x, inf) in enumerate(zip(sysl, ors, xs, infos)):
        xo, it, *_ = oracle.pcg(ho, p.b, rtol=1e-14, max_it=K)
        assert it == inf["iterations"], (m, inf, it)
        if it < K:
            assert inf["status"] == E.EAMG_OK, (m, inf)
        else:
            assert inf["status"] == E.EAMG_NOT_CONVERGED, (m, inf)
        err = np.linalg.norm(x.cpu().numpy() - xo) / np.linalg.norm(xo)
        worst = max(worst, err)
        assert err <= 1e-10, (m, err)
    print(f"[fused vs oracle] max rel err {worst:.1e}", flush=True)


@pytest.mark.parametrize("precond", [E.EAMG_PRECOND_VCYCLE, E.EAMG_PRECOND_VCYCLE_FP32])
def test_fused_converges_like_individual_solves(systems, precond):
    sysl, f = systems
    bs = _bs(sysl)
    ref = [h.solve(b, rtol=1e-8, precond=precond) for (p, h), b in zip(sysl, bs)]
    xs, st, infos = f.solve(bs, rtol=1e-8, precond=precond)
    assert st == E.EAMG_OK
    for m, ((p, _), (xr, ir), x, inf) in enumerate(zip(sysl, ref, xs, infos)):
        assert inf["status"] == E.EAMG_OK, (m, inf)
        assert abs(inf["iterations"] - ir["iterations"]) <= 1, (m, inf, ir)
        r = _true_res(p, x.cpu().numpy())
        assert r <= 1e-8 and abs(inf["rel_res_true"] - r) <= 1e-3 * r + 1e-14, (m, r, inf)
    print(f"[fused precond={precond}] its {[i['iterations'] for i in infos]} "
          f"own {[i['iterations'] for _, i in ref]} ms {infos[0]['ms']:.2f}", flush=True)


@pytest.mark.parametrize("precond,bar", [(E.EAMG_PRECOND_VCYCLE, 1e-10),
                                         (E.EAMG_PRECOND_VCYCLE_FP32, 1e-5)])
def test_fused_equals_individual_at_fixed_count(systems, precond, bar):
    # the same recurrences as eamg_solve: after K iterations the iterates differ only by the
    # order of sums (FP64), or by FP32 rounding in that order (FP32 V-cycle)
    sysl, f = systems
    bs = _bs(sysl)
    K = 6
    xs, st, infos = f.solve(bs, rtol=1e-14, max_it=K, precond=precond)
    for m, ((p, h), b, x, inf) in enumerate(zip(sysl, bs, xs, infos)):
        xr, ir = h.solve(b, rtol=1e-14, max_it=K, precond=precond)
        # FP32: the system without coarsening gains ~1e-7 per iteration and may cross 1e-14
        # one iteration apart
        slack = 0 if precond == E.EAMG_PRECOND_VCYCLE else 1
        assert abs(inf["iterations"] - ir["iterations"]) <= slack, (m, inf, ir)
        err = float((x - xr).norm() / xr.norm())
        assert err <= bar, (m, err)


@pytest.mark.parametrize("mode", [-1, 2048], ids=["own_tails", "fused_tails"])
def test_fused_fp32_tails(hierarchies, mode):
    # systems set up with dense_tail_fp32 = 1: the fused FP32 V-cycle reads FP32 copies of the
    # dense tails (its own and the systems'), and equals each system's own FP32 solve (which
    # reads its FP32 tail) at a fixed count up to FP32 rounding
    sysl = []
    try:
        for n, nu, seed, tail in SIZES[2:5]:
            p = make_problem(n, nu=nu, seed=seed)
            sysl.append((p, E.Hierarchy(p.dim, p.coords, p.row_ptr, p.col_idx, p.vals, p.dirichlet,
                                        E.eamg_default_setup_params(vcycle_fp32=1, dense_tail_dofs=tail,
                                                                    dense_tail_fp32=1))))
        f = E.Fused([h for _, h in sysl], dense_tail_dofs=mode)
        try:
            bs = _bs(sysl)
            K = 6
            xs, _, infos = f.solve(bs, rtol=1e-14, max_it=K, precond=E.EAMG_PRECOND_VCYCLE_FP32)
            for m, ((p, h), b, x, inf) in enumerate(zip(sysl, bs, xs, infos)):
                xr, ir = h.solve(b, rtol=1e-14, max_it=K, precond=E.EAMG_PRECOND_VCYCLE_FP32)
                assert abs(inf["iterations"] - ir["iterations"]) <= 1, (m, inf, ir)
                err = float((x - xr).norm() / xr.norm())
                assert err <= 1e-5, (m, err)
            xs, st, infos = f.solve(bs, rtol=1e-8, precond=E.EAMG_PRECOND_VCYCLE_FP32)
            assert st == E.EAMG_OK
            for (p, _), x in zip(sysl, xs):
                assert _true_res(p, x.cpu().numpy()) <= 1e-8
        finally:
            f.close()
    finally:
        for _, h in sysl:
            h.close()


def test_fused_reproducible_and_graph_equals_eager(systems):
    sysl, f = systems
    bs = _bs(sysl)
    x1, _, i1 = f.solve(bs, rtol=1e-8, precond=E.EAMG_PRECOND_VCYCLE_FP32)
    x2, _, i2 = f.solve(bs, rtol=1e-8, precond=E.EAMG_PRECOND_VCYCLE_FP32)
    for a, b in zip(x1, x2):
        assert torch.equal(a, b)
    os.environ["EAMG_GRAPH"] = "0"
    try:
        f2 = E.Fused([h for _, h in sysl], dense_tail_dofs=f.dense_tail_dofs)
        x3, _, i3 = f2.solve(bs, rtol=1e-8, precond=E.EAMG_PRECOND_VCYCLE_FP32)
        f2.close()
    finally:
        del os.environ["EAMG_GRAPH"]
    for a, b, ia, ib in zip(x1, x3, i1, i3):
        assert ia["iterations"] == ib["iterations"]
        assert torch.equal(a, b)


def test_fused_special_systems(systems):
    sysl, f = systems
    bs = _bs(sysl)
    bs[1] = torch.zeros_like(bs[1])                 # zero right-hand side
    bs[3] = bs[3].clone()
    bs[3][5] = float("nan")                         # breakdown
    xs = [torch.full_like(b, 7.0) for b in bs]
    xs, st, infos = f.solve(bs, xs, rtol=1e-8)
    assert st == E.EAMG_NOT_CONVERGED
    assert infos[1]["status"] == E.EAMG_OK and infos[1]["iterations"] == 0
    assert torch.count_nonzero(xs[1]) == 0
    assert infos[3]["status"] == E.EAMG_ERR_BREAKDOWN
    assert torch.all(xs[3] == 7.0)                  # not written
    for m in (0, 2, 4, 5):
        assert infos[m]["status"] == E.EAMG_OK, (m, infos[m])
        assert _true_res(sysl[m][0], xs[m].cpu().numpy()) <= 1e-8
    # iteration limit: systems that need more stop there, NOT_CONVERGED
    xs, st, infos = f.solve(_bs(sysl), rtol=1e-12, max_it=3)
    assert st == E.EAMG_NOT_CONVERGED
    for m, inf in enumerate(infos):
        assert inf["iterations"] <= 3
        if inf["status"] != E.EAMG_OK:
            assert inf["status"] == E.EAMG_NOT_CONVERGED and inf["iterations"] == 3, (m, inf)


def test_fused_initial_guess(systems):
    sysl, f = systems
    bs = _bs(sysl)
    x0 = [torch.tensor(np.random.default_rng(60 + m).uniform(-1, 1, p.n_dofs), device="cuda")
          for m, (p, _) in enumerate(sysl)]
    ref = [h.solve(b, x.clone(), rtol=1e-14, max_it=5, use_x0=True)[0] for (p, h), b, x in zip(sysl, bs, x0)]
    xs, st, infos = f.solve(bs, [x.clone() for x in x0], rtol=1e-14, max_it=5, use_x0=True)
    for m, (x, xr) in enumerate(zip(xs, ref)):
        assert float((x - xr).norm() / xr.norm()) <= 1e-10, m


def test_fused_autotune_and_profiler():
    cases = [(5, 0.3, 11, 0), (10, 0.4, 12, 16384), (13, 0.25, 13, 0)]
    sysl = [_hier(*c) for c in cases]
    f = E.Fused([h for _, h in sysl], dense_tail_dofs=-1)
    try:
        before, after = E.eamg_autotune(f.h, 0)
        assert after <= before * 1.05
        bs = _bs(sysl)
        K = 5
        xs, st, infos = f.solve(bs, rtol=1e-14, max_it=K)
        for m, ((p, _), x) in enumerate(zip(sysl, xs)):
            ho = oracle.setup(p.dim, p.coords, p.row_ptr, p.col_idx, p.vals, p.dirichlet)
            xo, *_ = oracle.pcg(ho, p.b, rtol=1e-14, max_it=K)
            assert np.linalg.norm(x.cpu().numpy() - xo) / np.linalg.norm(xo) <= 1e-10, m
        E.eamg_profile_enable(f.h, True)
        f.solve(bs, rtol=1e-8, precond=E.EAMG_PRECOND_VCYCLE_FP32)
        names = [k["name"] for k in E.eamg_profile_read(f.h)]
        E.eamg_profile_enable(f.h, False)
        assert any(n.startswith("k_gs_color<float, 6") for n in names), names
        assert any(n.startswith("k_dense_symv_multi<") for n in names), names
    finally:
        f.close()
        for _, h in sysl:
            h.close()


def test_fused_single_system_and_plain_cg():
    # one system alone: the fused solve is that system's PCG; without a preconditioner the fused
    # CG follows each system's plain CG
    sysl = [_hier(*c) for c in [(10, 0.4, 31, 16384), (5, 0.3, 32, 0)]]
    try:
        bs = _bs(sysl)
        f1 = E.Fused([sysl[0][1]], dense_tail_dofs=-1)
        xs, st, infos = f1.solve(bs[:1], rtol=1e-14, max_it=6)
        xr, ir = sysl[0][1].solve(bs[0], rtol=1e-14, max_it=6)
        assert infos[0]["iterations"] == ir["iterations"]
        assert float((xs[0] - xr).norm() / xr.norm()) <= 1e-10
        f1.close()
        f2 = E.Fused([h for _, h in sysl], dense_tail_dofs=0)
        xs, st, infos = f2.solve(bs, rtol=1e-14, max_it=8, precond=E.EAMG_PRECOND_NONE)
        for m, ((p, h), b, x, inf) in enumerate(zip(sysl, bs, xs, infos)):
            xr, ir = h.solve(b, rtol=1e-14, max_it=8, precond=E.EAMG_PRECOND_NONE)
            assert inf["iterations"] == ir["iterations"] == 8, (m, inf, ir)
            assert float((x - xr).norm() / xr.norm()) <= 1e-10, m
        f2.close()
    finally:
        for _, h in sysl:
            h.close()


def test_fused_component_destroyed_first():
    sysl = [_hier(*c) for c in [(6, 0.3, 21, 0), (9, 0.35, 22, 16384)]]
    f = E.Fused([h for _, h in sysl], dense_tail_dofs=-1)
    bs = _bs(sysl)
    xr = [h.solve(b, rtol=1e-8)[0] for (_, h), b in zip(sysl, bs)]
    for _, h in sysl:
        h.close()                      # only marked: the fused hierarchy still reads them
    xs, st, infos = f.solve(bs, rtol=1e-8)
    assert st == E.EAMG_OK
    for p_h, x in zip(sysl, xs):
        assert _true_res(p_h[0], x.cpu().numpy()) <= 1e-8
    f.close()                          # frees the components too


def test_fused_argument_checks(systems):
    sysl, f = systems
    h0 = sysl[0][1].h
    with pytest.raises(E.EamgError) as e:
        E.eamg_fuse([h0, h0])
    assert e.value.status == E.EAMG_ERR_INVALID_ARG
    with pytest.raises(E.EamgError) as e:
        E.eamg_fuse([f.h])
    assert e.value.status == E.EAMG_ERR_INVALID_ARG
    for bad in (-2, 16385):
        with pytest.raises(E.EamgError) as e:
            E.eamg_fuse([h0], dense_tail_dofs=bad)
        assert e.value.status == E.EAMG_ERR_INVALID_ARG
    pq = make_problem(5, kind="poisson")
    hq = E.Hierarchy(pq.dim, pq.coords, pq.row_ptr, pq.col_idx, pq.vals, pq.dirichlet)
    try:
        with pytest.raises(E.EamgError) as e:
            E.eamg_fuse([h0, hq.h])
        assert e.value.status == E.EAMG_ERR_INVALID_ARG
    finally:
        hq.close()
    b = torch.zeros(10, dtype=torch.float64, device="cuda")
    for call in (lambda: E.eamg_solve(f.h, b, torch.zeros_like(b)),
                 lambda: E.eamg_vcycle(f.h, b, torch.zeros_like(b)),
                 lambda: E.eamg_vcycle_noalloc(f.h, b, torch.zeros_like(b)),
                 lambda: E.eamg_stats(f.h),
                 lambda: E.eamg_autotune(f.h, 8)):
        with pytest.raises(E.EamgError) as e:
            call()
        assert e.value.status == E.EAMG_ERR_INVALID_ARG
    with pytest.raises(E.EamgError) as e:
        E.eamg_solve_fused(h0, [b], [torch.zeros_like(b)])
    assert e.value.status == E.EAMG_ERR_INVALID_ARG
    bs = _bs(sysl)
    with pytest.raises(E.EamgError) as e:
        E.eamg_solve_fused(f.h, bs, bs)
    assert e.value.status == E.EAMG_ERR_INVALID_ARG
