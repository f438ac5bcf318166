"""GPU tests of eamg_solve_multi: independent systems of uneven size solved together.

Each system follows eamg_solve's recurrence with the same kernels in the same order, so its
result must equal its own eamg_solve bit for bit.  Each system is also compared with the FP64
oracle's PCG (CG preconditioned by one V-cycle, section "res") on its own hierarchy: at a
fixed iteration count the iterates agree within 1e-10 relative (the FP64 parity bar).
Covered: meshes of different sizes and Poisson ratios (including one without coarsening),
FP64 and FP32 V-cycles, graph replay against eager launches, a system with a non-finite
right-hand side among healthy ones, a zero right-hand side, ordering after the caller's stream
(b and x0 written there just before the call), and argument checks.
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

SIZES = [(4, 0.30, 1), (6, 0.41, 2), (9, 0.22, 3), (12, 0.35, 4), (7, 0.45, 5)]


@pytest.fixture(scope="module")
def systems():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    out = []
    for n, nu, seed in SIZES:
        p = make_problem(n, nu=nu, seed=seed)
        h = E.Hierarchy(p.dim, p.coords, p.row_ptr, p.col_idx, p.vals, p.dirichlet,
                        E.eamg_default_setup_params(vcycle_fp32=1))
        out.append((p, h))
    print("\n[multi] levels", [h.stats()["n_levels"] for _, h in out], flush=True)
    yield out
    for _, h in out:
        h.close()


def _true_res(p, x):
    A = sp.bsr_matrix((p.vals, p.col_idx, p.row_ptr), shape=(p.n_dofs,) * 2).tocsr()
    dm = np.repeat(p.dirichlet.astype(bool), p.dim)
    Dm = sp.diags((~dm).astype(float))
    Ab = Dm @ A @ Dm + sp.diags(dm.astype(float))
    return np.linalg.norm(p.b - Ab @ x) / np.linalg.norm(p.b)


@pytest.mark.parametrize("precond", [E.EAMG_PRECOND_VCYCLE, E.EAMG_PRECOND_VCYCLE_FP32])
def test_multi_equals_individual_solves(systems, precond):
    bs = [torch.tensor(p.b, device="cuda") for p, _ in systems]
    ref = [h.solve(b, rtol=1e-8, precond=precond) for (p, h), b in zip(systems, bs)]
    xs = [torch.full_like(b, 3.0) for b in bs]
    st, infos = E.eamg_solve_multi([h.h for _, h in systems], bs, xs, rtol=1e-8, precond=precond)
    assert st == E.EAMG_OK
    for m, ((p, _), (xr, ir), x, inf) in enumerate(zip(systems, ref, xs, infos)):
        assert inf["status"] == E.EAMG_OK and inf["iterations"] == ir["iterations"], (m, inf, ir)
        assert torch.equal(x, xr), m
        assert _true_res(p, x.cpu().numpy()) <= 1e-8
    print(f"[multi precond={precond}] its {[i['iterations'] for i in infos]}", flush=True)


def test_multi_matches_oracle_at_fixed_iteration_count(systems):
    # every system's iterate after K iterations against the oracle's PCG after K iterations;
    # K is the smallest iteration count the oracle needs to reach 1e-8 on any of the systems
    ors, kstar = [], []
    for p, _ in systems:
        ho = oracle.setup(p.dim, p.coords, p.row_ptr, p.col_idx, p.vals, p.dirichlet)
        _, it, _, rel_true, conv = oracle.pcg(ho, p.b, rtol=1e-8)
        assert conv and rel_true <= 1e-8
        ors.append(ho)
        kstar.append(it)
    K = min(kstar)
    bs = [torch.tensor(p.b, device="cuda") for p, _ in systems]
    xs = [torch.zeros_like(b) for b in bs]
    st, infos = E.eamg_solve_multi([h.h for _, h in systems], bs, xs, rtol=0.0, max_it=K)
    worst = 0.0
    for m, ((p, _), ho, x, inf) in enumerate(zip(systems, ors, xs, infos)):
        xo, it, *_ = oracle.pcg(ho, p.b, rtol=0.0, max_it=K)
        if inf["iterations"] < K:       # a system without coarsening can be solved exactly
            assert inf["status"] == E.EAMG_OK and it == inf["iterations"], (m, inf, it)
        else:
            assert it == K and inf["iterations"] == K, (m, inf, it)
        err = np.linalg.norm(x.cpu().numpy() - xo) / np.linalg.norm(xo)
        worst = max(worst, err)
        assert err <= 1e-10, (m, err)
    print(f"[multi vs oracle] K={K} oracle its {kstar} max rel err {worst:.1e}", flush=True)


def test_multi_waits_for_callers_stream(systems):
    # b and x0 are written on the caller's stream behind a long-running kernel, right before
    # the call on that stream: the systems' own streams must not read them earlier
    hs = [h.h for _, h in systems]
    ref = []
    x0s = [torch.tensor(np.random.default_rng(40 + m).uniform(-1, 1, p.n_dofs), device="cuda")
           for m, (p, _) in enumerate(systems)]
    for (p, h), x0 in zip(systems, x0s):
        x, info = h.solve(torch.tensor(p.b, device="cuda"), x0.clone(), rtol=1e-8, use_x0=True)
        ref.append(x)
    cs = torch.cuda.Stream()
    bs = [torch.zeros(p.n_dofs, dtype=torch.float64, device="cuda") for p, _ in systems]
    xs = [torch.zeros_like(b) for b in bs]
    srcb = [torch.tensor(p.b, device="cuda") for p, _ in systems]
    torch.cuda.synchronize()
    with torch.cuda.stream(cs):
        torch.cuda._sleep(50_000_000)
        for b, sb, x, x0 in zip(bs, srcb, xs, x0s):
            b.copy_(sb)
            x.copy_(x0)
        st, infos = E.eamg_solve_multi(hs, bs, xs, rtol=1e-8, use_x0=True, stream=cs)
    assert st == E.EAMG_OK
    for m, (x, xr) in enumerate(zip(xs, ref)):
        assert torch.equal(x, xr), m


def test_multi_graph_equals_eager(systems):
    bs = [torch.tensor(p.b, device="cuda") for p, _ in systems]
    hs = [h.h for _, h in systems]
    xg = [torch.zeros_like(b) for b in bs]
    E.eamg_solve_multi(hs, bs, xg, rtol=1e-8)
    old = os.environ.get("EAMG_GRAPH")
    os.environ["EAMG_GRAPH"] = "0"
    try:
        xe = [torch.zeros_like(b) for b in bs]
        E.eamg_solve_multi(hs, bs, xe, rtol=1e-8)
    finally:
        if old is None:
            del os.environ["EAMG_GRAPH"]
        else:
            os.environ["EAMG_GRAPH"] = old
    for a, b in zip(xg, xe):
        assert torch.equal(a, b)


def test_multi_failing_and_zero_systems(systems):
    bs = [torch.tensor(p.b, device="cuda") for p, _ in systems]
    p1 = systems[1][0]
    free = np.nonzero(~np.repeat(p1.dirichlet.astype(bool), p1.dim))[0]
    bs[1][int(free[2])] = float("nan")
    bs[3] = torch.zeros_like(bs[3])
    xs = [torch.full_like(b, 5.0) for b in bs]
    st, infos = E.eamg_solve_multi([h.h for _, h in systems], bs, xs, rtol=1e-8)
    assert st == E.EAMG_NOT_CONVERGED
    assert [i["status"] for i in infos] == [E.EAMG_OK, E.EAMG_ERR_BREAKDOWN, E.EAMG_OK, E.EAMG_OK, E.EAMG_OK]
    assert float(xs[1].min()) == 5.0 and float(xs[1].max()) == 5.0    # not written
    assert infos[3]["iterations"] == 0 and float(xs[3].abs().max()) == 0.0
    for m in (0, 2, 4):
        xr, _ = systems[m][1].solve(bs[m], rtol=1e-8)
        assert torch.equal(xs[m], xr)
    # the iteration limit holds per system
    st, infos = E.eamg_solve_multi([systems[2][1].h, systems[4][1].h], [bs[2], bs[4]],
                                   [xs[2], xs[4]], rtol=1e-12, max_it=3)
    assert st == E.EAMG_NOT_CONVERGED and all(i["iterations"] == 3 for i in infos)


def test_multi_rejects_bad_arguments(systems):
    p, h = systems[0]
    b = torch.tensor(p.b, device="cuda")
    with pytest.raises(E.EamgError) as ei:
        E.eamg_solve_multi([h.h, h.h], [b, b.clone()], [torch.zeros_like(b), torch.zeros_like(b)])
    assert ei.value.status == E.EAMG_ERR_INVALID_ARG
    with pytest.raises(E.EamgError) as ei:
        E.eamg_solve_multi([h.h], [b], [b])
    assert ei.value.status == E.EAMG_ERR_INVALID_ARG
