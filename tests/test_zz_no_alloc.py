"""GPU test of eamg_vcycle_noalloc (the V-cycle for callers that cannot allocate): through the C
ABI, two calls in a row -- a larger hierarchy, then a smaller one, sharing the library's fixed
staging array -- each equal bit for bit to eamg_vcycle on the same hierarchy (same kernels in the
same order; eamg_vcycle is itself checked against the FP64 oracle's V-cycle in
test_gpu_parity.py), in FP64 and FP32, without a dense tail and with one (FP64, or with its FP32
copy); and the size limit, the
profiler check and the precision check."""
import numpy as np
import pytest

import paper_2011_13325_amd as E
from gen import make_problem

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _hier(p, **prm):
    return E.Hierarchy(p.dim, p.coords, p.row_ptr, p.col_idx, p.vals, p.dirichlet,
                       E.eamg_default_setup_params(vcycle_fp32=1, **prm))


def _r(p, seed):
    r = np.random.default_rng(seed).standard_normal(p.n_dofs)
    return torch.tensor(r, device="cuda")


@pytest.mark.parametrize("tail,tail32", [(0, 0), (16384, 0), (16384, 1)])
def test_noalloc_vcycle_equals_vcycle_on_two_calls(tail, tail32):
    big = make_problem(14, nu=0.35, seed=2)
    small = make_problem(7, seed=3)
    hb = _hier(big, dense_tail_dofs=tail, dense_tail_fp32=tail32)
    hs = _hier(small, dense_tail_dofs=tail, dense_tail_fp32=tail32)
    try:
        for prec in (E.EAMG_PRECOND_VCYCLE, E.EAMG_PRECOND_VCYCLE_FP32):
            for p, h, seed in ((big, hb, 1), (small, hs, 2)):
                r = _r(p, seed)
                z_ref = torch.empty_like(r)
                E.eamg_vcycle(h.h, r, z_ref, prec)
                z = torch.full_like(r, float("nan"))
                stream = torch.cuda.current_stream()
                E.eamg_vcycle_noalloc(h.h, r, z, prec, stream=stream)
                torch.cuda.synchronize()
                assert torch.equal(z, z_ref), (p.n_vertices, prec, tail, tail32)
                print(f"[noalloc tail={tail} tail32={tail32} prec={prec}] n={p.n_dofs} equal", flush=True)
    finally:
        hb.close()
        hs.close()


def test_noalloc_rejects_large_levels_and_profiler():
    p = make_problem(6, seed=4)
    h = _hier(p)
    try:
        r = _r(p, 5)
        z = torch.empty_like(r)
        E.eamg_profile_enable(h.h, True)
        with pytest.raises(E.EamgError) as ei:
            E.eamg_vcycle_noalloc(h.h, r, z)
        assert ei.value.status == E.EAMG_ERR_INVALID_ARG
        E.eamg_profile_enable(h.h, False)
        with pytest.raises(E.EamgError) as ei:
            E.eamg_vcycle_noalloc(h.h, r, z, precision=7)
        assert ei.value.status == E.EAMG_ERR_INVALID_ARG
    finally:
        h.close()
    # 2,097,152 dofs at most: a 90^3 elasticity cube (2,187,000 dofs) is refused before any work
    p = make_problem(90, seed=1)
    h = _hier(p, coarsest_max_dofs=16384)
    try:
        r = _r(p, 6)
        z = torch.zeros_like(r)
        with pytest.raises(E.EamgError) as ei:
            E.eamg_vcycle_noalloc(h.h, r, z)
        assert ei.value.status == E.EAMG_ERR_INVALID_ARG
        assert float(z.abs().max()) == 0.0
    finally:
        h.close()
