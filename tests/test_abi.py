"""The C ABI without a GPU: the library loads and exports every symbol include/eamg.h
declares; input validation returns the documented status before any device work; the
host-side successive matching (Algorithm alg:pwagg) reproduces the oracle's agglomerates
bit for bit."""
import ctypes
import os
import re

import numpy as np
import pytest

import paper_2011_13325_amd as E
from gen import make_problem
from oracle.auxtop import finest_aux
from oracle.coarsen import successive_matching

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_library_exports_every_declared_symbol():
    hdr = open(os.path.join(ROOT, "include", "eamg.h")).read()
    hdr = re.sub(r"/\*.*?\*/", "", hdr, flags=re.S)
    declared = set(re.findall(r"\b(eamg_[a-z_]+)\s*\(", hdr))
    assert declared == set(E.EXPORTED)
    lib = ctypes.CDLL(E.LIB_PATH)
    for name in declared:
        assert hasattr(lib, name), name


def _setup_status(p, **kw):
    pb, keep = E._problem(p["dim"], p["coords"], p["row_ptr"], p["col_idx"], p["vals"],
                          p.get("dirichlet"), p.get("kernel"), p.get("edges"))
    for k, v in kw.items():
        setattr(pb, k, v)
    h = ctypes.c_void_p()
    prm = p.get("params")
    st = E.lib().eamg_setup(ctypes.byref(pb), ctypes.byref(prm) if prm is not None else None,
                            ctypes.c_void_p(0), ctypes.byref(h))
    assert not h.value
    return st, E.eamg_last_error()


def _base():
    g = make_problem(4)
    return dict(dim=3, coords=g.coords, row_ptr=g.row_ptr.copy(), col_idx=g.col_idx.copy(),
                vals=g.vals.copy(), dirichlet=g.dirichlet)


def test_malformed_inputs_are_rejected_before_device_work():
    p = _base()
    p["col_idx"][[1, 2]] = p["col_idx"][[2, 1]]              # unsorted row
    assert _setup_status(p)[0] == E.EAMG_ERR_INVALID_ARG
    p = _base()
    rp = p["row_ptr"]
    p["col_idx"] = np.delete(p["col_idx"], 0)                # drop row 0's diagonal block
    p["vals"] = np.delete(p["vals"], 0, axis=0)
    p["row_ptr"] = np.concatenate([[0], rp[1:] - 1])
    st, msg = _setup_status(p)
    assert st == E.EAMG_ERR_INVALID_ARG and "diagonal" in msg
    p = _base()
    # asymmetric pattern: remove block (0, 1) but keep (1, 0)
    s = p["row_ptr"][0]
    j = np.nonzero(p["col_idx"][s:p["row_ptr"][1]] == 1)[0][0] + s
    p["col_idx"] = np.delete(p["col_idx"], j)
    p["vals"] = np.delete(p["vals"], j, axis=0)
    p["row_ptr"] = np.concatenate([[0], p["row_ptr"][1:] - 1])
    assert _setup_status(p)[0] == E.EAMG_ERR_INVALID_ARG
    p = _base()
    p["vals"][5, 1, 1] = np.nan
    assert _setup_status(p)[0] == E.EAMG_ERR_INVALID_ARG
    p = _base()
    assert _setup_status(p, dim=2)[0] == E.EAMG_ERR_UNSUPPORTED_KERNEL
    p = _base()
    st, msg = _setup_status(p, n_vertices=0)                 # empty problem
    assert st == E.EAMG_ERR_INVALID_ARG and "n_vertices" in msg
    p = _base()
    p["params"] = E.eamg_default_setup_params(delta=0)
    assert _setup_status(p)[0] == E.EAMG_ERR_INVALID_ARG
    p = _base()
    p["params"] = E.eamg_default_setup_params(rounds=9)
    assert _setup_status(p)[0] == E.EAMG_ERR_INVALID_ARG
    for bad in (-1, 3):
        p = _base()
        p["params"] = E.eamg_default_setup_params(gpu_criteria=bad)
        assert _setup_status(p)[0] == E.EAMG_ERR_INVALID_ARG


def test_kernel_vectors_must_span_rigid_body_modes():
    p = _base()
    n = p["coords"].shape[0]
    rng = np.random.default_rng(0)
    p["kernel"] = rng.standard_normal((3 * n, 6))
    assert _setup_status(p)[0] == E.EAMG_ERR_UNSUPPORTED_KERNEL
    p = _base()
    p["kernel"] = np.zeros((3 * n, 6))
    assert _setup_status(p)[0] == E.EAMG_ERR_UNSUPPORTED_KERNEL


@pytest.mark.parametrize("n,kind", [(9, "elasticity"), (13, "elasticity"), (8, "poisson")])
def test_host_matching_matches_oracle_bit_for_bit(n, kind):
    p = make_problem(n, kind=kind, clamp="x0" if kind == "elasticity" else "all")
    lev = finest_aux(p.dim, p.coords, p.row_ptr, p.col_idx, p.vals)
    vd = p.dirichlet.astype(bool)
    for level in range(2):
        res = successive_matching(lev, vd)
        agg, nc, cc, margin = E.eamg_host_match(lev.k, lev.coords, lev.edges, lev.E, lev.M, vd)
        ao = np.full(lev.n, -1)
        for I, m in enumerate(res.aggs):
            ao[m] = I
        assert nc == len(res.aggs)
        assert np.array_equal(agg, ao)
        assert np.abs(cc - res.coarse_coords).max() <= 1e-15
        lev, vd = res.coarse_level, np.zeros(res.coarse_level.n, bool)


def test_solve_entry_points_reject_null_hierarchy():
    """Argument checks that run before any device work (no GPU needed)."""
    import ctypes
    L = E.lib()
    sp = E.eamg_solve_params(1e-8, 10, 0, 1)
    info = (E.eamg_solve_info * 2)()
    buf = ctypes.c_void_p(16)
    assert L.eamg_solve_batch(None, 2, buf, 8, buf, ctypes.byref(sp), None, info) == E.EAMG_ERR_INVALID_ARG
    assert L.eamg_solve(None, buf, buf, ctypes.byref(sp), None, info) == E.EAMG_ERR_INVALID_ARG
    assert L.eamg_vcycle(None, buf, buf, E.EAMG_PRECOND_VCYCLE, None) == E.EAMG_ERR_INVALID_ARG
    v, it = ctypes.c_double(), ctypes.c_double()
    assert L.eamg_traffic_model(None, 1, ctypes.byref(v), ctypes.byref(it)) == E.EAMG_ERR_INVALID_ARG
    p = E.eamg_default_setup_params()
    assert p.vcycle_fp32 == 0
    assert p.gpu_criteria == 1


@pytest.mark.parametrize("mu_s_only", [0, 1])
def test_host_matching_on_eleven_boxes_matches_oracle(mu_s_only):
    """The coefficient-jump geometry, robust and scalar-only pairing: the library's host matching
    equals the oracle's agglomerates bit for bit (two passes, two levels)."""
    p = make_problem(12, boxes=True, seed=14)
    lev = finest_aux(p.dim, p.coords, p.row_ptr, p.col_idx, p.vals)
    vd = p.dirichlet.astype(bool)
    prm = E.eamg_default_setup_params(mu_s_only=mu_s_only)
    for level in range(2):
        res = successive_matching(lev, vd, mu_s_only=bool(mu_s_only))
        agg, nc, cc, margin = E.eamg_host_match(lev.k, lev.coords, lev.edges, lev.E, lev.M, vd, prm)
        ao = np.full(lev.n, -1)
        for I, m in enumerate(res.aggs):
            ao[m] = I
        assert nc == len(res.aggs)
        assert np.array_equal(agg, ao)
        lev, vd = res.coarse_level, np.zeros(res.coarse_level.n, bool)


@pytest.mark.parametrize("kind", ["elasticity", "poisson"])
def test_host_criteria_match_oracle(kind):
    """mu_b (Lemma thm:mu2) and mu_g (Thm thm:mu1) of the library's host code against the oracle's
    numpy evaluation, on the finest level and on a coarse level (vertex weights M != 0)."""
    from oracle.auxtop import dhat_all
    from oracle.criteria import mu_b as o_mu_b, mu_g as o_mu_g
    p = make_problem(8, kind=kind, clamp="x0" if kind == "elasticity" else "all")
    lev = finest_aux(p.dim, p.coords, p.row_ptr, p.col_idx, p.vals)
    rng = np.random.default_rng(5)
    for level in range(2):
        pairs = np.asarray(lev.edges, np.int32)[rng.choice(len(lev.edges), 80, replace=False)]
        unions = []
        for i, j in pairs[:30]:
            nb = [int(v) for v in lev.neighbors(int(j))[0] if v != i]
            if nb:
                mem = sorted({int(i), int(j), nb[0]} | ({nb[-1]} if len(nb) > 1 else set()))
                unions.append(mem + [-1] * (4 - len(mem)))
        mub, mug = E.eamg_criteria_eval(lev.k, lev.coords, lev.edges, lev.E, lev.M, pairs,
                                        np.asarray(unions), use_device=False)
        D = dhat_all(lev)
        bo = np.array([o_mu_b(lev, int(i), int(j), D) for i, j in pairs])
        go = np.array([o_mu_g(lev, [v for v in u if v >= 0], D) for u in unions])
        for got, ref in ((mub, bo), (mug, go)):
            fin = np.isfinite(ref)
            assert np.array_equal(np.isfinite(got), fin)
            assert np.all(np.abs(got[fin] - ref[fin]) <= 1e-7 * np.abs(ref[fin]))
        res = successive_matching(lev, p.dirichlet.astype(bool) if level == 0 else np.zeros(lev.n, bool))
        lev = res.coarse_level


def test_criteria_eval_argument_checks_on_the_host():
    p = make_problem(5, kind="poisson", clamp="all")
    lev = finest_aux(p.dim, p.coords, p.row_ptr, p.col_idx, p.vals)
    i, j = (int(v) for v in lev.edges[0])
    far = int(np.setdiff1d(np.arange(lev.n), lev.neighbors(i)[0])[-1])
    for pairs, unions in (([[i, far]], np.zeros((0, 4))), ([[i, j]], [[j, i, -1, -1]]),
                          ([[i, j]], [[i, lev.n, -1, -1]])):
        with pytest.raises(E.EamgError) as ei:
            E.eamg_criteria_eval(lev.k, lev.coords, lev.edges, lev.E, lev.M, np.asarray(pairs),
                                 np.asarray(unions), use_device=False)
        assert ei.value.status == E.EAMG_ERR_INVALID_ARG
    b, g = E.eamg_criteria_eval(lev.k, lev.coords, lev.edges, lev.E, lev.M, np.zeros((0, 2)),
                                np.zeros((0, 4)), use_device=False)
    assert b.size == 0 and g.size == 0
