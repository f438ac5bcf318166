"""Pins of the oracle's edge-scoring network (oracle/gnn.py), CPU only.

* bfloat16 rounding against values fixed by the format (7 stored mantissa bits, ties to even);
* the backward pass against central differences of the forward pass (float64, rounding off),
  for every parameter array -- a dropped term, a transposed product or a wrong aggregation
  scale each fail it;
* symmetry of the logits in the two ends of a pair and equivariance under edge reordering;
* the features against the oracle's own criteria (log mu_s) and the structure of finest-level
  edge matrices (rank one: normalized spectrum (1, 0, ..., 0)), symmetric in (i, j).
"""
import numpy as np
import pytest

from oracle import gnn
from oracle.auxtop import dhat_all, finest_aux
from oracle.criteria import mu_s, trace_strength
from gen import make_problem


def test_bf16_round_known_values():
    one = np.float32(1.0)
    vals = np.array([1.0, 1.0 + 2.0**-8, 1.0 + 3 * 2.0**-8, 1.0 + 2.0**-7, -2.5, 3.14159265,
                     65504.0, np.inf, -np.inf], dtype=np.float32)
    want = np.array([1.0, 1.0, 1.0 + 2.0**-6, 1.0 + 2.0**-7, -2.5, 3.140625, 65536.0, np.inf,
                     -np.inf], dtype=np.float32)
    assert np.array_equal(gnn.bf16_round(vals), want)
    assert np.isnan(gnn.bf16_round(np.float32(np.nan)))
    # idempotent, and the result keeps only the top 16 bits
    r = gnn.bf16_round(np.random.default_rng(0).standard_normal(1000).astype(np.float32))
    assert np.array_equal(gnn.bf16_round(r), r)
    assert np.all((r.view(np.uint32) & 0xFFFF) == 0)
    assert gnn.bf16_round(one) == one


def _toy(seed=1, n=9, m=17):
    rng = np.random.default_rng(seed)
    edges = []
    while len(edges) < m:
        a, b = sorted(rng.integers(0, n, 2))
        if a != b and (a, b) not in edges:
            edges.append((a, b))
    edges = np.array(edges)
    X = rng.standard_normal((m, gnn.F))
    y = (rng.random(m) < 0.4).astype(float)
    p = gnn.init_params(seed)
    for k in p:   # non-zero biases so every term is exercised
        if k.startswith("b"):
            p[k] = 0.1 * rng.standard_normal(p[k].shape)
    return p, X, edges, n, y


def test_gradients_match_central_differences():
    p, X, edges, n, y = _toy()
    w = np.linspace(0.5, 1.5, len(y))
    loss, g, _ = gnn.loss_and_grads(p, X, edges, n, y, weight=w, round_bf16=False)
    rng = np.random.default_rng(2)
    h = 1e-6
    for name, arr in p.items():
        idx = [tuple(rng.integers(0, s) for s in arr.shape) for _ in range(6)]
        for ix in idx:
            pp = {k: v.copy() for k, v in p.items()}
            pm = {k: v.copy() for k, v in p.items()}
            pp[name][ix] += h
            pm[name][ix] -= h
            lp = gnn.loss_and_grads(pp, X, edges, n, y, weight=w, round_bf16=False)[0]
            lm = gnn.loss_and_grads(pm, X, edges, n, y, weight=w, round_bf16=False)[0]
            fd = (lp - lm) / (2 * h)
            assert abs(fd - g[name][ix]) <= 1e-6 * max(1.0, abs(fd)) + 1e-9, (name, ix, fd, g[name][ix])


def test_logits_symmetric_and_equivariant():
    p, X, edges, n, y = _toy(3)
    z, _ = gnn.forward(p, X, edges, n)
    z2, _ = gnn.forward(p, X, edges[:, ::-1], n)
    assert np.allclose(z, z2, rtol=0, atol=1e-12)
    perm = np.random.default_rng(4).permutation(len(z))
    z3, _ = gnn.forward(p, X[perm], edges[perm], n)
    assert np.allclose(z3, z[perm], rtol=0, atol=1e-12)


def test_features_follow_the_criteria():
    prob = make_problem(5, seed=2)
    lev = finest_aux(3, prob.coords, prob.row_ptr, prob.col_idx, prob.vals)
    D = dhat_all(lev)
    mtr = trace_strength(lev)
    for e in (0, 7, 23):
        i, j = (int(v) for v in lev.edges[e])
        f = gnn.edge_features(lev.E[e], D[i], D[j], lev.M[i], lev.M[j], mtr[i], mtr[j], 1, 1)
        fr = gnn.edge_features(lev.E[e], D[j], D[i], lev.M[j], lev.M[i], mtr[j], mtr[i], 1, 1)
        assert np.array_equal(f, fr)
        assert f[0] == pytest.approx(np.log(mu_s(lev, i, j, mtr)), rel=1e-12)
        assert np.allclose(f[1:7], [1, 0, 0, 0, 0, 0], atol=1e-12)   # rank-one finest E
        assert f[7] <= f[8] and f[9] == 0.0 and f[10] == 0.5
