"""Hand-worked fixtures under tests/golden/ against the oracle (CPU).

pwagg_path4.txt: successive pairwise matching (Algorithm alg:pwagg) on a four-vertex scalar
path, with the criteria it decides by (mu_D of Thm thm:mu1, mu_s of Def. def:muc, mu_b of Lemma
thm:mu2, mu_g of Thm thm:mu1) worked out by hand in the fixture's header."""
import os

import numpy as np
import pytest

from oracle.auxtop import AuxLevel, dhat_all
from oracle.coarsen import successive_matching
from oracle.criteria import mu_D, mu_b, mu_g, mu_s, trace_strength

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _cases(name):
    cases, cur = [], None
    for raw in open(os.path.join(GOLDEN, name)):
        line = raw.split("#", 1)[0].strip()
        if not line:
            continue
        key, _, val = (t.strip() for t in line.partition("="))
        if key == "case":
            cur = {"case": val}
            cases.append(cur)
        else:
            cur[key] = val
    return cases


def _pairs(spec):
    """'0-1 1.5, 1-2 2.0' -> {(0, 1): 1.5, (1, 2): 2.0}"""
    out = {}
    for item in spec.split(","):
        ij, v = item.split()
        i, j = (int(t) for t in ij.split("-"))
        out[(i, j)] = float(v)
    return out


def _path4(M):
    edges = np.array([[0, 1], [1, 2], [2, 3]], dtype=np.int64)
    E = np.array([1.0, 2.0, 1.0]).reshape(-1, 1, 1)
    coords = np.zeros((4, 3))
    coords[:, 0] = np.arange(4)
    return AuxLevel(1, coords, edges, E, np.asarray(M, dtype=np.float64).reshape(4, 1, 1))


CASES = _cases("pwagg_path4.txt")


@pytest.mark.parametrize("c", CASES, ids=[c["case"] for c in CASES])
def test_pwagg_path4(c):
    lev = _path4([float(v) for v in c["M"].split()])
    r = successive_matching(lev, np.zeros(4, dtype=bool), sigma=float(c["sigma"]), rounds=int(c["rounds"]))
    aggs = [[int(v) for v in grp.split()] for grp in c["aggregates"].split("|")]
    assert [a.tolist() for a in r.aggs] == aggs
    assert np.nonzero(r.dmask)[0].tolist() == [int(v) for v in c["D"].split()]
    assert r.cm_order == [int(v) for v in c["order"].split()]
    D = dhat_all(lev)
    mtr = trace_strength(lev)
    for (i, j), v in _pairs(c.get("mu_s", "0-1 nan")).items():
        if not np.isnan(v):
            assert mu_s(lev, i, j, mtr) == pytest.approx(v, rel=1e-12)
    if "mu_b" in c:
        for (i, j), v in _pairs(c["mu_b"]).items():
            assert mu_b(lev, i, j, D) == pytest.approx(v, rel=1e-12)
    if "mu_D" in c:
        i, v = c["mu_D"].split()
        assert mu_D(lev, int(i), D) == pytest.approx(float(v), rel=1e-12)
    if "mu_g" in c:
        *mem, v = c["mu_g"].split()
        assert mu_g(lev, [int(t) for t in mem], D) == pytest.approx(float(v), rel=1e-12)
    if "mu_g_bound" in c:
        *mem, v = c["mu_g_bound"].split()
        g = mu_g(lev, [int(t) for t in mem], D)
        assert 0.0 < g <= float(v)
