"""The hand-worked matching fixture (tests/golden/pwagg_path4.txt, Algorithm alg:pwagg) through
the C ABI: the four-vertex path as a scalar problem whose matrix gives exactly the fixture's
weights (edge weights |A_ij|, vertex weights the diagonal excess over the off-diagonal sum), set
up by the library with one coarsening step; its level-0 agglomerates must be the fixture's.
Only the cases with a positive vertex weight give a nonsingular matrix; with every vertex weight
zero the matrix is the singular path Laplacian, whose coarsest level the library rejects as not
positive definite (the regularization of the coarsest level removes the kernels of its diagonal
blocks only), so those cases stay oracle pins."""
import numpy as np
import pytest

import paper_2011_13325_amd as E

from test_oracle_golden import CASES

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


def _problem(M):
    # weighted path Laplacian (weights 1, 2, 1) plus the vertex weights on the diagonal
    A = np.array([[1, -1, 0, 0], [-1, 3, -2, 0], [0, -2, 3, -1], [0, 0, -1, 1]], dtype=np.float64)
    A += np.diag(M)
    rp, col, val = [0], [], []
    for i in range(4):
        for j in range(4):
            if A[i, j] != 0.0:
                col.append(j)
                val.append(A[i, j])
        rp.append(len(col))
    coords = np.zeros((4, 3))
    coords[:, 0] = np.arange(4)
    return (coords, np.array(rp, np.int32), np.array(col, np.int32), np.array(val),
            np.zeros(4, np.uint8))


SPD = [c for c in CASES if any(float(v) > 0.0 for v in c["M"].split())]


@pytest.mark.parametrize("c", SPD, ids=[c["case"] for c in SPD])
def test_library_matching_equals_hand_worked(c):
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    coords, rp, col, val, dirichlet = _problem([float(v) for v in c["M"].split()])
    prm = E.eamg_default_setup_params(sigma=float(c["sigma"]), rounds=int(c["rounds"]),
                                      coarsest_max_dofs=2, max_levels=2)
    print(f"\n[golden {c['case']}] sigma {c['sigma']} rounds {c['rounds']}", flush=True)
    h = E.Hierarchy(1, coords, rp, col, val, dirichlet, prm)
    try:
        assert h.stats()["n_levels"] == 2
        agg = E.eamg_export_level(h.h, 0)["agg"]
        want = np.full(4, -1)
        for I, grp in enumerate(c["aggregates"].split("|")):
            for v in grp.split():
                want[int(v)] = I
        assert agg.tolist() == want.tolist()
        assert sorted(np.nonzero(agg < 0)[0].tolist()) == [int(v) for v in c["D"].split()]
        b = torch.tensor([1.0, -2.0, 0.5, 3.0], dtype=torch.float64, device="cuda")
        x, info = h.solve(b, rtol=1e-10)
        assert info["status"] == E.EAMG_OK and info["rel_res_true"] <= 1e-10
    finally:
        h.close()
