"""GPU kernels of the edge-scoring network against the oracle network (oracle/gnn.py).

The oracle computes in float64 with the same bfloat16-rounded weights; the GPU sums in FP32.
Bars: logits within 2e-5 relative to the largest logit (sums of <= 141 FP32 products per unit);
gradients within 1e-4 of the largest gradient entry of their array (FP32 sums over all pairs);
the loss within 1e-5 relative.  Also: bitwise reproducibility, and Adam training on the GPU
lowering the loss of a learnable labelling.
"""
import numpy as np
import pytest

import paper_2011_13325_amd as E
from oracle import gnn

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _graph(seed, n=40, m=150):
    rng = np.random.default_rng(seed)
    pairs = set()
    while len(pairs) < m:
        a, b = rng.integers(0, n, 2)
        if a != b:
            pairs.add((min(a, b), max(a, b)))
    edges = np.array(sorted(pairs), dtype=np.int32)
    X = rng.standard_normal((m, gnn.F)).astype(np.float32)
    y = ((X[:, 0] + 0.5 * X[:, 3] - 0.3 * X[:, 7]) > 0).astype(np.float32)
    w = rng.uniform(0.2, 1.0, m).astype(np.float32)
    w[::7] = 0.0                          # unlabelled pairs still pass messages
    return X, edges, n, y, w


def _pack(p):
    return np.concatenate([np.asarray(p[k], dtype=np.float64).ravel() for k in gnn.PARAM_SHAPES]).astype(np.float32)


def _unpack(v):
    out, o = {}, 0
    for k, shp in gnn.PARAM_SHAPES.items():
        sz = int(np.prod(shp))
        out[k] = np.asarray(v[o:o + sz], dtype=np.float64).reshape(shp)
        o += sz
    return out


def test_forward_and_gradients_match_oracle():
    X, edges, n, y, w = _graph(0)
    p = gnn.init_params(3)
    rng = np.random.default_rng(5)
    for k in p:
        if k.startswith("b"):
            p[k] = 0.05 * rng.standard_normal(p[k].shape)
    flat = _pack(p)
    assert flat.size == E.GNN_PARAMS
    p32 = _unpack(flat)                   # the float32 masters both sides use
    net = E.EdgeNet(flat)
    z = net.forward(X, edges, n)
    zo, _ = gnn.forward(p32, X.astype(np.float64), edges, n)
    assert np.abs(z - zo).max() <= 2e-5 * np.abs(zo).max()
    loss, g = net.loss_grad(X, edges, n, y, w)
    lo, go, _ = gnn.loss_and_grads(p32, X.astype(np.float64), edges, n, y, weight=w)
    assert abs(loss - lo) <= 1e-5 * abs(lo)
    gg = _unpack(g)
    for k in gnn.PARAM_SHAPES:
        scale = np.abs(go[k]).max()
        err = np.abs(gg[k] - go[k]).max()
        print(f"[gnn] grad {k}: max err {err:.2e} of {scale:.2e}", flush=True)
        assert err <= 1e-4 * scale + 1e-9, k
    loss2, g2 = net.loss_grad(X, edges, n, y, w)
    assert loss2 == loss and np.array_equal(g2, g)
    net.close()


def test_training_lowers_the_loss():
    graphs = [_graph(s) for s in (11, 12, 13)]
    net = E.EdgeNet(seed=7)
    l0 = np.mean([net.loss_grad(*g)[0] for g in graphs])
    hist = net.train(graphs, epochs=150, lr=3e-3)
    l1 = np.mean([net.loss_grad(*g)[0] for g in graphs])
    print(f"[gnn] loss {l0:.4f} -> {l1:.4f} (epoch losses {hist[0]:.4f} .. {hist[-1]:.4f})", flush=True)
    assert np.all(np.isfinite(hist)) and l1 < 0.5 * l0
    # accuracy on a held-out graph of the same labelling
    X, edges, n, y, w = _graph(99)
    acc = np.mean((net.forward(X, edges, n) > 0) == (y > 0))
    assert acc > 0.8, acc
    net.close()


def test_bad_graphs_are_rejected():
    net = E.EdgeNet(seed=1)
    X, edges, n, y, w = _graph(0)
    bad = edges.copy()
    bad[3] = [5, 5]
    with pytest.raises(E.EamgError) as ei:
        net.forward(X, bad, n)
    assert ei.value.status == E.EAMG_ERR_INVALID_ARG
    Xn = X.copy()
    Xn[2, 2] = np.nan
    with pytest.raises(E.EamgError):
        net.forward(Xn, edges, n)
    net.close()
