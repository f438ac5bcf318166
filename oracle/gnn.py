"""Edge-scoring graph network for learned pairwise aggregation (oracle side).

TEST INFRASTRUCTURE ONLY (see the package docstring).  This module states, in plain NumPy and
float64, what the library's learned-coarsening kernels compute, so that their forward pass and
gradients can be checked element by element:

* ``edge_features``  the input of one candidate pair (i, j) of a matching pass, built from the
  quantities the coarsening criteria of the paper use: mu_s (Def. def:muc), the spectrum of the
  edge matrix E^{ij} (Def. def:deng), the traces of D-hat_i = M^i + sum of pulled edge matrices
  (the vertex form of eq. auxa) and of M^i, and the aggregate sizes (Algorithm alg:pwagg).
* ``forward`` / ``loss_and_grads``  a three-layer edge network: an edge layer, one round of
  mean message passing over the candidate-edge graph, and a linear read-out giving the logit of
  "the exact criterion accepts this pair".  Weights are rounded to bfloat16 for use (the masters
  stay float); all sums are float.  The loss is the mean binary cross-entropy on logits.
* ``bf16_round``  round-to-nearest-even to bfloat16, from the definition of the format (keep the
  top 16 bits of the IEEE float32 pattern).

The network and its use are this build's additions to the method (the paper has no learned
part); the exact criterion still decides every pair that is formed.
"""
import numpy as np

F = 12          # input features per candidate pair
H = 64          # hidden width
PARAM_SHAPES = {"W1": (H, F), "b1": (H,), "W2a": (H, H), "W2b": (H, H), "b2": (H,), "w3": (H,),
                "b3": (1,)}
BF16_PARAMS = ("W1", "W2a", "W2b", "w3")   # weights used in bfloat16; biases stay float


def bf16_round(x):
    """float32 -> nearest bfloat16 (ties to even), returned as float32."""
    a = np.ascontiguousarray(np.asarray(x, dtype=np.float32))
    u = a.view(np.uint32).astype(np.uint64)
    lsb = (u >> 16) & 1
    r = ((u + 0x7FFF + lsb) >> 16) << 16
    out = r.astype(np.uint32).view(np.float32).reshape(a.shape)
    nan = np.isnan(a)
    if nan.any():
        out = np.where(nan, a, out)
    return out


def init_params(seed=0):
    """He-uniform weights, zero biases (float64 masters)."""
    rng = np.random.default_rng(seed)
    p = {}
    for name, shape in PARAM_SHAPES.items():
        if name.startswith("b"):
            p[name] = np.zeros(shape)
        else:
            fan_in = shape[-1] if len(shape) == 2 else H
            lim = np.sqrt(6.0 / fan_in)
            p[name] = rng.uniform(-lim, lim, size=shape)
    return p


def used_params(p, round_bf16=True):
    """The values the network computes with: bfloat16-rounded weights, float biases."""
    q = {}
    for k, v in p.items():
        q[k] = bf16_round(v).astype(np.float64) if (round_bf16 and k in BF16_PARAMS) else np.asarray(v, dtype=np.float64)
    return q


def edge_features(E_ij, Dhat_i, Dhat_j, M_i, M_j, mtr_i, mtr_j, nmem_i, nmem_j):
    """Features of candidate pair (i, j); symmetric in (i, j).

    E_ij, Dhat_*, M_*: k x k matrices (k = 6 elasticity, 1 scalar); mtr_*: the trace strengths
    max(tr M, max_e tr E) used by mu_s; nmem_*: members of the current aggregates."""
    k = E_ij.shape[0]
    t = np.trace(E_ij)
    f = np.zeros(F)
    f[0] = np.log(np.sqrt(mtr_i * mtr_j) / t)              # log mu_s
    ev = np.sort(np.linalg.eigvalsh(0.5 * (E_ij + E_ij.T)))[::-1] / t
    f[1:1 + min(k, 6)] = ev[:6]
    di, dj = np.trace(Dhat_i), np.trace(Dhat_j)
    f[7] = np.log(min(di, dj) / t)
    f[8] = np.log(max(di, dj) / t)
    f[9] = np.log1p(np.trace(M_i) / di + np.trace(M_j) / dj)
    f[10] = (nmem_i + nmem_j) / 4.0
    f[11] = abs(np.log(mtr_i / mtr_j))
    return f


def _incidence(edges, n_nodes):
    deg = np.zeros(n_nodes)
    np.add.at(deg, edges[:, 0], 1.0)
    np.add.at(deg, edges[:, 1], 1.0)
    return deg


def forward(p, X, edges, n_nodes, round_bf16=True):
    """Logits of the m candidate pairs.  X: (m, F); edges: (m, 2) node ids.  Returns (z, cache)."""
    q = used_params(p, round_bf16)
    X = np.asarray(X, dtype=np.float64)
    edges = np.asarray(edges, dtype=np.int64)
    a1 = X @ q["W1"].T + q["b1"]
    h1 = np.maximum(a1, 0.0)
    deg = _incidence(edges, n_nodes)
    msum = np.zeros((n_nodes, H))
    np.add.at(msum, edges[:, 0], h1)
    np.add.at(msum, edges[:, 1], h1)
    m = msum / np.maximum(deg, 1.0)[:, None]
    s = m[edges[:, 0]] + m[edges[:, 1]]
    a2 = h1 @ q["W2a"].T + s @ q["W2b"].T + q["b2"]
    h2 = np.maximum(a2, 0.0)
    z = h2 @ q["w3"] + q["b3"][0]
    return z, dict(q=q, X=X, edges=edges, a1=a1, h1=h1, deg=deg, s=s, a2=a2, h2=h2)


def loss_and_grads(p, X, edges, n_nodes, y, weight=None, round_bf16=True):
    """Mean binary cross-entropy of the logits against labels y in {0, 1} (optionally weighted
    per pair), and its gradients with respect to the parameters used (the same arrays serve as
    gradients of the float masters under the straight-through reading of the rounding)."""
    z, c = forward(p, X, edges, n_nodes, round_bf16)
    y = np.asarray(y, dtype=np.float64)
    w = np.ones_like(z) if weight is None else np.asarray(weight, dtype=np.float64)
    wsum = w.sum()
    loss = float(np.sum(w * (np.logaddexp(0.0, z) - y * z)) / wsum)
    q = c["q"]
    dz = w * (1.0 / (1.0 + np.exp(-z)) - y) / wsum
    g = {"w3": c["h2"].T @ dz, "b3": np.array([dz.sum()])}
    da2 = np.outer(dz, q["w3"]) * (c["a2"] > 0.0)
    g["W2a"] = da2.T @ c["h1"]
    g["W2b"] = da2.T @ c["s"]
    g["b2"] = da2.sum(axis=0)
    dh1 = da2 @ q["W2a"]
    ds = da2 @ q["W2b"]                       # d loss / d s_e, s_e = m_u + m_v
    e = c["edges"]
    dm = np.zeros((n_nodes, H))
    np.add.at(dm, e[:, 0], ds)
    np.add.at(dm, e[:, 1], ds)
    dm /= np.maximum(c["deg"], 1.0)[:, None]   # m_i = sum / deg_i
    dh1 = dh1 + dm[e[:, 0]] + dm[e[:, 1]]
    da1 = dh1 * (c["a1"] > 0.0)
    g["W1"] = da1.T @ c["X"]
    g["b1"] = da1.sum(axis=0)
    return loss, g, z
