"""A small APR-native convolutional network and its training step, in FP64.
Test infrastructure only.

Section 7 suggests CNNs whose layers are APR convolutions, with per-level
filters learned by back-propagating through the interpolation across
resolution levels.  The paper fixes no architecture, loss or optimiser; the
readings used here (all parity unpinned by the paper, pinned below by
finite differences and closed forms in the tests):

* input statistics (mu, sd) of u (additive mode) or of log(max(u, 1))
  (multiplicative mode), population standard deviation, 1 when zero;
* layers h_{i+1} = ReLU(conv_i(h_i) + b_i), the last one without ReLU,
  h_0 = (u - mu)/sd or (log u+ - mu)/sd, u+ = max(u, 1);
* output s = u + sd * h_L (additive) or s = u * exp(sd * h_L) (multiplicative);
* per-level weights from weight sets indexed by the distance l_max - l to the
  finest level, levels coarser than the last set sharing it;
* loss = |s - t|^2 / |t|^2 (squared relative L2 over particles);
* Adam with bias correction.
"""
from __future__ import annotations

from typing import List, Optional, Sequence, Tuple

import numpy as np

from .access import LinearAccess, tree_structure
from .conv import apr_conv, apr_conv_bwd_data, apr_conv_bwd_weight

ADDITIVE, MULTIPLICATIVE = "add", "mul"


def moments(u, log: bool = False) -> Tuple[float, float]:
    v = np.asarray(u, np.float64)
    if log:
        v = np.log(np.maximum(v, 1.0))
    if v.size == 0:
        return 0.0, 1.0
    mu = float(v.sum() / v.size)
    var = max(float((v * v).sum() / v.size - mu * mu), 0.0)
    return mu, (float(np.sqrt(var)) if var > 0.0 else 1.0)


def _logp(a):
    return np.log(np.maximum(np.asarray(a, np.float64), 1.0))


def pointwise(op: int, a, b, stats) -> np.ndarray:
    """The elementwise maps between particle values and network space."""
    mu, sd = stats
    a = np.asarray(a, np.float64)
    b = None if b is None else np.asarray(b, np.float64)
    return {
        0: lambda: (a - mu) / sd,
        1: lambda: (a - b) / sd,
        2: lambda: b + sd * a,
        3: lambda: sd * a,
        4: lambda: (_logp(a) - mu) / sd,
        5: lambda: (_logp(a) - _logp(b)) / sd,
        6: lambda: b * np.exp(sd * a),
        7: lambda: sd * a * b,
    }[op]()


def set_of_level(l: int, l_max: int, n_sets: int) -> int:
    return min(l_max - l, n_sets - 1)


def expand_sets(P, l_min: int, l_max: int) -> np.ndarray:
    """[n_sets, ...] -> [l_max - l_min + 1, ...]."""
    P = np.asarray(P, np.float64)
    return np.stack([P[set_of_level(l, l_max, P.shape[0])] for l in range(l_min, l_max + 1)])


def fold_sets(G, n_sets: int, l_min: int, l_max: int) -> np.ndarray:
    """Adjoint of expand_sets: sum the per-level rows of each set."""
    G = np.asarray(G, np.float64)
    out = np.zeros((n_sets,) + G.shape[1:])
    for l in range(l_min, l_max + 1):
        out[set_of_level(l, l_max, n_sets)] += G[l - l_min]
    return out


def rel_l2_sq(a, b) -> float:
    a = np.asarray(a, np.float64)
    b = np.asarray(b, np.float64)
    q = float((b * b).sum())
    d = float(((a - b) ** 2).sum())
    return d / q if q > 0 else d


def adam_step(p, g, m, v, step: int, lr: float, b1: float = 0.9, b2: float = 0.999, eps: float = 1e-8):
    """Returns the updated (p, m, v)."""
    g = np.asarray(g, np.float64)
    m = b1 * np.asarray(m, np.float64) + (1 - b1) * g
    v = b2 * np.asarray(v, np.float64) + (1 - b2) * g * g
    mh = m / (1 - b1 ** step)
    vh = v / (1 - b2 ** step)
    return np.asarray(p, np.float64) - lr * mh / (np.sqrt(vh) + eps), m, v


class Params:
    """Per-layer weight sets W_i [n_sets, c_out, c_in, k, k, k] and biases b_i [c_out]."""

    def __init__(self, weights: Sequence[np.ndarray], biases: Sequence[np.ndarray]):
        self.weights = [np.asarray(w, np.float64) for w in weights]
        self.biases = [np.asarray(b, np.float64) for b in biases]

    @property
    def k(self) -> int:
        return self.weights[0].shape[-1]


def forward(apr: LinearAccess, u, params: Params, mode: str = ADDITIVE,
            tree: Optional[LinearAccess] = None):
    """Returns (s, cache) with cache = (stats, inputs of every layer, outputs)."""
    tree = tree_structure(apr) if tree is None else tree
    u = np.asarray(u, np.float64)
    log = mode == MULTIPLICATIVE
    stats = moments(u, log)
    h = pointwise(4 if log else 0, u, None, stats)[:, None]
    ins: List[np.ndarray] = []
    outs: List[np.ndarray] = []
    L = len(params.weights)
    for i, (Wset, b) in enumerate(zip(params.weights, params.biases)):
        W = expand_sets(Wset, apr.l_min, apr.l_max)
        ins.append(h)
        y = apr_conv(apr, h, W, bias=b, tree=tree)
        if i < L - 1:
            y = np.maximum(y, 0.0)
        outs.append(y)
        h = y
    net = h[:, 0]
    s = pointwise(6 if log else 2, net, u, stats)
    return s, (stats, ins, outs)


def loss_and_grad(apr: LinearAccess, u, t, params: Params, mode: str = ADDITIVE,
                  tree: Optional[LinearAccess] = None):
    """Loss |s - t|^2/|t|^2 and its gradient with respect to every weight
    set and bias, by reverse-mode differentiation of ``forward`` written out
    layer by layer with the adjoint convolutions."""
    tree = tree_structure(apr) if tree is None else tree
    t = np.asarray(t, np.float64)
    s, (stats, ins, outs) = forward(apr, u, params, mode, tree)
    loss = rel_l2_sq(s, t)
    q = float((t * t).sum())
    ds = 2.0 * (s - t) / (q if q > 0 else 1.0)
    # ds/dnet: sd (additive) or sd * s (multiplicative)
    g = pointwise(7 if mode == MULTIPLICATIVE else 3, ds, s, stats)[:, None]
    L = len(params.weights)
    gW: List[np.ndarray] = [None] * L
    gb: List[np.ndarray] = [None] * L
    for i in range(L - 1, -1, -1):
        if i < L - 1:
            g = g * (outs[i] > 0)
        Wset = params.weights[i]
        k = Wset.shape[-1]
        gb[i] = g.sum(axis=0)
        dW = apr_conv_bwd_weight(apr, ins[i], g, k, tree=tree)
        gW[i] = fold_sets(dW, Wset.shape[0], apr.l_min, apr.l_max)
        if i > 0:
            g = apr_conv_bwd_data(apr, g, expand_sets(Wset, apr.l_min, apr.l_max), tree=tree)
    return loss, gW, gb
