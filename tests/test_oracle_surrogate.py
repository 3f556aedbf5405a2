"""Pins for the oracle's surrogate network pieces (CPU only): closed forms of
the statistics, maps, loss and optimiser step; the weight-set layout and its
adjoint; the network gradient against central finite differences."""
import numpy as np
import pytest

from aprgen.apr_input import random_apr
from oracle import access as A
from oracle import surrogate as S


def _la(inp):
    return A.LinearAccess(inp.dims, inp.l_min, inp.l_max, inp.y_idx, inp.xz_end)


def test_moments_closed_forms():
    assert S.moments(np.full(7, 3.5)) == (3.5, 1.0)            # zero spread -> sd 1
    assert S.moments(np.array([0.0, 2.0])) == (1.0, 1.0)
    mu, sd = S.moments(np.array([1.0, np.e ** 2]), log=True)  # logs 0 and 2
    assert np.isclose(mu, 1.0) and np.isclose(sd, 1.0)
    mu, sd = S.moments(np.array([0.25, np.e ** 2]), log=True)  # 0.25 clamps to 1
    assert np.isclose(mu, 1.0) and np.isclose(sd, 1.0)
    assert S.moments(np.zeros(0)) == (0.0, 1.0)


def test_pointwise_inverse_pairs():
    rng = np.random.default_rng(0)
    u = rng.uniform(1.0, 1000.0, 50)
    t = rng.uniform(1.0, 1000.0, 50)
    st = (0.3, 2.5)
    assert np.allclose(S.pointwise(2, S.pointwise(1, t, u, st), u, st), t)
    assert np.allclose(S.pointwise(6, S.pointwise(5, t, u, st), u, st), t)
    assert np.allclose(S.pointwise(0, u, None, st) * 2.5 + 0.3, u)
    assert np.allclose(S.pointwise(4, u, None, st) * 2.5 + 0.3, np.log(u))
    # op 7 is the derivative of op 6 in a, times the incoming gradient
    a = rng.normal(size=50) * 0.1
    h = 1e-6
    fd = (S.pointwise(6, a + h, u, st) - S.pointwise(6, a - h, u, st)) / (2 * h)
    assert np.allclose(S.pointwise(7, np.ones(50), S.pointwise(6, a, u, st), st), fd, rtol=1e-6)
    assert np.allclose(S.pointwise(3, np.ones(50), None, st), 2.5)


def test_level_sets_layout_and_adjoint():
    P = np.arange(3 * 2, dtype=float).reshape(3, 2)
    E = S.expand_sets(P, 2, 6)      # levels 2..6: distances 4 3 2 1 0
    assert E.tolist() == [P[2].tolist(), P[2].tolist(), P[2].tolist(), P[1].tolist(), P[0].tolist()]
    rng = np.random.default_rng(1)
    Q = rng.normal(size=E.shape)
    assert np.isclose((E * Q).sum(), (P * S.fold_sets(Q, 3, 2, 6)).sum())
    # one level and more sets than levels
    assert S.expand_sets(P, 4, 4).tolist() == [P[0].tolist()]


def test_rel_l2_and_adam_closed_forms():
    b = np.array([3.0, 4.0])
    assert S.rel_l2_sq(b, b) == 0.0
    assert S.rel_l2_sq(np.zeros(2), b) == 1.0
    assert S.rel_l2_sq(2 * b, b) == 1.0
    assert S.rel_l2_sq(b, np.zeros(2)) == 25.0
    # first Adam step: m_hat = g, v_hat = g^2, so p moves by lr * g / (|g| + eps)
    g = np.array([0.5, -2.0, 1e-3])
    p, m, v = S.adam_step(np.zeros(3), g, np.zeros(3), np.zeros(3), 1, lr=0.01, eps=0.0)
    assert np.allclose(p, -0.01 * np.sign(g))
    assert np.allclose(m, 0.1 * g) and np.allclose(v, 0.001 * g * g)
    # a constant gradient keeps the step at lr * sign(g) (bias correction exact)
    for step in range(2, 6):
        p, m, v = S.adam_step(p, g, m, v, step, lr=0.01, eps=0.0)
    assert np.allclose(p, -0.05 * np.sign(g))


def _params(rng, k, chans, n_sets, scale_last=1.0):
    W, B = [], []
    for i in range(len(chans) - 1):
        ci, co = chans[i], chans[i + 1]
        w = rng.normal(size=(n_sets, co, ci, k, k, k)) * np.sqrt(2.0 / (ci * k ** 3))
        if i == len(chans) - 2:
            w *= scale_last
        W.append(w)
        B.append(rng.normal(size=co) * 0.1)
    return S.Params(W, B)


@pytest.mark.parametrize("mode", [S.ADDITIVE, S.MULTIPLICATIVE])
def test_zero_last_layer_is_identity(mode):
    inp = random_apr((8, 8, 8), l_min=1, seed=3, p_refine=0.3)
    la = _la(inp)
    rng = np.random.default_rng(2)
    u = rng.uniform(50, 500, la.n)
    p = _params(rng, 3, [1, 4, 1], 2)
    p.weights[-1][:] = 0.0
    p.biases[-1][:] = 0.0
    s, _ = S.forward(la, u, p, mode)
    assert np.allclose(s, u, rtol=1e-14)


@pytest.mark.parametrize("mode", [S.ADDITIVE, S.MULTIPLICATIVE])
def test_network_gradient_matches_finite_differences(mode):
    inp = random_apr((6, 7, 5), l_min=1, seed=4, p_refine=0.35)
    la = _la(inp)
    tr = A.tree_structure(la)
    rng = np.random.default_rng(5)
    u = rng.uniform(50, 500, la.n)
    t = u * rng.uniform(0.8, 1.25, la.n)
    p = _params(rng, 3, [1, 3, 2, 1], 2, scale_last=0.3)
    loss, gW, gb = S.loss_and_grad(la, u, t, p, mode, tree=tr)
    h = 1e-6

    def f():
        s, _ = S.forward(la, u, p, mode, tree=tr)
        return S.rel_l2_sq(s, t)

    assert np.isclose(loss, f())
    checked = 0
    for i in range(len(p.weights)):
        flat = p.weights[i].reshape(-1)
        for j in rng.choice(flat.size, 6, replace=False):
            old = flat[j]
            flat[j] = old + h
            fp = f()
            flat[j] = old - h
            fm = f()
            flat[j] = old
            fd = (fp - fm) / (2 * h)
            assert abs(fd - gW[i].reshape(-1)[j]) <= 1e-5 * max(1e-3, abs(fd)), (i, j, fd, gW[i].reshape(-1)[j])
            checked += 1
        for j in range(p.biases[i].size):
            old = p.biases[i][j]
            p.biases[i][j] = old + h
            fp = f()
            p.biases[i][j] = old - h
            fm = f()
            p.biases[i][j] = old
            fd = (fp - fm) / (2 * h)
            assert abs(fd - gb[i][j]) <= 1e-5 * max(1e-3, abs(fd)), (i, j, fd, gb[i][j])
            checked += 1
    assert checked > 20
