"""GPU parity of the surrogate-network entry points and of the network's
forward and gradient against the FP64 oracle; the autograd wrapper; the
over-relaxed Richardson-Lucy start; training gain; monitor and fallback."""
import os
import sys

import numpy as np
import pytest
import torch

from aprgen.apr_input import (CONFIGS, SphereConfig, deconv_config, deconv_psf, deconv_set, gaussian_stencil,
                              random_apr, sphere_apr)
from oracle import access as A
from oracle import conv as C
from oracle import surrogate as S
from oracle.rl import richardson_lucy as oracle_rl
from paper_2112_03592_amd import apr as G
from paper_2112_03592_amd import surrogate as N
from tests.gpu_common import linear_access

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True, file=sys.stderr)


def dev(x):
    return torch.from_numpy(np.ascontiguousarray(x, dtype=np.float32)).cuda()


# ---------------------------------------------------------------------------
# the small entry points
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("n", [0, 1, 1000, 300001])
@pytest.mark.parametrize("log", [False, True])
def test_moments(n, log):
    rng = np.random.default_rng(n)
    u = rng.uniform(0.2, 900.0, n).astype(np.float32)
    ws = G.Workspace(16)
    st = G.moments(dev(u), log, ws).cpu().numpy()
    ref = S.moments(u.astype(np.float64), log)
    assert np.allclose(st, ref, rtol=1e-12, atol=1e-300)


@pytest.mark.parametrize("op", range(8))
def test_pointwise_ops(op):
    rng = np.random.default_rng(op)
    n = 70001
    a = rng.uniform(0.5, 900.0, n).astype(np.float32) if op in (0, 1, 2, 4, 5) else \
        rng.normal(size=n).astype(np.float32) * 0.3
    b = rng.uniform(0.5, 900.0, n).astype(np.float32)
    st = (5.1, 1.7)
    ref = S.pointwise(op, a.astype(np.float64), b.astype(np.float64), st)
    got = G.pointwise(op, dev(a), dev(b), torch.tensor(st, dtype=torch.float64, device="cuda")).cpu().numpy()
    assert np.allclose(got, ref, rtol=2e-7, atol=1e-30)


@pytest.mark.parametrize("rows,c,relu", [(0, 16, True), (1, 1, False), (5000, 16, True), (70001, 16, False),
                                         (3333, 3, True)])
def test_relu_bias_grad(rows, c, relu):
    rng = np.random.default_rng(rows + c)
    y = np.maximum(rng.normal(size=(rows, c)), 0).astype(np.float32)
    dy = rng.normal(size=(rows, c)).astype(np.float32)
    ws = G.Workspace(16)
    dpre, db = G.relu_bias_grad(dev(y), dev(dy), relu, ws)
    ref = dy * (y > 0) if relu else dy
    assert np.array_equal(dpre.cpu().numpy(), ref)
    assert np.allclose(db.cpu().numpy(), ref.astype(np.float64).sum(axis=0), rtol=1e-6, atol=1e-6)


@pytest.mark.parametrize("n", [1, 999, 200001])
def test_rel_l2_and_gradient(n):
    rng = np.random.default_rng(n)
    a = rng.normal(size=n).astype(np.float32)
    b = rng.normal(size=n).astype(np.float32)
    ws = G.Workspace(16)
    out, g = G.rel_l2(dev(a), dev(b), ws, grad=True, grad_scale=0.5)
    out = out.cpu().numpy()
    a64, b64 = a.astype(np.float64), b.astype(np.float64)
    assert np.isclose(out[0], S.rel_l2_sq(a64, b64), rtol=1e-12)
    assert np.isclose(out[1], (b64 * b64).sum(), rtol=1e-12)
    assert np.allclose(g.cpu().numpy(), 0.5 * 2 * (a64 - b64) / (b64 * b64).sum(), rtol=2e-7, atol=1e-30)


def test_adam_three_steps():
    rng = np.random.default_rng(3)
    n = 4097
    p = rng.normal(size=n).astype(np.float32)
    pd, md, vd = dev(p), torch.zeros(n, device="cuda"), torch.zeros(n, device="cuda")
    P, M, V = p.astype(np.float64), np.zeros(n), np.zeros(n)
    for step in (1, 2, 3):
        g = rng.normal(size=n).astype(np.float32)
        G.adam(pd, dev(g), md, vd, step, lr=1e-2)
        P, M, V = S.adam_step(P, g.astype(np.float64), M, V, step, lr=1e-2)
    assert np.allclose(pd.cpu().numpy(), P, rtol=1e-5, atol=1e-6)
    assert np.allclose(md.cpu().numpy(), M, rtol=1e-5, atol=1e-7)


@pytest.mark.parametrize("l_min,l_max,n_sets", [(2, 6, 4), (0, 9, 3), (5, 5, 4), (1, 3, 1)])
def test_level_weights_expand_and_fold(l_min, l_max, n_sets):
    rng = np.random.default_rng(l_max)
    P = rng.normal(size=(n_sets, 16, 16, 3, 3, 3)).astype(np.float32)
    E = G.level_weights(dev(P), l_min, l_max).cpu().numpy()
    assert np.array_equal(E, S.expand_sets(P, l_min, l_max).astype(np.float32))
    Q = rng.normal(size=E.shape).astype(np.float32)
    F = G.fold_level_weights(dev(Q), n_sets, l_min, l_max).cpu().numpy()
    assert np.allclose(F, S.fold_sets(Q.astype(np.float64), n_sets, l_min, l_max), rtol=1e-6, atol=1e-6)


# ---------------------------------------------------------------------------
# over-relaxed Richardson-Lucy from an initial estimate
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("power", [1.0, 2.1])
def test_rl_power_and_init(power):
    inp = sphere_apr(SphereConfig((32, 32, 32), 3, 3.0, 6.0, 1, 4100, psf_sigma=1.5))
    la = linear_access(inp)
    psf = gaussian_stencil(5, 1.5)
    u = inp.values.astype(np.float64)
    init = u * np.random.default_rng(1).uniform(0.9, 1.1, u.size)
    ref = oracle_rl(la, u, psf, 3, init=init.astype(np.float32).astype(np.float64), power=power)
    with G.AprAccess.from_input(inp) as acc:
        got = G.richardson_lucy(acc, dev(u), psf, 3, init=dev(init), power=power).cpu().numpy()
    rel = np.abs(got - ref) / np.abs(ref)
    assert rel.max() < 1e-4, rel.max()


# ---------------------------------------------------------------------------
# the network against the oracle
# ---------------------------------------------------------------------------

NET_CASES = {
    "sphere32": lambda: sphere_apr(CONFIGS["sphere32"]),
    "rand33x20x70": lambda: random_apr((33, 20, 70), l_min=2, seed=5, p_refine=0.2),
    "blur48": lambda: sphere_apr(SphereConfig((48, 48, 48), 6, 4.0, 10.0, 2, 4200, psf_sigma=1.5)),
}


def _oracle_params(net):
    return S.Params([w.cpu().numpy().astype(np.float64) for w in net.W],
                    [b.cpu().numpy().astype(np.float64) for b in net.b])


@pytest.mark.parametrize("name", list(NET_CASES))
@pytest.mark.parametrize("mode", [N.ADDITIVE, N.MULTIPLICATIVE])
def test_network_forward_and_gradient(name, mode):
    say("net", name, mode)
    inp = NET_CASES[name]()
    la = linear_access(inp)
    tr = A.tree_structure(la)
    rng = np.random.default_rng(7)
    u = np.maximum(inp.values.astype(np.float64), 1.0)
    t = (u * rng.uniform(0.8, 1.25, u.size)).astype(np.float32)
    net = N.SurrogateNet(N.NetConfig(channels=16, layers=4, n_sets=3, mode=mode, seed=3, last_scale=1.0))
    for b in net.b:     # non-zero biases exercise the bias path
        b.copy_(dev(rng.normal(size=b.numel()) * 0.1))
    net._version += 1
    P = _oracle_params(net)
    u32 = u.astype(np.float32)
    s_ref, _ = S.forward(la, u32.astype(np.float64), P, mode, tree=tr)
    loss_ref, gW_ref, gb_ref = S.loss_and_grad(la, u32.astype(np.float64), t.astype(np.float64), P, mode, tree=tr)
    with G.AprAccess.from_input(inp, gather=(3,)) as acc:
        s, _ = net.forward(acc, dev(u32))
        out, grads = net.loss_and_grad(acc, dev(u32), dev(t))
        s = s.cpu().numpy()
        loss = float(out[0].item())
        grads = [g.cpu().numpy() for g in grads]
    # additive outputs may cross zero: bound each element against |s| plus a
    # tenth of the RMS of s
    err = np.abs(s - s_ref) / (np.abs(s_ref) + 0.1 * np.sqrt(np.mean(s_ref ** 2)))
    assert np.linalg.norm(s - s_ref) <= 1e-5 * np.linalg.norm(s_ref), np.linalg.norm(s - s_ref) / np.linalg.norm(s_ref)
    assert err.max() < 1e-4, err.max()
    assert abs(loss - loss_ref) <= 1e-4 * loss_ref
    for g, r, what in zip(grads, gW_ref + gb_ref, [f"W{i}" for i in range(4)] + [f"b{i}" for i in range(4)]):
        rel = np.linalg.norm(g - r) / max(np.linalg.norm(r), 1e-30)
        assert rel < 1e-4, (what, rel)


def test_bf16_activations_forward_close_to_oracle():
    inp = NET_CASES["blur48"]()
    la = linear_access(inp)
    u = np.maximum(inp.values, 1.0).astype(np.float32)
    net = N.SurrogateNet(N.NetConfig(channels=16, layers=4, n_sets=3, seed=4, last_scale=1.0))
    s_ref, _ = S.forward(la, u.astype(np.float64), _oracle_params(net), N.MULTIPLICATIVE)
    with G.AprAccess.from_input(inp, gather=(3,)) as acc:
        s, _ = net.forward(acc, dev(u), act_dtype=torch.bfloat16)
        s = s.cpu().numpy()
    assert np.linalg.norm(s - s_ref) <= 2e-2 * np.linalg.norm(s_ref)


@pytest.mark.parametrize("relu", [False, True])
def test_autograd_function_matches_oracle(relu):
    inp = sphere_apr(CONFIGS["sphere32"])
    la = linear_access(inp)
    tr = A.tree_structure(la)
    rng = np.random.default_rng(2)
    nl = la.l_max - la.l_min + 1
    x = rng.normal(size=(la.n, 16)).astype(np.float32)
    W = rng.normal(size=(nl, 16, 16, 3, 3, 3)).astype(np.float32) * 0.1
    b = rng.normal(size=16).astype(np.float32)
    g = rng.normal(size=(la.n, 16)).astype(np.float32)
    pre = C.apr_conv(la, x.astype(np.float64), W.astype(np.float64), bias=b.astype(np.float64), tree=tr)
    dpre = g.astype(np.float64) * (pre > 0) if relu else g.astype(np.float64)
    ref_dx = C.apr_conv_bwd_data(la, dpre, W.astype(np.float64), tree=tr)
    ref_dw = C.apr_conv_bwd_weight(la, x.astype(np.float64), dpre, 3, tree=tr)
    with G.AprAccess.from_input(inp, gather=(3,)) as acc:
        xd, wd, bd = dev(x).requires_grad_(), dev(W).requires_grad_(), dev(b).requires_grad_()
        y = N.apr_conv_layer(acc, xd, wd, bd, 3, relu=relu)
        y.backward(dev(g))
        dx, dw, db = xd.grad.cpu().numpy(), wd.grad.cpu().numpy(), bd.grad.cpu().numpy()
        yv = y.detach().cpu().numpy()
    assert np.linalg.norm(yv - (np.maximum(pre, 0) if relu else pre)) <= 1e-5 * np.linalg.norm(pre)
    for got, ref in ((dx, ref_dx), (dw, ref_dw), (db, dpre.sum(axis=0))):
        assert np.linalg.norm(got - ref) <= 1e-5 * np.linalg.norm(ref)


# ---------------------------------------------------------------------------
# monitor and fallback
# ---------------------------------------------------------------------------

def test_monitor_and_fallback_paths():
    inp = NET_CASES["blur48"]()
    psf = gaussian_stencil(5, 1.5)
    u = dev(np.maximum(inp.values, 0.0))
    net = N.SurrogateNet(N.NetConfig(seed=5))
    with G.AprAccess.from_input(inp, gather=(3,)) as acc:
        sur = N.RLSurrogate(net, psf, n_iter=10, n_pre=4, power=2.0, tau=0.0)
        plain = G.richardson_lucy(acc, u, psf, 10).cpu().numpy()
        r0 = sur(acc, u)
        assert r0.fallback and np.array_equal(r0.values.cpu().numpy(), plain)
        sur.tau = float("inf")
        s, out = sur.estimate(acc, u)
        s = s.cpu().numpy()
        m_ref = float(np.sqrt(out[0].item()))
        r1 = sur(acc, u)
        assert not r1.fallback and np.array_equal(r1.values.cpu().numpy(), s)
        assert r1.monitor == m_ref and 0.0 < m_ref < 1.0
        # the monitor is the relative change of one plain step started at s
        r = G.richardson_lucy(acc, u, psf, 1, init=dev(s)).cpu().numpy().astype(np.float64)
        assert np.isclose(m_ref, np.linalg.norm(r - s) / np.linalg.norm(s), rtol=1e-5)



# ---------------------------------------------------------------------------
# the trained surrogate (weights written by train_surrogate on the GPU)
# ---------------------------------------------------------------------------

TRAINED = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "paper_2112_03592_amd",
                       "weights", "rl10_surrogate.npz")


@pytest.mark.parametrize("edge,seed", [(96, 8001), (112, 8003), (128, 8002)])
def test_trained_surrogate_against_fp64_oracle_rl10(edge, seed):
    """Held-out deconvolution APR against the FP64 oracle's 10 Richardson-Lucy
    iterations: the trained network's estimate gains over its start (the
    over-relaxed iterations alone, at least 2x), over the same network
    untrained, and over the input (at least 6x on these small two-to-four
    sphere APRs); an estimate the monitor accepts is within 2e-2, so what the
    surrogate returns (the estimate, else the plain iteration) always is."""
    say("trained", edge, seed)
    inp = sphere_apr(deconv_config(edge, seed))
    la = linear_access(inp)
    psf = deconv_psf()
    u = np.maximum(inp.values, 0).astype(np.float32)
    t = oracle_rl(la, u.astype(np.float64), psf, 10)
    sur = N.load_surrogate(TRAINED)
    fresh = N.RLSurrogate(N.SurrogateNet(N.NetConfig(layers=sur.net.cfg.layers, seed=7)), psf, 10, sur.n_pre, sur.power)
    with G.AprAccess.from_input(inp, gather=(3,)) as acc:
        ud = dev(u)
        est, mon = sur.estimate(acc, ud)
        est = est.cpu().numpy().astype(np.float64)
        m = float(np.sqrt(mon[0].item()))
        res = sur(acc, ud)
        got = res.values.cpu().numpy().astype(np.float64)
        base = sur.base(acc, ud).cpu().numpy().astype(np.float64)
        s_fresh = fresh.estimate(acc, ud)[0].cpu().numpy().astype(np.float64)
        plain = sur.plain(acc, ud).cpu().numpy().astype(np.float64)

    def err(a):
        return float(np.linalg.norm(a - t) / np.linalg.norm(t))

    say(f"  error: estimate {err(est):.4f} returned {err(got):.4f} start {err(base):.4f} untrained "
        f"{err(s_fresh):.4f} input {err(u):.4f} plain FP32 {err(plain):.2e}; monitor {m:.4f} tau {sur.tau:.4f} "
        f"fallback {res.fallback}")
    assert err(plain) < 1e-4
    assert err(est) < 0.5 * err(base)
    assert err(est) < 0.5 * err(s_fresh)
    assert err(est) < 0.15 * err(u)
    assert res.monitor == m and res.fallback == (m > sur.tau)
    if not res.fallback:
        assert err(est) <= 2e-2
    assert err(got) <= 2e-2
    assert np.array_equal(got, plain if res.fallback else est)


GOLDEN_RL10 = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "rl10_deconv256.npz")


def test_bench_size_surrogate_against_stored_oracle_rl10():
    """The first APR of the benchmark batch (256^3, seed 7000, 0.5M
    particles) against the FP64 oracle's RL10, stored by
    tests/golden/make_rl10_deconv256.py (a digest of the input guards the
    pairing): the device RL10 within 1e-4, the surrogate's returned values
    within 2e-2."""
    from aprgen.apr_input import input_digest
    gold = np.load(GOLDEN_RL10)
    inp = deconv_set([int(gold["edge"])], int(gold["seed"]))[0]
    assert str(gold["digest"]) == input_digest(inp), "stored oracle RL10 belongs to another input"
    t = gold["rl10"].astype(np.float64)
    u = np.maximum(inp.values, 0).astype(np.float32)
    sur = N.load_surrogate(TRAINED)
    with G.AprAccess.from_input(inp, gather=(3,)) as acc:
        ud = dev(u)
        plain = G.richardson_lucy(acc, ud, deconv_psf(), 10).cpu().numpy().astype(np.float64)
        res = sur(acc, ud)
        got = res.values.cpu().numpy().astype(np.float64)

    def err(a):
        return float(np.linalg.norm(a - t) / np.linalg.norm(t))

    say(f"  256^3: plain FP32 {err(plain):.2e}, surrogate {err(got):.4f} (monitor {res.monitor:.4f}, "
        f"fallback {res.fallback})")
    assert err(plain) < 1e-4
    assert err(got) <= 2e-2


def test_short_training_reduces_the_loss():
    rl = N.RichardsonLucy(deconv_psf())
    cases = []
    for inp in deconv_set((64, 80), 8100):
        acc = G.AprAccess.from_input(inp, gather=(3,))
        u = dev(np.maximum(inp.values, 0))
        cases.append((acc, rl(acc, u, 4, power=2.0), rl(acc, u, 10)))
    net = N.SurrogateNet(N.NetConfig(seed=11))
    losses = N.train(net, cases, 80, lr=2e-3, log_every=1)
    for acc, _, _ in cases:
        acc.close()
    assert np.mean(losses[-10:]) < 0.7 * np.mean(losses[:2]), (losses[:2], losses[-10:])
