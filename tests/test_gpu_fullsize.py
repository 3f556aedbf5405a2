"""The gather path at the benchmark's size (the 512^3 sphere field, 6.6M
particles): the 16 -> 16 layer on both matrix-core paths against the FP64
oracle on sampled particles, and both gradients through identities that hold
exactly at any size (the forward is linear in x and in W)."""
import sys

import numpy as np
import pytest
import torch

from aprgen.apr_input import cached_sphere_apr
from oracle import access as A
from oracle import conv as C
from oracle.tree import fill_tree as oracle_fill
from paper_2112_03592_amd import apr as G
from tests.gpu_common import assert_close_scaled, linear_access

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True, file=sys.stderr)


@pytest.fixture(scope="module")
def field():
    say("sphere512 for the gather path")
    inp = cached_sphere_apr("sphere512")
    la = linear_access(inp)
    tr = A.tree_structure(la)
    acc = G.AprAccess.from_input(inp, gather=(3,))
    yield inp, la, tr, acc
    acc.close()


def _bf16(a):
    return torch.from_numpy(np.ascontiguousarray(a, np.float32)).to(torch.bfloat16).float().numpy().astype(np.float64)


@pytest.mark.parametrize("storage", ["f32", "bf16"])
def test_sphere512_16x16_layer_sampled(field, storage):
    inp, la, tr, acc = field
    say("sphere512 16->16", storage)
    rng = np.random.default_rng(31)
    nl = la.l_max - la.l_min + 1
    x = rng.normal(size=(la.n, 16)).astype(np.float32)
    W = (rng.normal(size=(nl, 16, 16, 3, 3, 3)) * 0.1).astype(np.float32)
    b = rng.normal(size=16).astype(np.float32)
    smp = np.sort(rng.choice(la.n, 2048, replace=False))
    if storage == "f32":
        x64, W64 = x.astype(np.float64), W.astype(np.float64)
        tv = oracle_fill(la, tr, x64)
    else:
        # weights and values rounded to BF16 as the matrix-core path takes them;
        # the tree is rounded once (the device rounds every level: a few taps
        # may differ by one BF16 unit, bounded below)
        x64, W64 = _bf16(x), _bf16(W)
        tv = _bf16(oracle_fill(la, tr, x64))
    ref = C.apr_conv_keyed(la, x64, W64, smp, bias=b.astype(np.float64), tree=tr, tvals=tv)
    scale = C.apr_conv_keyed(la, np.abs(x64), np.abs(W64), smp, tree=tr, tvals=np.abs(tv)) + np.abs(b)
    xd = torch.from_numpy(x).cuda()
    if storage == "bf16":
        xd = xd.to(torch.bfloat16)
    t = G.fill_tree(acc, xd)
    y = G.conv(acc, xd, t, torch.from_numpy(W).cuda(), 3, bias=torch.from_numpy(b).cuda(),
               out_dtype=torch.float32).cpu().numpy()
    if storage == "f32":
        assert_close_scaled(y[smp], ref, scale, 1e-5, "sphere512 16->16 FP32")
    else:
        r = np.abs(y[smp] - ref) / scale
        assert r.max() < 5e-3 and (r > 2e-5).mean() < 2e-2, (r.max(), (r > 2e-5).mean())


def test_sphere512_gradients_by_identities(field):
    """<A v, g> = <v, A^T g> for the data gradient; <dW(x, g), W'> =
    <A_W'(x), g> for the weight gradient (bias zero), FP64 sums on the
    device."""
    inp, la, tr, acc = field
    say("sphere512 gradient identities")
    g = torch.Generator(device="cuda").manual_seed(7)
    nl = acc.n_levels
    W = torch.randn(nl, 16, 16, 3, 3, 3, generator=g, device="cuda") * 0.1
    W2 = torch.randn(nl, 16, 16, 3, 3, 3, generator=g, device="cuda") * 0.1
    v = torch.randn(acc.n_particles, 16, generator=g, device="cuda")
    dy = torch.randn(acc.n_particles, 16, generator=g, device="cuda")
    zero = torch.zeros(16, device="cuda")
    tv = G.fill_tree(acc, v)
    lhs = float((G.conv(acc, v, tv, W, 3, bias=zero).double() * dy.double()).sum())
    rhs = float((v.double() * G.conv_bwd_data(acc, dy, W, 3).double()).sum())
    assert abs(lhs - rhs) <= 1e-5 * (abs(lhs) + abs(rhs)), (lhs, rhs)
    dW = G.conv_bwd_weight(acc, v, tv, dy, 3, nl, 16, 16)
    lhs = float((dW.double() * W2.double()).sum())
    rhs = float((G.conv(acc, v, tv, W2, 3, bias=zero).double() * dy.double()).sum())
    assert abs(lhs - rhs) <= 1e-5 * (abs(lhs) + abs(rhs)), (lhs, rhs)
