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
from oracle.bf16 import round_bf16, store_mean_bf16
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


@pytest.mark.parametrize("storage", ["f32", "bf16"])
def test_sphere512_16x16_layer_sampled(field, storage):
    """FP32: normal activations.  BF16 (matrix cores): positive BF16
    activations in [1, 4), BF16 weights, and the oracle's tree stored level
    by level in BF16 like the library's (every sum of children exact in
    FP32), so only the summation order differs."""
    inp, la, tr, acc = field
    say("sphere512 16->16", storage)
    rng = np.random.default_rng(31)
    nl = la.l_max - la.l_min + 1
    if storage == "f32":
        x = rng.normal(size=(la.n, 16)).astype(np.float32)
    else:
        x = round_bf16(rng.uniform(1.0, 4.0, size=(la.n, 16))).astype(np.float32)
    W = (rng.normal(size=(nl, 16, 16, 3, 3, 3)) * 0.1).astype(np.float32)
    b = rng.normal(size=16).astype(np.float32)
    smp = np.sort(rng.choice(la.n, 2048, replace=False))
    if storage == "f32":
        x64, W64 = x.astype(np.float64), W.astype(np.float64)
        tv = oracle_fill(la, tr, x64)
    else:
        x64, W64 = x.astype(np.float64), round_bf16(W)
        tv = oracle_fill(la, tr, x64, store=store_mean_bf16)
    ref = C.apr_conv_keyed(la, x64, W64, smp, bias=b.astype(np.float64), tree=tr, tvals=tv)
    scale = C.apr_conv_keyed(la, np.abs(x64), np.abs(W64), smp, tree=tr, tvals=np.abs(tv)) + np.abs(b)
    xd = torch.from_numpy(x).cuda()
    if storage == "bf16":
        xd = xd.to(torch.bfloat16)
    t = G.fill_tree(acc, xd)
    if storage == "bf16":
        assert np.array_equal(t.float().cpu().numpy().astype(np.float64), tv), "BF16 tree differs from the oracle's"
    y = G.conv(acc, xd, t, torch.from_numpy(W).cuda(), 3, bias=torch.from_numpy(b).cuda(),
               out_dtype=torch.float32).cpu().numpy()
    assert_close_scaled(y[smp], ref, scale, 1e-5 if storage == "f32" else 2e-5, f"sphere512 16->16 {storage}")


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


@pytest.mark.parametrize("k", [3, 5])
def test_dense256_equals_pixel_correlation(k):
    """Section 4.1: with every particle at the finest level the APR
    convolution is the pixel image's correlation with the stencil (zero
    padding outside the image).  256^3, 16.8M particles, every output
    compared with scipy's correlate; the stencil is asymmetric so a
    convolution (flipped stencil) or a transposed axis fails."""
    from scipy import ndimage
    from aprgen.apr_input import dense_apr
    say("dense 256^3 against pixel correlation, k =", k)
    rng = np.random.default_rng(50 + k)
    img = rng.uniform(0.5, 2.0, size=(256, 256, 256)).astype(np.float32)
    w = rng.normal(size=(k, k, k))
    w[0, 0, 0] += 3.0                       # break every symmetry of the stencil
    inp = dense_apr((256, 256, 256), l_min=2, values=img.reshape(-1))
    ref = ndimage.correlate(img.astype(np.float64), w, mode="constant", cval=0.0)
    scale = ndimage.correlate(img.astype(np.float64), np.abs(w), mode="constant", cval=0.0)
    w32 = G.stencil_levels(w, "same", k, inp.l_min, inp.l_max)
    with G.AprAccess.from_input(inp) as acc:
        x = torch.from_numpy(inp.values).cuda()
        t = G.fill_tree(acc, x)
        y = G.conv(acc, x, t, torch.from_numpy(w32).cuda(), k).cpu().numpy().reshape(256, 256, 256)
    # the stencil as passed to the device is FP32
    ref32 = ndimage.correlate(img.astype(np.float64), w.astype(np.float32).astype(np.float64), mode="constant",
                              cval=0.0)
    assert_close_scaled(y.reshape(-1), ref32.reshape(-1), scale.reshape(-1), 1e-5, f"dense256 k={k}")
    assert np.abs(ref32 - ref).max() <= 1e-6 * scale.max()
