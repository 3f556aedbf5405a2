"""GPU parity of the gather-map path (multichannel convolution) and of the
hand-written backward kernels, against the FP64 oracle and by the adjoint
identity / finite differences on the device."""
import sys

import numpy as np
import pytest
import torch

from aprgen.apr_input import CONFIGS, random_apr, sphere_apr
from oracle import access as A
from oracle import conv as C
from oracle.bf16 import round_bf16, store_mean_bf16
from oracle.tree import fill_tree as oracle_fill
from paper_2112_03592_amd import apr as G
from tests.gpu_common import SMALL_CASES, assert_close_scaled, linear_access

pytestmark = pytest.mark.gpu

CASES = {
    "rand16_l1": lambda: random_apr((16, 16, 16), l_min=1, seed=2, p_refine=0.25),
    "rand9x12x7": lambda: random_apr((9, 12, 7), l_min=1, seed=3, p_refine=0.3),
    "rand33x20x70": lambda: random_apr((33, 20, 70), l_min=2, seed=5, p_refine=0.2),
    "sphere32": lambda: sphere_apr(CONFIGS["sphere32"]),
    # degenerate structures: one particle and no tree levels; one level
    # only; every particle at the finest level; levels down to 0
    "single_cell": SMALL_CASES["single_cell"],
    "one_level": SMALL_CASES["one_level"],
    "dense13x11x70": SMALL_CASES["dense13x11x70"],
    "rand8_l0": SMALL_CASES["rand8_l0"],
}
_cache = {}


def say(*a):
    print(*a, flush=True, file=sys.stderr)


def case(name):
    if name not in _cache:
        inp = CASES[name]()
        la = linear_access(inp)
        _cache[name] = (inp, la, A.tree_structure(la))
    return _cache[name]


def _setup(name, k, cin, cout, nw_shared=False, seed=0):
    inp, la, tr = case(name)
    rng = np.random.default_rng(seed)
    nl = 1 if nw_shared else la.l_max - la.l_min + 1
    W = rng.normal(size=(nl, cout, cin, k, k, k)).astype(np.float32)
    x = rng.normal(size=(la.n, cin)).astype(np.float32)
    return inp, la, tr, W, x


CH = [(3, 2, 3), (5, 2, 3), (3, 1, 16), (3, 16, 16), (3, 16, 1), (5, 1, 1), (3, 1, 1)]


@pytest.mark.parametrize("name", list(CASES))
@pytest.mark.parametrize("k,cin,cout", CH)
def test_multichannel_forward(name, k, cin, cout):
    say("mc fwd", name, k, cin, cout)
    inp, la, tr, W, x = _setup(name, k, cin, cout, seed=k * 100 + cin * 10 + cout)
    b = np.random.default_rng(1).normal(size=cout).astype(np.float32)
    ref = C.apr_conv(la, x.astype(np.float64), W.astype(np.float64), bias=b.astype(np.float64), tree=tr)
    scale = C.apr_conv(la, np.abs(x.astype(np.float64)), np.abs(W.astype(np.float64)), tree=tr) + np.abs(b)
    with G.AprAccess.from_input(inp, gather=(k,)) as acc:
        xd = torch.from_numpy(x).cuda()
        t = G.fill_tree(acc, xd)
        wd = torch.from_numpy(W).cuda()
        bd = torch.from_numpy(b).cuda()
        y = G.conv(acc, xd, t, wd, k, bias=bd).cpu().numpy()
        yr = G.conv(acc, xd, t, wd, k, bias=bd, relu=True).cpu().numpy()
    assert_close_scaled(y, ref, scale, 1e-5, f"{name} k={k} {cin}->{cout}")
    assert_close_scaled(yr, np.maximum(ref, 0), scale, 1e-5, "relu")


def test_multichannel_bf16_storage():
    inp, la, tr, W, x = _setup("sphere32", 3, 16, 16, seed=3)
    with G.AprAccess.from_input(inp, gather=(3,)) as acc:
        xb = torch.from_numpy(x).cuda().to(torch.bfloat16)
        x64 = xb.float().cpu().numpy().astype(np.float64)
        ref = C.apr_conv(la, x64, W.astype(np.float64), tree=tr)
        scale = C.apr_conv(la, np.abs(x64), np.abs(W.astype(np.float64)), tree=tr)
        t = G.fill_tree(acc, xb)
        y = G.conv(acc, xb, t, torch.from_numpy(W).cuda(), 3, bias=torch.zeros(16, device="cuda"),
                   out_dtype=torch.float32).cpu().numpy()
    assert_close_scaled(y, ref, scale, 1e-2, "bf16 storage 16->16")


@pytest.mark.parametrize("name", list(CASES))
@pytest.mark.parametrize("k,cin,cout", CH)
@pytest.mark.parametrize("shared", [False, True])
def test_backward_data_and_weight(name, k, cin, cout, shared):
    say("bwd", name, k, cin, cout, shared)
    inp, la, tr, W, x = _setup(name, k, cin, cout, nw_shared=shared, seed=7 + k + cin + cout)
    g = np.random.default_rng(11).normal(size=(la.n, cout)).astype(np.float32)
    W64, g64, x64 = W.astype(np.float64), g.astype(np.float64), x.astype(np.float64)
    ref_dx = C.apr_conv_bwd_data(la, g64, W64, tree=tr)
    sc_dx = C.apr_conv_bwd_data(la, np.abs(g64), np.abs(W64), tree=tr)
    ref_dw = C.apr_conv_bwd_weight(la, x64, g64, k, n_wlevels=W.shape[0], tree=tr)
    sc_dw = C.apr_conv_bwd_weight(la, np.abs(x64), np.abs(g64), k, n_wlevels=W.shape[0], tree=tr)
    with G.AprAccess.from_input(inp, gather=(k,)) as acc:
        xd = torch.from_numpy(x).cuda()
        t = G.fill_tree(acc, xd)
        dx = G.conv_bwd_data(acc, torch.from_numpy(g).cuda(), torch.from_numpy(W).cuda(), k).cpu().numpy()
        dw = G.conv_bwd_weight(acc, xd, t, torch.from_numpy(g).cuda(), k, W.shape[0], cin, cout).cpu().numpy()
    assert_close_scaled(dx, ref_dx, sc_dx, 1e-5, f"dX {name} k={k} {cin}->{cout}")
    assert_close_scaled(dw, ref_dw, sc_dw, 1e-5, f"dW {name} k={k} {cin}->{cout}")


@pytest.mark.parametrize("name", ["rand33x20x70", "sphere32"])
@pytest.mark.parametrize("cin,cout", [(1, 1), (1, 16), (16, 16), (16, 1), (2, 3)])
def test_backward_weight_bf16_x(name, cin, cout):
    """Weight gradient with BF16 activations (the 16 -> 16 matrix-core kernel
    and the block-sum kernel): the oracle takes the same BF16 values and the
    tree stored level by level in BF16 (positive values in [1, 4): every sum
    of children is exact in FP32), so only the summation order differs."""
    say("bwd weight bf16 x", name, cin, cout)
    inp, la, tr, W, _ = _setup(name, 3, cin, cout, seed=40 + cin + cout)
    rng = np.random.default_rng(41)
    x = round_bf16(rng.uniform(1.0, 4.0, size=(la.n, cin))).astype(np.float32)
    g = rng.normal(size=(la.n, cout)).astype(np.float32)
    x64, g64 = x.astype(np.float64), g.astype(np.float64)
    tv = oracle_fill(la, tr, x64, store=store_mean_bf16)
    ref = C.apr_conv_bwd_weight(la, x64, g64, 3, n_wlevels=W.shape[0], tree=tr, tvals=tv)
    sc = C.apr_conv_bwd_weight(la, x64, np.abs(g64), 3, n_wlevels=W.shape[0], tree=tr, tvals=tv)
    with G.AprAccess.from_input(inp, gather=(3,)) as acc:
        xd = torch.from_numpy(x).cuda().to(torch.bfloat16)
        t = G.fill_tree(acc, xd)
        assert np.array_equal(t.float().cpu().numpy().astype(np.float64).reshape(tv.shape), tv)
        dw = G.conv_bwd_weight(acc, xd, t, torch.from_numpy(g).cuda(), 3, W.shape[0], cin, cout).cpu().numpy()
    assert_close_scaled(dw, ref, sc, 1e-5, f"dW BF16 x {name} {cin}->{cout}")


@pytest.mark.parametrize("name", ["rand33x20x70", "sphere32", "dense13x11x70"])
@pytest.mark.parametrize("dtype", ["f32", "bf16"])
def test_backward_16_both_address_forms(name, dtype, monkeypatch):
    """The 16 -> 16 weight and data gradients read their gathers through
    32-bit buffer offsets up to a size limit and through 64-bit addresses
    above it; APR_WIDE_OFFSETS=1 forces the second form here, and =2 the
    weight gradient's two-buffer form (x and the tree too far apart for one
    buffer).  All sum the same products in the same order, so they agree bit
    for bit, and with the oracle."""
    say("bwd weight address forms", name, dtype)
    inp, la, tr, W, _ = _setup(name, 3, 16, 16, seed=60)
    rng = np.random.default_rng(61)
    # BF16-exact values in [1, 4): the BF16 tree means are exact (as in the
    # BF16 test above), so the oracle's fill matches the stored tree
    x = round_bf16(rng.uniform(1.0, 4.0, size=(la.n, 16))).astype(np.float32)
    g = rng.normal(size=(la.n, 16)).astype(np.float32)
    with G.AprAccess.from_input(inp, gather=(3,)) as acc:
        xd = torch.from_numpy(x).cuda()
        if dtype == "bf16":
            xd = xd.to(torch.bfloat16)
        t = G.fill_tree(acc, xd)
        gd = torch.from_numpy(g).cuda()
        wd = torch.from_numpy(W).cuda()
        dw_buf = G.conv_bwd_weight(acc, xd, t, gd, 3, W.shape[0], 16, 16).cpu().numpy()
        dx_buf = G.conv_bwd_data(acc, gd, wd, 3).cpu().numpy()
        monkeypatch.setenv("APR_WIDE_OFFSETS", "1")
        dw_wide = G.conv_bwd_weight(acc, xd, t, gd, 3, W.shape[0], 16, 16).cpu().numpy()
        dx_wide = G.conv_bwd_data(acc, gd, wd, 3).cpu().numpy()
        monkeypatch.setenv("APR_WIDE_OFFSETS", "2")   # x and the tree as two buffers
        dw_two = G.conv_bwd_weight(acc, xd, t, gd, 3, W.shape[0], 16, 16).cpu().numpy()
        monkeypatch.delenv("APR_WIDE_OFFSETS")
    assert np.array_equal(dw_buf, dw_wide)
    assert np.array_equal(dw_buf, dw_two)
    assert np.array_equal(dx_buf, dx_wide)
    x64, g64 = x.astype(np.float64), g.astype(np.float64)
    tv = oracle_fill(la, tr, x64, store=store_mean_bf16) if dtype == "bf16" else None
    ref = C.apr_conv_bwd_weight(la, x64, g64, 3, n_wlevels=W.shape[0], tree=tr, tvals=tv)
    sc = C.apr_conv_bwd_weight(la, x64, np.abs(g64), 3, n_wlevels=W.shape[0], tree=tr, tvals=tv)
    assert_close_scaled(dw_buf, ref, sc, 1e-5, f"dW 16->16 {dtype} {name}")
    W64 = W.astype(np.float64)
    ref_dx = C.apr_conv_bwd_data(la, g64, W64, tree=tr)
    sc_dx = C.apr_conv_bwd_data(la, np.abs(g64), np.abs(W64), tree=tr)
    assert_close_scaled(dx_buf, ref_dx, sc_dx, 1e-5, f"dX 16->16 {name}")


@pytest.mark.parametrize("k,cin,cout", [(3, 16, 16), (5, 1, 1), (3, 1, 16)])
def test_adjoint_identity_on_device(k, cin, cout):
    """<A v, g> from the device forward equals <v, A^T g> from the device
    backward (the forward is linear in x: a central difference with any step
    is exact up to rounding)."""
    inp, la, tr, W, x = _setup("sphere32", k, cin, cout, seed=5)
    rng = np.random.default_rng(6)
    g = rng.normal(size=(la.n, cout)).astype(np.float32)
    with G.AprAccess.from_input(inp, gather=(k,)) as acc:
        wd = torch.from_numpy(W).cuda()
        zb = torch.zeros(cout, device="cuda")
        v = torch.from_numpy(rng.normal(size=(la.n, cin)).astype(np.float32)).cuda()
        gd = torch.from_numpy(g).cuda()
        yp = G.conv(acc, v, G.fill_tree(acc, v), wd, k, bias=zb)
        vm = -v
        ym = G.conv(acc, vm, G.fill_tree(acc, vm), wd, k, bias=zb)
        fd = float(((yp - ym) / 2).double().mul(gd.double()).sum())
        dx = G.conv_bwd_data(acc, gd, wd, k)
        an = float(dx.double().mul(v.double()).sum())
    assert abs(fd - an) <= 1e-5 * (abs(fd) + abs(an))


@pytest.mark.parametrize("name", list(CASES))
@pytest.mark.parametrize("dtype", [torch.float32, torch.bfloat16])
def test_fill_16_channels_via_child_map_equals_one_channel_fill(name, dtype):
    """The 16-channel fill (child map, built with the gather maps) sums the
    children in the one-channel kernel's order: bit-identical per channel."""
    inp, la, tr = case(name)
    x = np.random.default_rng(4).normal(size=(la.n, 16)).astype(np.float32)
    with G.AprAccess.from_input(inp, gather=(3,)) as acc:
        xd = torch.from_numpy(x).cuda().to(dtype)
        t16 = G.fill_tree(acc, xd).cpu()
        for c in (0, 7, 15):
            t1 = G.fill_tree(acc, xd[:, c].contiguous()).cpu()
            assert torch.equal(t16[:, c], t1), c
    x64 = xd.float().cpu().numpy().astype(np.float64)
    ref = oracle_fill(la, tr, x64)
    # every stored level is rounded to the storage type: bound the error by
    # the mean of |x| over the node's pixels
    scale = oracle_fill(la, tr, np.abs(x64))
    tol = 1e-6 if dtype == torch.float32 else 1e-2
    assert (np.abs(t16.float().numpy() - ref) <= tol * scale + 1e-30).all()


@pytest.mark.parametrize("name", list(CASES))
@pytest.mark.parametrize("out_dtype", [torch.float32, torch.bfloat16])
def test_mfma_16x16_forward(name, out_dtype):
    """16 -> 16 channels with BF16 activations runs on MFMA with BF16 weights
    and FP32 accumulation.  The oracle takes the BF16-rounded inputs and
    weights and stores every tree level in BF16 (FP32 mean, rounded, the
    library's storage rule): only the summation order differs.  Activations
    are positive BF16 values in [1, 4) (as after a ReLU), so every sum of
    children is exact in FP32 and the stored tree is bit-exact."""
    say("mfma", name, out_dtype)
    inp, la, tr, W, _ = _setup(name, 3, 16, 16, seed=21)
    rng = np.random.default_rng(22)
    x = round_bf16(rng.uniform(1.0, 4.0, size=(la.n, 16))).astype(np.float32)
    b = rng.normal(size=16).astype(np.float32)
    res = rng.normal(size=(la.n, 16)).astype(np.float32)
    xb, Wb = x.astype(np.float64), round_bf16(W)
    resb = round_bf16(res) if out_dtype == torch.bfloat16 else res.astype(np.float64)
    tv = oracle_fill(la, tr, xb, store=store_mean_bf16)
    ref = C.apr_conv(la, xb, Wb, bias=b.astype(np.float64), tree=tr, tvals=tv)
    scale = C.apr_conv(la, np.abs(xb), np.abs(Wb), tree=tr, tvals=np.abs(tv)) + np.abs(b)
    with G.AprAccess.from_input(inp, gather=(3,)) as acc:
        xd = torch.from_numpy(x).cuda().to(torch.bfloat16)
        t = G.fill_tree(acc, xd)
        assert np.array_equal(t.float().cpu().numpy().astype(np.float64), tv), "BF16 tree differs from the oracle's"
        wd = torch.from_numpy(W).cuda()
        bd = torch.from_numpy(b).cuda()
        rd = torch.from_numpy(res).cuda().to(out_dtype)
        y = G.conv(acc, xd, t, wd, 3, bias=bd, out_dtype=out_dtype).float().cpu().numpy()
        yr = G.conv(acc, xd, t, wd, 3, bias=bd, relu=True, residual=rd, out_dtype=out_dtype).float().cpu().numpy()
    if out_dtype == torch.float32:
        assert_close_scaled(y, ref, scale, 2e-5, f"{name} plain")
        assert_close_scaled(yr, np.maximum(ref + resb, 0), scale + np.abs(resb), 2e-5, f"{name} relu")
    else:
        # BF16 outputs: the FP32 result rounded once, half a BF16 unit of it
        for got, want, sc, what in ((y, ref, scale, "plain"),
                                    (yr, np.maximum(ref + resb, 0), scale + np.abs(resb), "relu")):
            bound = (np.abs(want) + 2e-5 * sc) * 2.0 ** -8 + 2e-5 * sc
            assert (np.abs(got - want) <= bound).all(), (what, name, float(np.max(np.abs(got - want) / sc)))
