"""Parity on the largest workloads, in the launch configuration the benchmark
times, outputs checked on seeded samples against the FP64 oracle:

* the 2048 x 2048 x 1024 sphere field at a pixels/particles ratio of ~200
  (21.5M particles, levels 2..11): tree structure bit-exact, tree values,
  3^3 / 5^3 convolution with FP32 and BF16 storage;
* the 1024^3 sphere field (35.8M particles, levels 2..10): the 16 -> 16
  layer on the BF16 matrix-core path.

Both fields are generated slab by slab (``load_sphere_apr``)."""
import sys

import numpy as np
import pytest
import torch

from aprgen.apr_input import load_sphere_apr
from oracle import access as A
from oracle import conv as C
from oracle import stencil as S
from oracle.tree import fill_tree as oracle_fill
from paper_2112_03592_amd import apr as G
from tests.gpu_common import assert_close_scaled, encode_oracle_map, linear_access

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True, file=sys.stderr)


def _bf16(a):
    return torch.from_numpy(np.ascontiguousarray(a, np.float32)).to(torch.bfloat16).float().numpy().astype(np.float64)


@pytest.fixture(scope="module")
def field2k():
    say("generating field2k_cr200")
    inp = load_sphere_apr("field2k_cr200", progress=lambda d, n: say(f"  slab {d}/{n}") if d % 8 == 0 else None)
    la = linear_access(inp)
    say(f"oracle tree for field2k_cr200 ({inp.n_particles} particles)")
    tr = A.tree_structure(la)
    return inp, la, tr


def test_field2k_tree_bit_exact_and_values(field2k):
    inp, la, tr = field2k
    tv = oracle_fill(la, tr, inp.values.astype(np.float64))
    with G.AprAccess.from_input(inp) as acc:
        ty, te = acc.export_tree()
        assert np.array_equal(ty.astype(np.int64), tr.y_idx)
        assert np.array_equal(te.astype(np.int64), tr.xz_end)
        t = G.fill_tree(acc, torch.from_numpy(inp.values).cuda()).cpu().numpy()
    assert np.allclose(t.astype(np.float64), tv, rtol=4e-6, atol=0)


@pytest.mark.parametrize("storage", ["f32", "bf16"])
@pytest.mark.parametrize("k", [3, 5])
def test_field2k_conv_sampled(field2k, k, storage):
    inp, la, tr = field2k
    say("field2k conv", k, storage)
    w32 = G.stencil_levels(S.gaussian_stencil(k, 1.0), "same", k, la.l_min, la.l_max)
    smp = np.sort(np.random.default_rng(10 + k).choice(la.n, 4096, replace=False))
    x = torch.from_numpy(inp.values).cuda()
    if storage == "bf16":
        x = x.to(torch.bfloat16)
        x64 = _bf16(inp.values)
    else:
        x64 = inp.values.astype(np.float64)
    tv = oracle_fill(la, tr, x64)
    ref = C.apr_conv_keyed(la, x64, w32.astype(np.float64), smp, tree=tr, tvals=tv)[:, 0]
    scale = C.apr_conv_keyed(la, np.abs(x64), np.abs(w32.astype(np.float64)), smp, tree=tr,
                             tvals=oracle_fill(la, tr, np.abs(x64)))[:, 0]
    with G.AprAccess.from_input(inp) as acc:
        t = G.fill_tree(acc, x)
        y = G.conv(acc, x, t, torch.from_numpy(w32).cuda(), k, out_dtype=torch.float32).cpu().numpy()
        nm = G.neighbor_map(acc, k, torch.from_numpy(smp[:512]).cuda()).cpu().numpy()
    assert_close_scaled(y[smp], ref, scale, 1e-5 if storage == "f32" else 1e-2, f"field2k k={k} {storage}")
    src, idx = C.neighbor_map(la, k, smp[:512], tree=tr)
    assert np.array_equal(nm, encode_oracle_map(src, idx))


def test_field1k_16x16_layer_sampled():
    """The 16 -> 16 BF16 layer at 35.8M particles.  The input channels are
    combinations of two integer particle fields, x[:, c] = a_c u + b_c v with
    quarter-integer a_c, b_c, so every value is exact in BF16 and the
    oracle's tree values follow exactly from two single-channel fills (the
    fill is linear); the weights mix all channels."""
    say("generating field1k_layer")
    inp = load_sphere_apr("field1k_layer", progress=lambda d, n: say(f"  slab {d}/{n}") if d % 8 == 0 else None)
    la = linear_access(inp)
    say(f"oracle tree for field1k_layer ({inp.n_particles} particles)")
    tr = A.tree_structure(la)
    rng = np.random.default_rng(41)
    nl = la.l_max - la.l_min + 1
    u = rng.integers(-8, 9, size=la.n).astype(np.float64)
    v = rng.integers(-8, 9, size=la.n).astype(np.float64)
    a, b = rng.integers(-4, 5, size=16) / 4.0, rng.integers(-4, 5, size=16) / 4.0
    x = u[:, None] * a[None, :] + v[:, None] * b[None, :]          # exact in BF16
    tu, tv_ = oracle_fill(la, tr, u), oracle_fill(la, tr, v)
    # the device rounds tree values to BF16 at every level, the oracle's tree
    # once (a few taps may differ by one BF16 unit, bounded below)
    tvals = _bf16(tu[:, None] * a[None, :] + tv_[:, None] * b[None, :])
    del tu, tv_
    W = (rng.normal(size=(nl, 16, 16, 3, 3, 3)) * np.sqrt(2.0 / (16 * 27))).astype(np.float32)
    bias = rng.normal(size=16).astype(np.float32)
    W64 = _bf16(W)
    smp = np.sort(rng.choice(la.n, 2048, replace=False))
    with G.AprAccess.from_input(inp, gather=(3,)) as acc:
        xd = torch.from_numpy(x.astype(np.float32)).to(torch.bfloat16).cuda()
        t = G.fill_tree(acc, xd)
        y = G.conv(acc, xd, t, torch.from_numpy(W).cuda(), 3, bias=torch.from_numpy(bias).cuda(),
                   out_dtype=torch.float32)
        ys = y[torch.from_numpy(smp).cuda()].cpu().numpy()
        del y, t, xd
    ref = C.apr_conv_keyed(la, x, W64, smp, bias=bias.astype(np.float64), tree=tr, tvals=tvals)
    scale = C.apr_conv_keyed(la, np.abs(x), np.abs(W64), smp, tree=tr, tvals=np.abs(tvals)) + np.abs(bias)
    r = np.abs(ys - ref) / scale
    assert r.max() < 5e-3 and (r > 2e-5).mean() < 2e-2, (r.max(), (r > 2e-5).mean())
