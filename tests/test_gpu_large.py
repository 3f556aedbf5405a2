"""Parity on the largest workloads, in the launch configuration the benchmark
times (the whole field on the device), outputs checked against the FP64
oracle on a corner cube of the image:

* the 2048 x 2048 x 1024 sphere field at pixels/particle ratios of ~50, ~100
  and ~200 (86.6M, 43.1M and 21.6M particles, levels 2..11), built on the
  device: tree structure bit-exact, tree values, 3^3 / 5^3 convolution with
  FP32 and BF16 storage, neighbour indices bit-exact;
* the 1024^3 sphere field (35.8M particles, levels 2..10): the 16 -> 16
  layer on the BF16 matrix-core path.

The oracle runs on the APR of the corner cube [0, E)^3 (E a multiple of the
coarsest tree cell, so the cube's tree is the field's tree restricted to it).
Convolution outputs are compared at particles whose level-l neighbourhood
lies inside the cube: there every tap reads the same cells in both.  BF16
storage is checked twice: against the oracle on the same BF16 values with the
tree stored level by level in BF16 (the library's storage rule; only the
summation order differs), and end to end against the oracle on the FP32
values (the BF16 bound)."""
import sys

import numpy as np
import pytest
import torch

from aprgen.apr_input import CONFIGS, _sphere_params
from oracle import access as A
from oracle import conv as C
from oracle import stencil as S
from oracle.bf16 import round_bf16, store_mean_bf16
from oracle.tree import fill_tree as oracle_fill
from paper_2112_03592_amd import apr as G
from tests.gpu_common import assert_close_scaled, corner_block

pytestmark = pytest.mark.gpu

FIELDS = ["field2k_cr200", "field2k_cr100", "field2k_cr50"]


def say(*a):
    print(*a, flush=True, file=sys.stderr)


class Field:
    """One field built on the device, its access structure, and the oracle's
    structures for its corner cube of edge E."""

    def __init__(self, name, edge, gather=()):
        cfg = CONFIGS[name]
        cen, rad = _sphere_params(cfg)
        say(f"building {name} on the device")
        self.name = name
        self.f = G.sphere_field(cfg.dims, cfg.l_min, cen, rad, seed=cfg.seed)
        self.acc = G.AprAccess.from_input(self.f, gather=gather)
        f, acc = self.f, self.acc
        assert edge <= min(f.dims) and edge % (1 << (f.l_max - acc.tree_l_min)) == 0
        self.edge = edge
        self.ds = f.l_max - (edge.bit_length() - 1)
        y, e, self.pidx = corner_block(f.dims, f.l_max, f.l_min, f.l_max, f.y_idx, f.xz_end, edge)
        self.la = A.LinearAccess((edge,) * 3, f.l_min - self.ds, f.l_max - self.ds, y, e)
        say(f"oracle tree of the {edge}^3 corner cube ({self.la.n} of {f.n_particles} particles)")
        self.tr = A.tree_structure(self.la)
        ty, te = acc.export_tree()
        self.dev_ty, self.dev_te, self.tidx = corner_block(f.dims, f.l_max, acc.tree_l_min, acc.tree_l_max, ty, te,
                                                           edge)
        self.x32 = self.f.values[torch.from_numpy(self.pidx).cuda()].cpu().numpy()
        self._cache = {}

    def close(self):
        self.acc.close()

    def x64(self, storage):
        v = self.x32.astype(np.float64)
        return v if storage == "f32" else round_bf16(v)

    def tvals(self, storage):
        key = "t_" + storage
        if key not in self._cache:
            say(f"oracle fill of the cube ({storage})")
            store = None if storage == "f32" else store_mean_bf16
            self._cache[key] = oracle_fill(self.la, self.tr, self.x64(storage), store=store)
        return self._cache[key]

    def interior(self, k):
        """Cube particles whose level-l neighbourhood of radius k // 2 lies in
        the cube (along every axis where the cube's face is inside the
        image)."""
        r = k // 2
        out = []
        for l in range(self.la.l_min, self.la.l_max + 1):
            s = 1 << (self.la.l_max - l)
            c = self.la.cells(l)
            b, _ = self.la.level_range(l)
            ok = np.ones(c.shape[0], bool)
            for a in range(3):
                if self.edge < self.f.dims[a]:
                    ok &= (c[:, a] + r + 1) * s <= self.edge
            out.append(b + np.nonzero(ok)[0])
        return np.concatenate(out)


@pytest.fixture(scope="module", params=FIELDS)
def field(request):
    f = Field(request.param, 1024)
    yield f
    f.close()
    del f


def test_field_tree_bit_exact_and_values(field):
    assert np.array_equal(field.dev_ty, field.tr.y_idx)
    assert np.array_equal(field.dev_te, field.tr.xz_end)
    x = field.f.values
    tix = torch.from_numpy(field.tidx).cuda()
    t = G.fill_tree(field.acc, x)[tix].cpu().numpy()
    tb = G.fill_tree(field.acc, x.to(torch.bfloat16))[tix].float().cpu().numpy()
    assert np.allclose(t.astype(np.float64), field.tvals("f32"), rtol=4e-6, atol=0)
    # BF16 storage: every level's mean in FP32, rounded -- bit-exact
    assert np.array_equal(tb.astype(np.float64), field.tvals("bf16"))


@pytest.mark.parametrize("storage", ["f32", "bf16"])
@pytest.mark.parametrize("k", [3, 5])
def test_field_conv_sampled(field, k, storage):
    la, tr = field.la, field.tr
    say(field.name, "conv", k, storage)
    w32 = G.stencil_levels(S.gaussian_stencil(k, 1.0), "same", k, field.f.l_min, field.f.l_max)
    w64 = w32.astype(np.float64)
    inner = field.interior(k)
    smp = np.sort(np.random.default_rng(10 + k).choice(inner, 4096, replace=False))
    x = field.f.values if storage == "f32" else field.f.values.to(torch.bfloat16)
    x64, tv = field.x64(storage), field.tvals(storage)
    ref = C.apr_conv_keyed(la, x64, w64, smp, tree=tr, tvals=tv)[:, 0]
    scale = C.apr_conv_keyed(la, np.abs(x64), np.abs(w64), smp, tree=tr, tvals=np.abs(tv))[:, 0]
    full = torch.from_numpy(field.pidx[smp]).cuda()
    t = G.fill_tree(field.acc, x)
    y = G.conv(field.acc, x, t, torch.from_numpy(w32).cuda(), k, out_dtype=torch.float32)[full].cpu().numpy()
    nm = G.neighbor_map(field.acc, k, full[:512]).cpu().numpy()
    del t
    # arithmetic error: the same stored values on both sides
    assert_close_scaled(y, ref, scale, 1e-5, f"{field.name} k={k} {storage}")
    if storage == "bf16":
        # end to end against the FP32 values: the BF16 storage bound
        ref32 = C.apr_conv_keyed(la, field.x64("f32"), w64, smp, tree=tr, tvals=field.tvals("f32"))[:, 0]
        assert_close_scaled(y, ref32, scale, 1e-2, f"{field.name} k={k} BF16 end to end")
    # neighbour indices: the oracle's cube indices mapped to the field's
    src, idx = C.neighbor_map(la, k, smp[:512], tree=tr)
    want = np.where(src == 0, -1, 0).astype(np.int64)
    part = (src == 1) | (src == 2)
    want[part] = (src[part].astype(np.int64) << 40) | field.pidx[idx[part]]
    tre = src == 3
    want[tre] = (np.int64(3) << 40) | field.tidx[idx[tre]]
    assert np.array_equal(nm, want)


def test_field1k_16x16_layer_sampled():
    """The 16 -> 16 BF16 layer at 35.8M particles: positive BF16 activations
    in [1, 4) (every sum of children exact in FP32), BF16 weights, and the
    oracle's tree stored level by level in BF16 as the library stores it, so
    only the summation order differs.  Oracle on the 512^3 corner cube."""
    fld = Field("field1k_layer", 512, gather=(3,))
    la, tr = fld.la, fld.tr
    rng = np.random.default_rng(41)
    nl = fld.f.l_max - fld.f.l_min + 1
    gen = torch.Generator(device="cuda").manual_seed(41)
    xd = torch.empty(fld.f.n_particles, 16, device="cuda").uniform_(1.0, 4.0, generator=gen).to(torch.bfloat16)
    x = xd[torch.from_numpy(fld.pidx).cuda()].float().cpu().numpy().astype(np.float64)
    say("oracle 16-channel BF16 fill of the cube")
    tvals = oracle_fill(la, tr, x, store=store_mean_bf16)
    W = (rng.normal(size=(nl, 16, 16, 3, 3, 3)) * np.sqrt(2.0 / (16 * 27))).astype(np.float32)
    bias = rng.normal(size=16).astype(np.float32)
    W64 = round_bf16(W)
    smp = np.sort(rng.choice(fld.interior(3), 2048, replace=False))
    t = G.fill_tree(fld.acc, xd)
    ts = t[torch.from_numpy(fld.tidx).cuda()].float().cpu().numpy()
    y = G.conv(fld.acc, xd, t, torch.from_numpy(W).cuda(), 3, bias=torch.from_numpy(bias).cuda(),
               out_dtype=torch.float32)
    ys = y[torch.from_numpy(fld.pidx[smp]).cuda()].cpu().numpy()
    del y, t, xd
    fld.close()
    assert np.array_equal(ts.astype(np.float64), tvals), "BF16 tree differs from the oracle's"
    ref = C.apr_conv_keyed(la, x, W64, smp, bias=bias.astype(np.float64), tree=tr, tvals=tvals)
    scale = C.apr_conv_keyed(la, x, np.abs(W64), smp, tree=tr, tvals=tvals) + np.abs(bias)
    assert_close_scaled(ys, ref, scale, 2e-5, "field1k 16->16 BF16 on matrix cores")
