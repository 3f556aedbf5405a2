"""GPU parity of the HIP library against the FP64 oracle, through the C ABI.

Bars (from the design targets): access/tree/neighbour indexing bit-exact;
FP32 outputs within 1e-5 * M_p where M_p = sum_o |w_l[o]| |V_l(c_p+o)|;
BF16 storage within 1e-2 * M_p."""
import sys

import numpy as np
import pytest
import torch

from aprgen.apr_input import cached_sphere_apr, random_apr
from oracle import access as A
from oracle import conv as C
from oracle import stencil as S
from oracle.tree import fill_tree as oracle_fill
from tests.gpu_common import (SMALL_CASES, assert_close_scaled, encode_oracle_map, linear_access)

pytestmark = pytest.mark.gpu

from paper_2112_03592_amd import apr as G  # noqa: E402


def say(*a):
    print(*a, flush=True, file=sys.stderr)


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a HIP device")
    G.AprAccess  # library must be loadable
    from paper_2112_03592_amd import _lib
    _lib.load()


_cache = {}


def case(name):
    if name not in _cache:
        inp = SMALL_CASES[name]()
        la = linear_access(inp)
        tr = A.tree_structure(la)
        _cache[name] = (inp, la, tr)
    return _cache[name]


@pytest.mark.parametrize("name", list(SMALL_CASES))
def test_tree_structure_bit_exact(name):
    say("tree structure", name)
    inp, la, tr = case(name)
    with G.AprAccess.from_input(inp) as acc:
        ty, te = acc.export_tree()
        assert acc.n_tree == tr.n
        assert np.array_equal(ty.astype(np.int64), tr.y_idx)
        assert np.array_equal(te.astype(np.int64), tr.xz_end)
        assert (acc.tree_l_min, acc.tree_l_max) == (tr.l_min, tr.l_max)


@pytest.mark.parametrize("name", list(SMALL_CASES))
def test_export_apr_and_tiles(name):
    """The particle LinearAccess round-trips bit-exactly; the tile list is
    the set of 8 x 8-row tiles of each level that hold a particle, each with
    the smallest y of its particles, split into eight launch ranges."""
    say("export", name)
    inp, la, tr = case(name)
    with G.AprAccess.from_input(inp) as acc:
        y, e = acc.export_apr()
        tiles, off = acc.export_tiles()
    assert np.array_equal(y, inp.y_idx) and np.array_equal(e, inp.xz_end)
    want = {}
    for l in range(la.l_min, la.l_max + 1):
        c = la.cells(l)
        for (z, x, yy) in c:
            key = (l, int(z) // 8, int(x) // 8)
            want[key] = min(want.get(key, 1 << 30), int(yy))
    got = {(int(t[0]), int(t[1]), int(t[2])): int(t[3]) for t in tiles}
    assert len(got) == tiles.shape[0], "a tile is listed twice"
    assert got == want
    assert off[0] == 0 and off[8] >= tiles.shape[0] and np.all(np.diff(off) >= 0)
    # the pre-pass on its own: one flag and smallest y per candidate tile,
    # finest level first, then tile z, tile x
    with G.AprAccess.from_input(inp) as acc:
        flags, ymin = G.tile_prepass(acc)
        flags, ymin = flags.cpu().numpy(), ymin.cpu().numpy()
    k = 0
    for l in range(la.l_max, la.l_min - 1, -1):
        dz, dx = la.z_dim[l], la.x_dim[l]
        for tz in range(-(-dz // 8)):
            for tx in range(-(-dx // 8)):
                key = (l, tz, tx)
                assert flags[k] == (key in want), key
                assert ymin[k] == want.get(key, 0xffff), key
                k += 1
    assert k == flags.shape[0]


@pytest.mark.parametrize("name", list(SMALL_CASES))
def test_fill_tree_fp32(name):
    say("fill tree", name)
    inp, la, tr = case(name)
    ref = oracle_fill(la, tr, inp.values.astype(np.float64))
    with G.AprAccess.from_input(inp) as acc:
        x = torch.from_numpy(inp.values).cuda()
        t = G.fill_tree(acc, x).cpu().numpy().astype(np.float64)
    # mean of <= 8 positive children per level, FP32
    assert np.allclose(t, ref, rtol=4e-6, atol=0)


def _weights(k, mode, la, seed):
    """(library FP32 stencils for the GPU, the oracle's FP64 stencils for the
    reference): per-level stencils are built on each side independently."""
    rng = np.random.default_rng(seed)
    if mode == "explicit":
        w = rng.normal(size=(la.l_max - la.l_min + 1, k, k, k)).astype(np.float32)
        return w, w.astype(np.float64)
    if mode == "asym":
        w = rng.normal(size=(k, k, k))
        return G.stencil_levels(w, "same", k, la.l_min, la.l_max), S.level_stencils(w, S.SAME, la.l_min, la.l_max)
    g = S.gaussian_stencil(k, 1.0)
    return G.stencil_levels(g, mode, k, la.l_min, la.l_max), S.level_stencils(g, mode, la.l_min, la.l_max)


@pytest.mark.parametrize("name", list(SMALL_CASES))
@pytest.mark.parametrize("k", [3, 5])
@pytest.mark.parametrize("mode", ["restrict", "explicit"])
def test_conv_fp32(name, k, mode):
    say("conv fp32", name, k, mode)
    inp, la, tr = case(name)
    w32, w64 = _weights(k, mode, la, seed=k)
    x64 = inp.values.astype(np.float64)
    ref = C.apr_conv(la, x64, w64, tree=tr)
    scale = C.apr_conv(la, np.abs(x64), np.abs(w64), tree=tr)
    with G.AprAccess.from_input(inp) as acc:
        x = torch.from_numpy(inp.values).cuda()
        t = G.fill_tree(acc, x)
        y = G.conv(acc, x, t, torch.from_numpy(np.ascontiguousarray(w32)).cuda(), k).cpu().numpy()
    assert_close_scaled(y, ref, scale, 1e-5, f"{name} k={k} {mode}")


@pytest.mark.parametrize("name", ["rand8_l0", "rand9x12x7", "rand33x20x70", "rand_long_y", "single_cell",
                                  "dense13x11x70", "sphere64"])
@pytest.mark.parametrize("k", [7, 9, 11, 13])
@pytest.mark.parametrize("mode", ["restrict", "explicit"])
def test_conv_large_stencils(name, k, mode):
    """Stencils above 5^3: taps reach APR level l-2; patches of at most 32
    output cells along y."""
    say("conv large", name, k, mode)
    inp, la, tr = case(name)
    w32, w64 = _weights(k, mode, la, seed=k)
    x64 = inp.values.astype(np.float64)
    ref = C.apr_conv(la, x64, w64, tree=tr)
    scale = C.apr_conv(la, np.abs(x64), np.abs(w64), tree=tr)
    with G.AprAccess.from_input(inp) as acc:
        x = torch.from_numpy(inp.values).cuda()
        t = G.fill_tree(acc, x)
        y = G.conv(acc, x, t, torch.from_numpy(np.ascontiguousarray(w32)).cuda(), k).cpu().numpy()
    assert_close_scaled(y, ref, scale, 1e-5, f"{name} k={k} {mode}")


@pytest.mark.parametrize("name", list(SMALL_CASES))
def test_conv5_central_3cubed_levels(name):
    """Levels whose 5^3 weights vanish outside the central 3^3 (restricted
    stencils at coarse levels, Eq. restrict_stenc) run the 3^3 body in the 5^3
    launch: bit-identical to the 3^3 convolution with those weights, and, with
    the finest level keeping a full 5^3 stencil, within the FP32 bar of the
    oracle."""
    say("conv5 central 3^3", name)
    inp, la, tr = case(name)
    nl = la.l_max - la.l_min + 1
    rng = np.random.default_rng(53)
    w3 = rng.normal(size=(nl, 3, 3, 3)).astype(np.float32)
    w5 = np.zeros((nl, 5, 5, 5), np.float32)
    w5[:, 1:4, 1:4, 1:4] = w3
    mixed = w5.copy()
    mixed[-1] = rng.normal(size=(5, 5, 5)).astype(np.float32)   # the finest level: full 5^3
    x64 = inp.values.astype(np.float64)
    with G.AprAccess.from_input(inp) as acc:
        x = torch.from_numpy(inp.values).cuda()
        t = G.fill_tree(acc, x)
        y3 = G.conv(acc, x, t, torch.from_numpy(w3).cuda(), 3).cpu().numpy()
        y5 = G.conv(acc, x, t, torch.from_numpy(w5).cuda(), 5).cpu().numpy()
        ym = G.conv(acc, x, t, torch.from_numpy(mixed).cuda(), 5).cpu().numpy()
    assert np.array_equal(y3, y5)
    ref = C.apr_conv(la, x64, mixed.astype(np.float64), tree=tr)
    scale = C.apr_conv(la, np.abs(x64), np.abs(mixed.astype(np.float64)), tree=tr)
    assert_close_scaled(ym, ref, scale, 1e-5, f"{name} mixed 3^3 / 5^3 levels")


@pytest.mark.parametrize("name", ["rand16_l1", "rand33x20x70", "sphere64"])
def test_conv_shared_stencil_and_signed_values(name):
    inp, la, tr = case(name)
    rng = np.random.default_rng(5)
    xs = rng.normal(size=la.n).astype(np.float32)
    w = rng.normal(size=(1, 5, 5, 5)).astype(np.float32)
    ref = C.apr_conv(la, xs.astype(np.float64), w.astype(np.float64), tree=tr)
    scale = C.apr_conv(la, np.abs(xs.astype(np.float64)), np.abs(w.astype(np.float64)), tree=tr)
    with G.AprAccess.from_input(inp) as acc:
        x = torch.from_numpy(xs).cuda()
        t = G.fill_tree(acc, x)
        y = G.conv(acc, x, t, torch.from_numpy(w).cuda(), 5).cpu().numpy()
    assert_close_scaled(y, ref, scale, 1e-5, name)


@pytest.mark.parametrize("name", ["rand8_l0", "rand9x12x7", "rand33x20x70", "rand_long_y", "sphere64",
                                  "dense13x11x70", "single_cell"])
@pytest.mark.parametrize("k", [3, 5])
def test_neighbor_map_bit_exact(name, k):
    say("neighbour map", name, k)
    inp, la, tr = case(name)
    sel = np.arange(la.n) if la.n <= 6000 else np.sort(np.random.default_rng(0).choice(la.n, 6000, replace=False))
    src, idx = C.neighbor_map(la, k, sel, tree=tr)
    ref = encode_oracle_map(src, idx)
    with G.AprAccess.from_input(inp) as acc:
        got = G.neighbor_map(acc, k, torch.from_numpy(sel).cuda()).cpu().numpy()
    assert np.array_equal(got, ref)


def test_conv_is_deterministic():
    inp, la, tr = case("sphere64")
    with G.AprAccess.from_input(inp) as acc:
        x = torch.from_numpy(inp.values).cuda()
        w = torch.from_numpy(_weights(5, "restrict", la, 0)[0]).cuda()
        t1 = G.fill_tree(acc, x)
        y1 = G.conv(acc, x, t1, w, 5)
        t2 = G.fill_tree(acc, x)
        y2 = G.conv(acc, x, t2, w, 5)
        assert torch.equal(t1, t2) and torch.equal(y1, y2)


@pytest.mark.parametrize("name", ["rand16_l1", "sphere64"])
@pytest.mark.parametrize("k", [3, 5])
def test_conv_bf16_storage(name, k):
    """BF16 particle and tree storage, FP32 accumulation: within 1e-2 * M_p of
    the oracle on the BF16-rounded particle values."""
    inp, la, tr = case(name)
    w32, w64 = _weights(k, "restrict", la, 0)
    with G.AprAccess.from_input(inp) as acc:
        xb = torch.from_numpy(inp.values).cuda().to(torch.bfloat16)
        x64 = xb.float().cpu().numpy().astype(np.float64)
        ref = C.apr_conv(la, x64, w64, tree=tr)
        scale = C.apr_conv(la, np.abs(x64), np.abs(w64), tree=tr)
        t = G.fill_tree(acc, xb)
        wd = torch.from_numpy(w32).cuda()
        y32 = G.conv(acc, xb, t, wd, k, out_dtype=torch.float32).cpu().numpy()
        yb = G.conv(acc, xb, t, wd, k).float().cpu().numpy()
    assert_close_scaled(y32, ref, scale, 1e-2, "bf16 in / fp32 out")
    assert_close_scaled(yb, ref, scale, 1e-2, "bf16 in / bf16 out")


def test_rl_epilogues():
    inp, la, tr = case("sphere64")
    psf = S.gaussian_stencil(5, 1.5)
    wl = G.stencil_levels(psf, "restrict", 5, la.l_min, la.l_max)
    ref_c = C.apr_conv(la, inp.values.astype(np.float64), S.level_stencils(psf, S.RESTRICT, la.l_min, la.l_max),
                       tree=tr)
    u = np.random.default_rng(1).uniform(50, 150, la.n).astype(np.float32)
    with G.AprAccess.from_input(inp) as acc:
        x = torch.from_numpy(inp.values).cuda()
        ud = torch.from_numpy(u).cuda()
        t = G.fill_tree(acc, x)
        w = torch.from_numpy(wl).cuda()
        r = G.conv(acc, x, t, w, 5, epilogue="ratio", epi_arg=ud, eps=1e-3).cpu().numpy()
        mres = G.conv(acc, x, t, w, 5, epilogue="mul", epi_arg=ud).cpu().numpy()
    assert np.allclose(r, u / np.maximum(ref_c, 1e-3), rtol=2e-5)
    assert np.allclose(mres, ref_c * u, rtol=2e-5)


@pytest.mark.parametrize("name", ["rand33x20x70", "sphere64", "rand_long_y", "single_cell", "one_level",
                                  "dense13x11x70"])
def test_richardson_lucy_iterations_equal_the_public_steps(name):
    """Two Richardson-Lucy iterations equal, bit for bit, the same steps
    through the public calls (tree fills, the ratio and multiply epilogues),
    including an APR without tree levels (a single cell)."""
    inp, la, tr = case(name)
    psf = S.gaussian_stencil(5, 1.5)
    u = np.random.default_rng(2).uniform(50, 150, la.n).astype(np.float32)
    with G.AprAccess.from_input(inp) as acc:
        ud = torch.from_numpy(u).cuda()
        got = G.richardson_lucy(acc, ud, psf, 2)
        w = torch.from_numpy(G.stencil_levels(psf, "restrict", 5, la.l_min, la.l_max)).cuda()
        wf = torch.from_numpy(G.stencil_levels(psf, "restrict", 5, la.l_min, la.l_max, flip=True)).cuda()
        eps = float(np.float32(np.abs(u).max()) * np.float32(1e-12))
        cur = ud
        for _ in range(2):
            rho = G.conv(acc, cur, G.fill_tree(acc, cur), wf, 5, epilogue="ratio", epi_arg=ud, eps=eps)
            cur = G.conv(acc, rho, G.fill_tree(acc, rho), w, 5, epilogue="mul", epi_arg=cur)
        assert torch.equal(got, cur)


def test_validation_rejects_unbalanced_and_broken_partitions():
    from paper_2112_03592_amd._lib import AprError, APR_EUNBALANCED, APR_EPARTITION
    unb = None
    for seed in range(40):
        u = random_apr((16, 16, 16), l_min=0, seed=seed, p_refine=0.06, balanced=False)
        if not A.check_balance(linear_access(u)):
            unb = u
            break
    assert unb is not None
    with pytest.raises(AprError) as ei:
        G.AprAccess.from_input(unb)
    assert ei.value.status == APR_EUNBALANCED
    ok = random_apr((8, 8, 8), l_min=1, seed=3, p_refine=0.3)
    # a gap: drop the last particle of the finest level
    cells = {l: c.copy() for l, c in ok.cells.items()}
    top = max(l for l in cells if cells[l].shape[0])
    cells[top] = cells[top][:-1]
    from aprgen.apr_input import encode_cells
    y, e = encode_cells(ok.dims, ok.l_min, ok.l_max, cells)
    with pytest.raises(AprError) as ei:
        G.AprAccess(ok.dims, ok.l_min, ok.l_max, y, e)
    assert ei.value.status == APR_EPARTITION
    # an overlap: add the parent cell of a finest-level particle as a particle
    cells = {l: c.copy() for l, c in ok.cells.items()}
    par = cells[top][0] // 2
    cells[top - 1] = np.unique(np.concatenate([cells[top - 1], par[None]]), axis=0)
    y, e = encode_cells(ok.dims, ok.l_min, ok.l_max, cells)
    with pytest.raises(AprError) as ei:
        G.AprAccess(ok.dims, ok.l_min, ok.l_max, y, e)
    assert ei.value.status == APR_EPARTITION


# ---------------------------------------------------------------------------
# Full-size sphere field (512^3, ~6.6M particles) in the launch configuration
# the benchmark times; outputs checked on a seeded sample by keyed lookup.
# ---------------------------------------------------------------------------
@pytest.fixture(scope="module")
def sphere512():
    say("generating sphere512")
    inp = cached_sphere_apr("sphere512")
    la = linear_access(inp)
    say("oracle tree for sphere512")
    tr = A.tree_structure(la)
    tv = oracle_fill(la, tr, inp.values.astype(np.float64))
    return inp, la, tr, tv


def test_sphere512_tree_bit_exact_and_values(sphere512):
    inp, la, tr, tv = sphere512
    with G.AprAccess.from_input(inp) as acc:
        ty, te = acc.export_tree()
        assert np.array_equal(ty.astype(np.int64), tr.y_idx)
        assert np.array_equal(te.astype(np.int64), tr.xz_end)
        t = G.fill_tree(acc, torch.from_numpy(inp.values).cuda()).cpu().numpy()
    assert np.allclose(t.astype(np.float64), tv, rtol=4e-6, atol=0)


@pytest.mark.parametrize("k", [3, 5])
def test_sphere512_conv_sampled(sphere512, k):
    inp, la, tr, tv = sphere512
    say("sphere512 conv", k)
    w32 = G.stencil_levels(S.gaussian_stencil(k, 1.0), "same", k, la.l_min, la.l_max)
    smp = np.sort(np.random.default_rng(k).choice(la.n, 4096, replace=False))
    x64 = inp.values.astype(np.float64)
    ref = C.apr_conv_keyed(la, x64, w32.astype(np.float64), smp, tree=tr, tvals=tv)[:, 0]
    tva = oracle_fill(la, tr, np.abs(x64))
    scale = C.apr_conv_keyed(la, np.abs(x64), np.abs(w32.astype(np.float64)), smp, tree=tr, tvals=tva)[:, 0]
    with G.AprAccess.from_input(inp) as acc:
        x = torch.from_numpy(inp.values).cuda()
        t = G.fill_tree(acc, x)
        y = G.conv(acc, x, t, torch.from_numpy(w32).cuda(), k).cpu().numpy()
        nm = G.neighbor_map(acc, k, torch.from_numpy(smp[:512]).cuda()).cpu().numpy()
    assert_close_scaled(y[smp], ref, scale, 1e-5, f"sphere512 k={k}")
    src, idx = C.neighbor_map(la, k, smp[:512], tree=tr)
    assert np.array_equal(nm, encode_oracle_map(src, idx))


@pytest.mark.parametrize("name,k", [("sphere64", 5), ("rand33x20x70", 3), ("sphere64", 13), ("rand33x20x70", 9)])
def test_richardson_lucy_10_iterations(name, k):
    """APR Richardson-Lucy (10 iterations, restricted Gaussian PSF) against
    the FP64 oracle."""
    from oracle.rl import richardson_lucy as oracle_rl
    inp, la, tr = case(name)
    psf = S.gaussian_stencil(k, 1.5)
    u = inp.values.astype(np.float64) + 1.0
    ref = oracle_rl(la, u, psf, 10)
    with G.AprAccess.from_input(inp) as acc:
        got = G.richardson_lucy(acc, torch.from_numpy(u.astype(np.float32)).cuda(), psf, 10).cpu().numpy()
    rel = np.abs(got - ref) / np.abs(ref)
    say("rl rel err max", rel.max(), "l2", np.linalg.norm(got - ref) / np.linalg.norm(ref))
    assert rel.max() < 1e-4
