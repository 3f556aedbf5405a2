"""Pins for the oracle's APR convolution, its adjoint and APR Richardson-Lucy
(CPU only)."""
import json
import os

import numpy as np
import pytest
from scipy import ndimage

from aprgen.apr_input import CONFIGS, dense_apr, random_apr, sphere_apr
from oracle import access as A
from oracle import conv as C
from oracle.rl import richardson_lucy
from oracle.stencil import RESTRICT, SAME, flip, gaussian_stencil, level_stencils
from oracle.tree import fill_tree

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _la(inp):
    return A.LinearAccess(inp.dims, inp.l_min, inp.l_max, inp.y_idx, inp.xz_end)


def test_golden_tiny4_outputs():
    with open(os.path.join(GOLD, "tiny4.json")) as f:
        g = json.load(f)
    la = A.LinearAccess(g["dims"], g["l_min"], g["l_max"], g["y_idx"], g["xz_end"])
    x = np.array(g["values"], float)
    y = C.apr_conv(la, x, np.ones((1, 3, 3, 3)))
    for i, v in g["ones3_outputs"].items():
        assert y[int(i)] == v
    ys = C.apr_conv_keyed(la, x, np.ones((1, 3, 3, 3)), np.array([int(i) for i in g["ones3_outputs"]]))
    assert ys[:, 0].tolist() == list(g["ones3_outputs"].values())


@pytest.mark.parametrize("dims,k,seed", [((5, 6, 7), 3, 0), ((8, 4, 9), 5, 1), ((16, 16, 16), 3, 2), ((6, 6, 6), 5, 3),
                                         ((11, 9, 14), 7, 4), ((10, 13, 8), 9, 5), ((9, 17, 15), 13, 6)])
def test_all_finest_equals_pixel_correlation(dims, k, seed):
    """Section 4.1: at the finest level APR convolution is convolution of the
    reconstructed image.  An asymmetric stencil pins orientation
    (cross-correlation, zero padding)."""
    rng = np.random.default_rng(seed)
    img = rng.uniform(0.5, 2.0, size=dims)
    inp = dense_apr(dims, l_min=0, values=img.reshape(-1))
    la = _la(inp)
    w = rng.normal(size=(k, k, k))
    y = C.apr_conv(la, inp.values.astype(np.float64), w[None])
    ref = ndimage.correlate(inp.values.astype(np.float64).reshape(dims), w, mode="constant", cval=0.0)
    assert np.allclose(y, ref.reshape(-1), rtol=1e-12, atol=1e-12)


@pytest.mark.parametrize("mode", [SAME, RESTRICT])
@pytest.mark.parametrize("k", [3, 5])
def test_constant_image(mode, k):
    inp = random_apr((12, 16, 10), l_min=1, seed=11)
    la = _la(inp)
    w = level_stencils(gaussian_stencil(k, 1.0), mode, la.l_min, la.l_max)
    y = C.apr_conv(la, np.full(la.n, 2.5), w)
    lev, crd = C.particle_table(la)
    r = (k - 1) // 2
    for p in range(la.n):
        l = lev[p]
        d = A.level_dims(la.dims, la.dims_lmax, l)
        tot = 0.0
        for (oz, ox, oy) in C.taps(k):
            c = crd[p] + (oz, ox, oy)
            if (c >= 0).all() and (c < d).all():
                tot += w[l - la.l_min][oz + r, ox + r, oy + r]
        assert np.isclose(y[p], 2.5 * tot, rtol=1e-13)


def _pixel_idx(la):
    _, idx, cnt = A.pixel_level_map(la)
    assert (cnt == 1).all()
    return idx


@pytest.mark.parametrize("dims,l_min,seed,k", [((8, 8, 8), 0, 1, 3), ((16, 16, 16), 1, 2, 5), ((16, 8, 8), 1, 3, 3)])
def test_brute_force_through_pixel_reconstruction(dims, l_min, seed, k):
    """Explicit pixels: u_hat (piecewise constant) -> block means at level l
    -> correlate with w_l -> sample at the level-l particles.  Equals the
    oracle's particle/tree formulation for power-of-two images."""
    inp = random_apr(dims, l_min=l_min, seed=seed, p_refine=0.3)
    la = _la(inp)
    rng = np.random.default_rng(seed)
    x = rng.normal(size=la.n)
    W = rng.normal(size=(la.l_max - la.l_min + 1, k, k, k))
    y = C.apr_conv(la, x, W)
    u = x[_pixel_idx(la)]
    lmax = la.dims_lmax
    for l in range(la.l_min, la.l_max + 1):
        b, e = la.level_range(l)
        if b == e:
            continue
        s = 2 ** (lmax - l)
        d = A.level_dims(la.dims, lmax, l)
        ul = u.reshape(d[0], s, d[1], s, d[2], s).mean(axis=(1, 3, 5))
        ref = ndimage.correlate(ul, W[l - la.l_min], mode="constant", cval=0.0)
        c = la.cells(l)
        assert np.allclose(y[b:e], ref[c[:, 0], c[:, 1], c[:, 2]], rtol=1e-12, atol=1e-12)


def test_restricted_stencil_is_pixel_consistent():
    """Eq. restrict_stenc with R_l P_l = I: where every level-l cell of the 3^3
    coarse neighbourhood of c_p lies inside a particle at a level <= l, the
    APR output equals the mean over cell(p) of (w correlated with u_hat)."""
    inp = random_apr((16, 16, 16), l_min=1, seed=21, p_refine=0.2)
    la = _la(inp)
    rng = np.random.default_rng(0)
    x = rng.uniform(0.5, 2.0, size=la.n)
    w = rng.normal(size=(5, 5, 5))
    y = C.apr_conv(la, x, level_stencils(w, RESTRICT, la.l_min, la.l_max))
    u = x[_pixel_idx(la)]
    full = ndimage.correlate(u, w, mode="constant", cval=0.0)
    lev, crd = C.particle_table(la)
    lmax = la.dims_lmax
    checked = 0
    for l in range(la.l_min, la.l_max + 1):
        cov = A.covered_index(la, l)
        d = cov.shape
        s = 2 ** (lmax - l)
        b, e = la.level_range(l)
        for p in range(b, e):
            c = crd[p]
            ok = True
            for o in C.taps(3):
                q = c + o
                if (q >= 0).all() and (q < d).all() and cov[tuple(q)] < 0:
                    ok = False
                    break
            if not ok:
                continue
            z, xx, yy = c * s
            assert np.isclose(y[p], full[z:z + s, xx:xx + s, yy:yy + s].mean(), rtol=1e-12, atol=1e-12)
            checked += 1
    assert checked > 50


@pytest.mark.parametrize("dims,l_min,seed,k,cin,cout", [((12, 10, 16), 1, 5, 3, 1, 1), ((16, 16, 16), 0, 6, 5, 2, 3)])
def test_dense_and_keyed_formulations_agree(dims, l_min, seed, k, cin, cout):
    inp = random_apr(dims, l_min=l_min, seed=seed, p_refine=0.3)
    la = _la(inp)
    rng = np.random.default_rng(seed)
    x = rng.normal(size=(la.n, cin))
    W = rng.normal(size=(la.l_max - la.l_min + 1, cout, cin, k, k, k))
    b = rng.normal(size=cout)
    y = C.apr_conv(la, x, W, bias=b)
    smp = rng.choice(la.n, size=min(la.n, 300), replace=False)
    ys = C.apr_conv_keyed(la, x, W, smp, bias=b)
    assert np.allclose(ys, y[smp], rtol=1e-12, atol=1e-12)


def test_sphere64_keyed_matches_dense():
    inp = sphere_apr(CONFIGS["sphere64"])
    la = _la(inp)
    x = inp.values.astype(np.float64)
    w = level_stencils(gaussian_stencil(3, 1.0), SAME, la.l_min, la.l_max)
    y = C.apr_conv(la, x, w)
    smp = np.random.default_rng(0).choice(la.n, 500, replace=False)
    assert np.allclose(C.apr_conv_keyed(la, x, w, smp)[:, 0], y[smp], rtol=1e-12)


@pytest.mark.parametrize("k", [3, 5])
def test_balanced_neighbourhoods_use_three_sources(k):
    """With 26-neighbour balance every tap of a level-l particle is supplied
    by APR level l, APR level l-1 or tree level l (Section 5.2 of the GPU
    design); an unbalanced APR breaks this."""
    inp = random_apr((16, 16, 16), l_min=0, seed=9, p_refine=0.25)
    la = _la(inp)
    src, _ = C.neighbor_map(la, k, np.arange(la.n))
    assert not (src == C.SRC_FAR).any()
    bad = False
    for seed in range(30):
        u = random_apr((16, 16, 16), l_min=0, seed=seed, p_refine=0.06, balanced=False)
        lu = _la(u)
        if not A.check_balance(lu):
            s2, _ = C.neighbor_map(lu, k, np.arange(lu.n))
            bad = bool((s2 == C.SRC_FAR).any())
            if bad:
                break
    assert bad


def test_adjoint_identity_and_explicit_matrix():
    inp = random_apr((8, 8, 8), l_min=0, seed=31, p_refine=0.3)
    la = _la(inp)
    rng = np.random.default_rng(2)
    k, cin, cout = 3, 2, 2
    W = rng.normal(size=(la.l_max - la.l_min + 1, cout, cin, k, k, k))
    x = rng.normal(size=(la.n, cin))
    g = rng.normal(size=(la.n, cout))
    lhs = np.sum(C.apr_conv(la, x, W) * g)
    rhs = np.sum(x * C.apr_conv_bwd_data(la, g, W))
    assert np.isclose(lhs, rhs, rtol=1e-12)
    # explicit matrix from unit vectors, single channel
    w1 = rng.normal(size=(la.l_max - la.l_min + 1, 5, 5, 5))
    Amat = np.stack([C.apr_conv(la, np.eye(la.n)[i], w1) for i in range(la.n)], axis=1)
    g1 = rng.normal(size=la.n)
    assert np.allclose(C.apr_conv_bwd_data(la, g1, w1)[:, 0], Amat.T @ g1, rtol=1e-11, atol=1e-11)


@pytest.mark.parametrize("nw", [None, 1])
def test_weight_gradient_by_finite_differences(nw):
    inp = random_apr((8, 8, 16), l_min=1, seed=41, p_refine=0.3)
    la = _la(inp)
    rng = np.random.default_rng(3)
    k, cin, cout = 3, 2, 3
    nl = 1 if nw == 1 else la.l_max - la.l_min + 1
    W = rng.normal(size=(nl, cout, cin, k, k, k))
    x = rng.normal(size=(la.n, cin))
    g = rng.normal(size=(la.n, cout))
    dW = C.apr_conv_bwd_weight(la, x, g, k, n_wlevels=nw)
    for _ in range(3):
        E = rng.normal(size=W.shape)
        h = 1e-3
        fd = (np.sum(C.apr_conv(la, x, W + h * E) * g) - np.sum(C.apr_conv(la, x, W - h * E) * g)) / (2 * h)
        assert np.isclose(fd, np.sum(dW * E), rtol=1e-9)


def test_data_gradient_by_finite_differences_on_sphere_field():
    inp = sphere_apr(CONFIGS["sphere32"])
    la = _la(inp)
    rng = np.random.default_rng(4)
    W = rng.normal(size=(la.l_max - la.l_min + 1, 2, 1, 3, 3, 3))
    x = inp.values.astype(np.float64)
    g = rng.normal(size=(la.n, 2))
    dx = C.apr_conv_bwd_data(la, g, W)[:, 0]
    for _ in range(3):
        v = rng.normal(size=la.n)
        fd = (np.sum(C.apr_conv(la, x + v, W) * g) - np.sum(C.apr_conv(la, x - v, W) * g)) / 2
        assert np.isclose(fd, np.dot(dx, v), rtol=1e-10)


def test_rl_all_finest_equals_pixel_rl():
    dims = (10, 12, 9)
    rng = np.random.default_rng(5)
    img = rng.uniform(50, 150, size=dims)
    inp = dense_apr(dims, l_min=0, values=img.reshape(-1))
    la = _la(inp)
    psf = gaussian_stencil(5, 1.5)
    psf[0, 1, 2] += 0.01     # break symmetry so the flip matters
    psf /= psf.sum()
    got = richardson_lucy(la, inp.values.astype(np.float64), psf, 4)
    u = inp.values.astype(np.float64).reshape(dims)
    i = u.copy()
    eps = 1e-12 * np.abs(u).max()
    for _ in range(4):
        e = ndimage.convolve(i, psf, mode="constant", cval=0.0)   # i * w
        rho = u / np.maximum(e, eps)
        i = i * ndimage.correlate(rho, psf, mode="constant", cval=0.0)   # rho * w_dagger
    assert np.allclose(got, i.reshape(-1), rtol=1e-11)


def test_rl_keeps_constant_field_constant_in_the_interior():
    """A constant image is a fixed point of RL with a normalised PSF wherever
    the zero padding cannot reach.  Levels l_max-1..l_max only, so one
    convolution looks at most (r + 2) * 2 pixels beyond a particle's cell."""
    inp = random_apr((64, 64, 64), l_min=5, seed=3, p_refine=0.5)
    la = _la(inp)
    K, r = 1, 2
    out = richardson_lucy(la, np.full(la.n, 7.0), gaussian_stencil(5, 1.5), K)
    lev, crd = C.particle_table(la)
    s = 2 ** (la.dims_lmax - lev)
    lo = crd * s[:, None]
    hi = (crd + 1) * s[:, None]
    margin = 2 * K * (r + 2) * 2
    far = ((lo - margin >= 0) & (hi + margin <= 64)).all(axis=1)
    assert far.sum() > 1000
    assert np.allclose(out[far], 7.0, rtol=1e-12)
    assert not np.allclose(out[~far], 7.0, rtol=1e-3)


def test_rl_with_identity_psf_returns_input():
    inp = random_apr((16, 16, 16), l_min=1, seed=4)
    la = _la(inp)
    d = np.zeros((3, 3, 3))
    d[1, 1, 1] = 1.0
    u = inp.values.astype(np.float64)
    assert np.allclose(richardson_lucy(la, u, d, 3), u, rtol=1e-14)


def test_rl_identity_psf_from_init_closed_form():
    """With a delta PSF one step from i_0 = s gives s * (u / s)^power, and
    the all-finest power step equals the pixel recursion."""
    inp = random_apr((16, 16, 16), l_min=1, seed=4)
    la = _la(inp)
    d = np.zeros((3, 3, 3))
    d[1, 1, 1] = 1.0
    rng = np.random.default_rng(8)
    u = rng.uniform(50, 500, la.n)
    s = rng.uniform(50, 500, la.n)
    for p in (1.0, 1.7, 2.5):
        got = richardson_lucy(la, u, d, 1, init=s, power=p)
        assert np.allclose(got, s * (u / s) ** p, rtol=1e-12)


def test_rl_power_all_finest_equals_pixel_recursion():
    dims = (9, 8, 10)
    rng = np.random.default_rng(9)
    img = rng.uniform(50, 150, size=dims)
    inp = dense_apr(dims, l_min=0, values=img.reshape(-1))
    la = _la(inp)
    psf = gaussian_stencil(5, 1.5)
    psf[1, 0, 2] += 0.02
    psf /= psf.sum()
    got = richardson_lucy(la, inp.values.astype(np.float64), psf, 3, power=2.2)
    u = inp.values.astype(np.float64).reshape(dims)
    i = u.copy()
    eps = 1e-12 * np.abs(u).max()
    for _ in range(3):
        rho = u / np.maximum(ndimage.convolve(i, psf, mode="constant", cval=0.0), eps)
        i = i * ndimage.correlate(rho, psf, mode="constant", cval=0.0) ** 2.2
    assert np.allclose(got, i.reshape(-1), rtol=1e-11)


@pytest.mark.parametrize("k,seed,sep", [(7, 0, True), (9, 1, False), (13, 2, True), (13, 3, False)])
def test_large_stencils_are_level_wise_correlations(k, seed, sep):
    """Stencils above 5^3 (the line / plane decomposition of Section 7): on
    every level l, the convolution of the level-l particles equals the
    correlation of the dense level-l reconstruction V_l (Section 3.5; taps now
    reach particles two levels coarser) with w_l, sampled at the particles.
    For a separable stencil the reference is computed line by line (three 1-D
    passes), otherwise plane by plane."""
    rng = np.random.default_rng(seed)
    inp = random_apr((30, 26, 34), l_min=0, seed=(41, 42, 43, 45)[seed], p_refine=0.2)
    la = _la(inp)
    tr = A.tree_structure(la)
    x = inp.values.astype(np.float64)
    if sep:
        g = [rng.uniform(0.1, 1.0, k) for _ in range(3)]
        w = g[0][:, None, None] * g[1][None, :, None] * g[2][None, None, :]
    else:
        w = rng.normal(size=(k, k, k))
    wl = level_stencils(w, RESTRICT, la.l_min, la.l_max)
    y = np.asarray(C.apr_conv(la, x, wl, tree=tr)).reshape(-1)
    t2 = fill_tree(la, tr, x[:, None])
    for l in range(la.l_min, la.l_max + 1):
        b, e = la.level_range(l)
        if e == b:
            continue
        V = C.level_grid(la, tr, x[:, None], t2, l)[..., 0]
        W = wl[l - la.l_min]
        if sep:
            # w_l = restrict(outer product) stays an outer product: recover its factors
            i = np.unravel_index(np.argmax(np.abs(W)), W.shape)
            fz, fx, fy = W[:, i[1], i[2]], W[i[0], :, i[2]], W[i[0], i[1], :]
            ref = ndimage.correlate1d(V, fz, axis=0, mode="constant")
            ref = ndimage.correlate1d(ref, fx / fx[i[1]], axis=1, mode="constant")
            ref = ndimage.correlate1d(ref, fy / fy[i[2]], axis=2, mode="constant")
        else:
            r = k // 2
            ref = np.zeros_like(V)
            for dz in range(-r, r + 1):
                plane = ndimage.correlate(V, W[dz + r][None], mode="constant")
                src = slice(max(0, dz), V.shape[0] + min(0, dz))
                dst = slice(max(0, -dz), V.shape[0] - max(0, dz))
                ref[dst] += plane[src]
        c = la.cells(l)
        want = ref[c[:, 0], c[:, 1], c[:, 2]]
        assert np.allclose(y[b:e], want, rtol=1e-10, atol=1e-10 * np.abs(want).max())
    if k >= 9:
        src, _ = C.neighbor_map(la, k, np.arange(la.n), tree=tr)
        assert (src == C.SRC_FAR).any(), "no tap reached a particle two levels coarser"
