"""Pins for the oracle's stencil restriction and tree values (CPU only)."""
import itertools

import numpy as np
import pytest

from aprgen.apr_input import random_apr
from oracle import access as A
from oracle.stencil import (ADAPTIVE, RESTRICT, SAME, flip, gaussian_stencil,
                            level_stencils, restrict_stencil, restrict_stencil_enumerated)
from oracle.tree import fill_tree


def test_restricted_gaussian_hand_value():
    # 3-tap normalised Gaussian (sigma = 1) restricted by s = 2: per axis
    # w_l = [w1/2, w0 + w1, w1/2] (hand evaluation of the averaging rule);
    # numerically [0.1370, 0.7259, 0.1370].
    g = np.exp(-0.5 * np.array([1.0, 0.0, 1.0]))
    g /= g.sum()
    v = np.array([g[0] / 2, g[1] + g[0], g[0] / 2])
    assert np.allclose(v, [0.1370, 0.7259, 0.1370], atol=5e-5)
    wl = restrict_stencil(gaussian_stencil(3, 1.0), 2)
    assert np.allclose(wl, np.einsum("i,j,k->ijk", v, v, v), atol=1e-15, rtol=0)


def _explicit_restriction(w, s, m):
    """R K P on a periodic coarse grid of m^3 cells; returns the stencil seen
    by coarse cell 0 (row 0 of the coarse operator), as a k^3 array."""
    k = w.shape[0]
    r = (k - 1) // 2
    n = m * s
    fine = list(itertools.product(range(n), repeat=3))
    fidx = {c: i for i, c in enumerate(fine)}
    coarse = list(itertools.product(range(m), repeat=3))
    P = np.zeros((n ** 3, m ** 3))
    for i, c in enumerate(fine):
        P[i, coarse.index(tuple(ci // s for ci in c))] = 1.0
    R = P.T / s ** 3
    K = np.zeros((n ** 3, n ** 3))
    for i, c in enumerate(fine):
        for t in itertools.product(range(-r, r + 1), repeat=3):
            j = fidx[tuple((ci + ti) % n for ci, ti in zip(c, t))]
            K[i, j] += w[t[0] + r, t[1] + r, t[2] + r]
    Kc = R @ K @ P
    near = {tuple(j % m for j in J) for J in itertools.product((-1, 0, 1), repeat=3)}
    for col, c in enumerate(coarse):
        if c not in near:
            assert abs(Kc[0, col]) < 1e-14   # nothing reaches beyond the 3^3 coarse neighbourhood
    out = np.zeros((k, k, k))
    for J in itertools.product(range(-r, r + 1), repeat=3):
        col = coarse.index(tuple(j % m for j in J))
        out[J[0] + r, J[1] + r, J[2] + r] = Kc[0, col] if max(abs(j) for j in J) <= 1 else 0.0
    return out


@pytest.mark.parametrize("k,s,m", [(3, 2, 4), (5, 2, 4), (3, 4, 3), (5, 4, 3)])
def test_restriction_equals_explicit_RKP(k, s, m):
    rng = np.random.default_rng(k * 10 + s)
    w = rng.normal(size=(k, k, k))
    ref = _explicit_restriction(w, s, m)
    got = restrict_stencil(w, s)
    assert np.allclose(got, ref, atol=1e-13, rtol=0)
    assert np.allclose(restrict_stencil_enumerated(w, s), ref, atol=1e-13, rtol=0)


def test_restriction_invariants():
    rng = np.random.default_rng(0)
    for k in (3, 5):
        w = rng.normal(size=(k, k, k))
        for s in (2, 4, 8):
            wl = restrict_stencil(w, s)
            assert np.isclose(wl.sum(), w.sum(), atol=1e-12)
            assert np.allclose(restrict_stencil(flip(w), s), flip(wl), atol=1e-13)
            r = (k - 1) // 2
            if k == 5:
                assert np.all(wl[[0, 4]] == 0) and np.all(wl[:, [0, 4]] == 0) and np.all(wl[:, :, [0, 4]] == 0)
        assert np.allclose(restrict_stencil(restrict_stencil(w, 2), 2), restrict_stencil(w, 4), atol=1e-13)
    g = gaussian_stencil(5, 1.5)
    assert np.allclose(restrict_stencil(g, 2), flip(restrict_stencil(g, 2)), atol=1e-15)


def test_level_stencil_modes():
    w = gaussian_stencil(3, 1.0)
    same = level_stencils(w, SAME, 2, 5)
    ada = level_stencils(w, ADAPTIVE, 2, 5)
    res = level_stencils(w, RESTRICT, 2, 5)
    assert same.shape == (4, 3, 3, 3)
    for i, l in enumerate(range(2, 6)):
        assert np.array_equal(same[i], w)
        assert np.allclose(ada[i], w * 2.0 ** -(5 - l))
    assert np.array_equal(res[-1], w)


def _pixel_reconstruction(la):
    """Piecewise-constant reconstruction u_hat at pixel resolution (Section 2.2)."""
    _, idx, cnt = A.pixel_level_map(la)
    assert (cnt == 1).all()
    return idx


@pytest.mark.parametrize("dims,l_min,seed", [((8, 8, 8), 0, 1), ((16, 16, 16), 1, 2), ((16, 8, 4), 0, 3)])
def test_tree_values_are_block_means_of_reconstruction(dims, l_min, seed):
    inp = random_apr(dims, l_min=l_min, seed=seed, p_refine=0.25)
    la = A.LinearAccess(inp.dims, inp.l_min, inp.l_max, inp.y_idx, inp.xz_end)
    tr = A.tree_structure(la)
    x = inp.values.astype(np.float64)
    t = fill_tree(la, tr, x)
    u = x[_pixel_reconstruction(la)]
    for L in range(tr.l_min, tr.l_max + 1):
        s = 2 ** (la.dims_lmax - L)
        c = tr.cells(L)
        b, e = tr.level_range(L)
        for j in range(c.shape[0]):
            z, xx, y = c[j] * s
            blk = u[z:z + s, xx:xx + s, y:y + s]
            assert np.isclose(t[b + j], blk.mean(), rtol=1e-13, atol=0)


def test_tree_fill_constant_and_linear():
    inp = random_apr((12, 9, 10), l_min=1, seed=7)
    la = A.LinearAccess(inp.dims, inp.l_min, inp.l_max, inp.y_idx, inp.xz_end)
    tr = A.tree_structure(la)
    assert np.allclose(fill_tree(la, tr, np.full(la.n, 3.25)), 3.25, rtol=1e-15)
    rng = np.random.default_rng(1)
    a, b = rng.normal(size=la.n), rng.normal(size=la.n)
    assert np.allclose(fill_tree(la, tr, 2 * a - b), 2 * fill_tree(la, tr, a) - fill_tree(la, tr, b), atol=1e-13)
