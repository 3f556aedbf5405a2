"""Pins of the oracle's resolution-adaptive gradient magnitude (Section 4.3,
Eq. adapt_grad, Sobel filters): an all-finest APR against scipy's pixel
correlation, and a linear ramp on a coarse level, where the level-scaled
stencils give the ramp's slope exactly."""
import numpy as np
from scipy import ndimage

from aprgen.apr_input import dense_apr, random_apr, sobel_stencils
from oracle import access as A
from oracle import conv as C
from oracle import stencil as S


def _la(inp):
    return A.LinearAccess(inp.dims, inp.l_min, inp.l_max, inp.y_idx, inp.xz_end)


def test_all_finest_equals_pixel_sobel():
    inp = dense_apr((12, 14, 10), l_min=1, seed=3)
    la = _la(inp)
    w3 = S.level_stencils(sobel_stencils(), S.ADAPTIVE, la.l_min, la.l_max)
    got = C.gradient_magnitude(la, inp.values, w3)
    img = inp.values.astype(np.float64).reshape(inp.dims)
    ref = np.sqrt(sum(ndimage.correlate(img, w, mode="constant") ** 2 for w in sobel_stencils()))
    assert np.allclose(got, ref.reshape(-1), rtol=1e-12, atol=1e-12)


def test_linear_ramp_on_a_coarse_level():
    a, b, c = 0.7, -1.3, 2.1
    inp = random_apr((32, 32, 32), l_min=3, seed=4, p_refine=0.0)   # every particle at level 3
    la = _la(inp)
    assert la.level_range(3) == (0, la.n)
    s = 2 ** (la.l_max - 3)
    cells = la.cells(3).astype(np.float64)
    centre = cells * s + s / 2.0
    x = a * centre[:, 0] + b * centre[:, 1] + c * centre[:, 2]
    w3 = S.level_stencils(sobel_stencils(), S.ADAPTIVE, la.l_min, la.l_max)
    got = C.gradient_magnitude(la, x, w3)
    d = 32 // s                                    # cells per axis at level 3
    inner = np.all((cells >= 1) & (cells <= d - 2), axis=1)
    assert inner.sum() > 0
    assert np.allclose(got[inner], np.sqrt(a * a + b * b + c * c), rtol=1e-12)
    # the same stencils without the level scaling give s times the slope
    w_same = S.level_stencils(sobel_stencils(), S.SAME, la.l_min, la.l_max)
    assert np.allclose(C.gradient_magnitude(la, x, w_same)[inner], s * np.sqrt(a * a + b * b + c * c), rtol=1e-12)


def test_keyed_equals_dense():
    inp = random_apr((20, 18, 24), l_min=1, seed=5, p_refine=0.3)
    la = _la(inp)
    w3 = S.level_stencils(sobel_stencils(), S.ADAPTIVE, la.l_min, la.l_max)
    full = C.gradient_magnitude(la, inp.values, w3)
    smp = np.arange(0, la.n, 7)
    assert np.allclose(C.gradient_magnitude(la, inp.values, w3, sample=smp), full[smp], rtol=1e-12, atol=1e-12)
