"""Per-level stencils.  Test infrastructure only.

A stencil ``w`` of side k (odd) is an array [..., k, k, k] indexed by
(dz+r, dx+r, dy+r), r = (k-1)/2; it multiplies the value at offset (dz,dx,dy)
from the output cell (cross-correlation, as in Section 4.1 where the filter is
centred on each particle).
"""
from __future__ import annotations

import itertools

import numpy as np

SAME, RESTRICT, ADAPTIVE = "same", "restrict", "adaptive"


def gaussian_stencil(k: int, sigma: float) -> np.ndarray:
    """Normalised separable Gaussian, FP64 [k, k, k]."""
    t = np.arange(k) - (k - 1) / 2.0
    g = np.exp(-0.5 * (t / sigma) ** 2)
    g3 = g[:, None, None] * g[None, :, None] * g[None, None, :]
    return g3 / g3.sum()


def _axis_counts(s: int, r: int) -> np.ndarray:
    """n[J + r, t + r] = #{a in [0, s) : floor((a + t) / s) == J}."""
    n = np.zeros((2 * r + 1, 2 * r + 1))
    for t in range(-r, r + 1):
        for a in range(s):
            J = (a + t) // s
            if abs(J) > r:
                raise ValueError("restricted stencil exceeds the stencil support")
            n[J + r, t + r] += 1
    return n


def restrict_stencil(w: np.ndarray, s: int) -> np.ndarray:
    """Restricted stencil w_l for coarsening factor s (Eq. restrict_stenc).

    With R_l the block average over s^3 pixels and P_l the piecewise-constant
    prolongation, K_{w_l} = R_l K_w P_l.  Applied to a coarse signal u at coarse
    cell I this reads  s^-3 sum_{a in [0,s)^3} sum_t w[t] u(I + floor((a+t)/s)),
    i.e. (Section 4.2) w_l averages the fine stencil applied at every position
    inside the coarse cell:
        w_l[J] = s^-3 sum_t w[t] #{a in [0,s)^3 : floor((a+t)/s) == J}.
    The count of positions a is a product of per-axis counts because both the
    condition and the range of a split over the axes.  The result is embedded,
    centred, in the same k^3 support as w (for s >= 2 and k <= 5 its non-zeros
    lie in [-1, 1]^3).  Leading axes are carried.
    """
    w = np.asarray(w, np.float64)
    k = w.shape[-1]
    r = (k - 1) // 2
    if s == 1:
        return w.copy()
    n = _axis_counts(s, r)
    # sum over t of w[t] times the product of the per-axis counts
    return np.einsum("ai,bj,ck,...ijk->...abc", n, n, n, w) / float(s) ** 3


def restrict_stencil_enumerated(w: np.ndarray, s: int) -> np.ndarray:
    """The same restriction by enumerating every position a in [0, s)^3
    (cross-check for small s)."""
    w = np.asarray(w, np.float64)
    k = w.shape[-1]
    r = (k - 1) // 2
    out = np.zeros_like(w)
    for t in itertools.product(range(-r, r + 1), repeat=3):
        wt = w[(...,) + tuple(ti + r for ti in t)]
        for a in itertools.product(range(s), repeat=3):
            J = tuple((ai + ti) // s for ai, ti in zip(a, t))
            out[(...,) + tuple(j + r for j in J)] += wt / s ** 3
    return out


def level_stencils(w: np.ndarray, mode: str, l_min: int, l_max: int) -> np.ndarray:
    """Stack of per-level stencils [l_max-l_min+1, ..., k, k, k] for levels
    l_min..l_max.

    * same:     w_l = w.
    * restrict: w_l = restrict_stencil(w, 2**(l_max-l))  (Section 4.2).
    * adaptive: w_l = 2**-(l_max-l) * w  (Eq. adapt_grad).
    """
    w = np.asarray(w, np.float64)
    out = []
    for l in range(l_min, l_max + 1):
        s = 2 ** (l_max - l)
        if mode == SAME:
            out.append(w.copy())
        elif mode == RESTRICT:
            out.append(restrict_stencil(w, s))
        elif mode == ADAPTIVE:
            out.append(w / s)
        else:
            raise ValueError(mode)
    return np.stack(out)


def flip(w: np.ndarray) -> np.ndarray:
    """w-dagger: elements reversed in each spatial dimension (Section 6.2)."""
    return np.ascontiguousarray(np.asarray(w)[..., ::-1, ::-1, ::-1])
