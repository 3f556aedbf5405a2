"""APR Richardson-Lucy deconvolution (Section 6.2).  Test infrastructure only.

i_{k+1} = i_k * ((u / (i_k conv w)) conv w_dagger), elementwise products and
quotients, with convolution replaced by APR convolution and the PSF w
restricted to every level (Eq. restrict_stenc).  Convolution with w equals
cross-correlation with the flipped stencil; convolution with the flipped PSF
w_dagger equals cross-correlation with w.  The paper gives neither the initial
estimate nor a guard for the quotient; readings: i_0 = u (unless an initial
estimate is passed) and the denominator is clamped below at
eps = 1e-12 * max|u|.
"""
from __future__ import annotations

import numpy as np

from .access import LinearAccess, tree_structure
from .conv import apr_conv
from .stencil import RESTRICT, flip, level_stencils


def richardson_lucy(apr: LinearAccess, u, psf, n_iter: int, eps_rel: float = 1e-12, init=None,
                    power: float = 1.0):
    """n_iter updates from i_0 = u (or ``init``).  ``power`` != 1 raises the
    multiplicative correction to that power (an over-relaxed variant used by
    the surrogate; not in the paper)."""
    tree = tree_structure(apr)
    u = np.asarray(u, np.float64)
    w_levels = level_stencils(psf, RESTRICT, apr.l_min, apr.l_max)
    wf_levels = level_stencils(flip(psf), RESTRICT, apr.l_min, apr.l_max)
    eps = eps_rel * float(np.max(np.abs(u))) if u.size else 0.0
    i = u.copy() if init is None else np.asarray(init, np.float64).copy()
    for _ in range(n_iter):
        e = apr_conv(apr, i, wf_levels, tree=tree)
        rho = u / np.maximum(e, eps)
        c = apr_conv(apr, rho, w_levels, tree=tree)
        i = i * (c if power == 1.0 else np.maximum(c, 0.0) ** power)
    return i
