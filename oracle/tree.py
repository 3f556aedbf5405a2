"""APR tree values (Section 3.4): every interior node holds the average of its
children, filled level by level from the finest.  Test infrastructure only."""
from __future__ import annotations

import itertools

import numpy as np

from .access import LinearAccess, level_dims, tree_levels

CHILD_OFFSETS = list(itertools.product((0, 1), repeat=3))


def fill_tree(apr: LinearAccess, tree: LinearAccess, x: np.ndarray, store=None) -> np.ndarray:
    """Tree values in FP64.

    ``x`` is [N_p] or [N_p, C].  For a node c at level L the value is the mean,
    over the children c' of c that lie in the image, of V_{L+1}(c'): the value
    of the particle at (L+1, c') if there is one, else the value of the tree
    node (L+1, c').  Section 2.3 and Section 3.4 define coarse values by
    average downsampling; at the image boundary a node may have fewer than
    eight children and the mean runs over the children that exist.

    ``store(sums, counts)``, when given, returns the stored value of each
    node of a level from its children's sum and count (a storage format:
    the next coarser level averages the stored values); by default the
    FP64 mean.
    """
    squeeze = x.ndim == 1
    xv = np.asarray(x, np.float64).reshape(x.shape[0], -1)
    C = xv.shape[1]
    t = np.zeros((tree.n, C), np.float64)
    t_lo, t_hi = tree_levels(apr)
    lmax = apr.dims_lmax
    for L in range(t_hi, t_lo - 1, -1):
        nodes = tree.cells(L)
        b, e = tree.level_range(L)
        if nodes.shape[0] == 0:
            continue
        dch = level_dims(apr.dims, lmax, L + 1)
        acc = np.zeros((nodes.shape[0], C), np.float64)
        cnt = np.zeros(nodes.shape[0], np.int64)
        for off in CHILD_OFFSETS:
            ch = nodes * 2 + np.asarray(off)
            inside = (ch[:, 0] < dch[0]) & (ch[:, 1] < dch[1]) & (ch[:, 2] < dch[2])
            ip = apr.lookup(L + 1, ch)
            it = tree.lookup(L + 1, ch) if L + 1 <= t_hi else np.full(ch.shape[0], -1)
            if np.any((ip >= 0) & (it >= 0)):
                raise AssertionError("a cell is both a particle and a tree node")
            if np.any(inside & (ip < 0) & (it < 0)):
                raise AssertionError("an in-image child of a tree node is neither particle nor node")
            v = np.zeros((nodes.shape[0], C))
            v[ip >= 0] = xv[ip[ip >= 0]]
            v[it >= 0] = t[it[it >= 0]]
            acc += v
            cnt += ((ip >= 0) | (it >= 0))
        t[b:e] = acc / cnt[:, None] if store is None else store(acc, cnt[:, None])
    return t[:, 0] if squeeze else t
