"""APR convolution (Section 4.1) and its adjoint, in FP64.  Test
infrastructure only.

Notation.  Particle values x are [N_p, C_in] (or [N_p]); per-level weights W
are [n_levels, C_out, C_in, k, k, k] (or [n_levels, k, k, k] for one channel,
or a leading axis of 1 for one stencil shared by every level); level index
``l - l_min``.  For a particle p at level l and cell c_p

    Y[p, co] = b[co] + sum_ci sum_{o in [-r, r]^3} W_l[co, ci, o] * V_l[ci](c_p + o)

where V_l is the isotropic reconstruction at level l (Section 3.5):
  * a cell inside a particle at level <= l takes that particle's value
    (piecewise-constant reconstruction, Section 2.2),
  * otherwise the cell contains finer particles and takes the tree value,
  * outside the image it is 0.  The paper pads at the image edge (Section
    5.1, CPU buffer) without naming the padding; reading: zeros.
"""
from __future__ import annotations

import itertools
from typing import Optional, Tuple

import numpy as np

from .access import LinearAccess, covered_index, level_dims, tree_levels, tree_structure
from .tree import CHILD_OFFSETS, fill_tree

SRC_PAD, SRC_SAME, SRC_COARSER, SRC_TREE, SRC_FAR = 0, 1, 2, 3, 4


def _as2d(x):
    x = np.asarray(x, np.float64)
    return x[:, None] if x.ndim == 1 else x


def norm_weights(w, n_levels: int) -> np.ndarray:
    w = np.asarray(w, np.float64)
    if w.ndim == 4:
        w = w[:, None, None]
    if w.shape[0] == 1 and n_levels > 1:
        w = np.repeat(w, n_levels, axis=0)
    if w.shape[0] != n_levels:
        raise ValueError("weights need one stencil per level or one shared stencil")
    return w


def taps(k: int):
    r = (k - 1) // 2
    return list(itertools.product(range(-r, r + 1), repeat=3))


def particle_table(apr: LinearAccess) -> Tuple[np.ndarray, np.ndarray]:
    """(level, (z, x, y)) of every particle, in storage order."""
    lv, cs = [], []
    for l in range(apr.l_min, apr.l_max + 1):
        c = apr.cells(l)
        lv.append(np.full(c.shape[0], l, np.int64))
        cs.append(c)
    return np.concatenate(lv), np.concatenate(cs)


# ---------------------------------------------------------------------------
# Level-l reconstruction
# ---------------------------------------------------------------------------

def level_grid(apr: LinearAccess, tree: LinearAccess, x2: np.ndarray, t2: np.ndarray, l: int) -> np.ndarray:
    """Dense V_l [D_z, D_x, D_y, C] (Section 3.5, both cases).  Small images."""
    d = level_dims(apr.dims, apr.dims_lmax, l)
    C = x2.shape[1]
    V = np.full(d + (C,), np.nan)
    cov = covered_index(apr, l)
    m = cov >= 0
    V[m] = x2[cov[m]]
    t_lo, t_hi = tree_levels(apr)
    if t_lo <= l <= t_hi:
        c = tree.cells(l)
        b, e = tree.level_range(l)
        V[c[:, 0], c[:, 1], c[:, 2]] = t2[b:e]
    if np.isnan(V).any():
        raise AssertionError("a level-l cell is neither inside a particle nor a tree node")
    return V


def value_at(apr: LinearAccess, tree: LinearAccess, x2, t2, l: int, cells: np.ndarray):
    """V_l at arbitrary cells by keyed lookup (no dense grids).

    Returns (values [n, C], source [n], index [n]); source is SRC_PAD outside
    the image, SRC_SAME / SRC_COARSER / SRC_FAR for a particle at level l /
    l-1 / coarser, SRC_TREE for a tree node at level l.
    """
    n = cells.shape[0]
    C = x2.shape[1]
    d = level_dims(apr.dims, apr.dims_lmax, l)
    vals = np.zeros((n, C))
    src = np.full(n, SRC_PAD, np.int64)
    idx = np.full(n, -1, np.int64)
    inside = (cells >= 0).all(axis=1) & (cells[:, 0] < d[0]) & (cells[:, 1] < d[1]) & (cells[:, 2] < d[2])
    todo = inside.copy()
    for lq in range(min(l, apr.l_max), apr.l_min - 1, -1):
        if not todo.any():
            break
        q = cells[todo] >> (l - lq)
        ip = apr.lookup(lq, q)
        hit = ip >= 0
        sel = np.nonzero(todo)[0][hit]
        vals[sel] = x2[ip[hit]]
        idx[sel] = ip[hit]
        src[sel] = SRC_SAME if lq == l else (SRC_COARSER if lq == l - 1 else SRC_FAR)
        todo[sel] = False
    if todo.any():
        t_lo, t_hi = tree_levels(apr)
        it = tree.lookup(l, cells[todo]) if t_lo <= l <= t_hi else np.full(int(todo.sum()), -1)
        if (it < 0).any():
            raise AssertionError("cell neither inside a particle nor a tree node")
        sel = np.nonzero(todo)[0]
        vals[sel] = t2[it]
        idx[sel] = it
        src[sel] = SRC_TREE
    return vals, src, idx


# ---------------------------------------------------------------------------
# Forward
# ---------------------------------------------------------------------------

def apr_conv(apr: LinearAccess, x, w, bias=None, tree: Optional[LinearAccess] = None,
             tvals=None) -> np.ndarray:
    """APR convolution via dense per-level reconstruction (small images)."""
    tree = tree_structure(apr) if tree is None else tree
    x2 = _as2d(x)
    t2 = _as2d(fill_tree(apr, tree, x2)) if tvals is None else _as2d(tvals)
    nl = apr.l_max - apr.l_min + 1
    W = norm_weights(w, nl)
    k = W.shape[-1]
    r = (k - 1) // 2
    C_out = W.shape[1]
    y = np.zeros((apr.n, C_out))
    for l in range(apr.l_min, apr.l_max + 1):
        b, e = apr.level_range(l)
        if b == e:
            continue
        V = level_grid(apr, tree, x2, t2, l)
        Vp = np.pad(V, ((r, r), (r, r), (r, r), (0, 0)))
        c = apr.cells(l)
        acc = np.zeros((e - b, C_out))
        Wl = W[l - apr.l_min]
        for (dz, dx, dy) in taps(k):
            v = Vp[c[:, 0] + dz + r, c[:, 1] + dx + r, c[:, 2] + dy + r]
            acc += v @ Wl[:, :, dz + r, dx + r, dy + r].T
        y[b:e] = acc
    if bias is not None:
        y += np.asarray(bias, np.float64)[None, :]
    return y[:, 0] if (np.asarray(w).ndim == 4 and np.asarray(x).ndim == 1) else y


def apr_conv_keyed(apr: LinearAccess, x, w, sample: np.ndarray, bias=None,
                   tree: Optional[LinearAccess] = None, tvals=None) -> np.ndarray:
    """APR convolution at the particles ``sample`` by keyed lookup of every
    tap; usable on large APRs.  Same definition as ``apr_conv``."""
    tree = tree_structure(apr) if tree is None else tree
    x2 = _as2d(x)
    t2 = _as2d(fill_tree(apr, tree, x2)) if tvals is None else _as2d(tvals)
    nl = apr.l_max - apr.l_min + 1
    W = norm_weights(w, nl)
    k = W.shape[-1]
    r = (k - 1) // 2
    lev, crd = particle_table(apr)
    sample = np.asarray(sample, np.int64)
    out = np.zeros((sample.shape[0], W.shape[1]))
    for l in np.unique(lev[sample]):
        sel = np.nonzero(lev[sample] == l)[0]
        c = crd[sample[sel]]
        Wl = W[l - apr.l_min]
        acc = np.zeros((sel.shape[0], W.shape[1]))
        for (dz, dx, dy) in taps(k):
            v, _, _ = value_at(apr, tree, x2, t2, int(l), c + np.array([dz, dx, dy]))
            acc += v @ Wl[:, :, dz + r, dx + r, dy + r].T
        out[sel] = acc
    if bias is not None:
        out += np.asarray(bias, np.float64)[None, :]
    return out


def neighbor_map(apr: LinearAccess, k: int, sample: np.ndarray, tree: Optional[LinearAccess] = None):
    """For every sampled particle and tap (tap order dz, dx, dy ascending):
    (source, index) of the element supplying V_l(c_p + o)."""
    tree = tree_structure(apr) if tree is None else tree
    lev, crd = particle_table(apr)
    sample = np.asarray(sample, np.int64)
    T = taps(k)
    src = np.zeros((sample.shape[0], len(T)), np.int64)
    idx = np.zeros((sample.shape[0], len(T)), np.int64)
    x2 = np.zeros((apr.n, 1))
    t2 = np.zeros((tree.n, 1))
    for j, o in enumerate(T):
        for l in np.unique(lev[sample]):
            sel = np.nonzero(lev[sample] == l)[0]
            _, s, i = value_at(apr, tree, x2, t2, int(l), crd[sample[sel]] + np.array(o))
            src[sel, j] = s
            idx[sel, j] = i
    return src, idx


# ---------------------------------------------------------------------------
# Adjoint
# ---------------------------------------------------------------------------

def apr_conv_bwd_data(apr: LinearAccess, dy, w, tree: Optional[LinearAccess] = None) -> np.ndarray:
    """dX = A^T dY for the linear map X -> Y (bias excluded).  Small images.

    Transposes each step of the forward definition:
      1. tap scatter: D_l(c_p + o) += W_l[o]^T dY[p] for in-image cells;
      2. level routing, coarse to fine: a cell inside a particle q at a level
         <= l sends D_l(c) to dX[q] (adjoint of the piecewise-constant copy);
         a tree node sends D_l(c)/|children| to each child at level l+1
         (adjoint of the child mean), which is routed in turn.
    """
    tree = tree_structure(apr) if tree is None else tree
    g = _as2d(dy)
    nl = apr.l_max - apr.l_min + 1
    W = norm_weights(w, nl)
    k = W.shape[-1]
    r = (k - 1) // 2
    C_in = W.shape[2]
    lmax = apr.dims_lmax
    dx = np.zeros((apr.n, C_in))
    t_lo, t_hi = tree_levels(apr)
    carry = None
    for l in range(apr.l_min, apr.l_max + 1):
        d = level_dims(apr.dims, lmax, l)
        D = np.zeros(d + (C_in,))
        b, e = apr.level_range(l)
        if e > b:
            Dp = np.zeros((d[0] + 2 * r, d[1] + 2 * r, d[2] + 2 * r, C_in))
            c = apr.cells(l)
            Wl = W[l - apr.l_min]
            for (oz, ox, oy) in taps(k):
                Dp[c[:, 0] + oz + r, c[:, 1] + ox + r, c[:, 2] + oy + r] += g[b:e] @ Wl[:, :, oz + r, ox + r, oy + r]
            D += Dp[r:r + d[0], r:r + d[1], r:r + d[2]]
        if carry is not None:
            D += carry
        cov = covered_index(apr, l)
        m = cov >= 0
        np.add.at(dx, cov[m], D[m])
        carry = None
        if l + 1 <= apr.l_max and t_lo <= l <= t_hi:
            dn = level_dims(apr.dims, lmax, l + 1)
            carry = np.zeros(dn + (C_in,))
            nodes = tree.cells(l)
            nch = np.zeros(nodes.shape[0])
            for off in CHILD_OFFSETS:
                ch = nodes * 2 + np.asarray(off)
                nch += (ch[:, 0] < dn[0]) & (ch[:, 1] < dn[1]) & (ch[:, 2] < dn[2])
            share = D[nodes[:, 0], nodes[:, 1], nodes[:, 2]] / nch[:, None]
            for off in CHILD_OFFSETS:
                ch = nodes * 2 + np.asarray(off)
                ok = (ch[:, 0] < dn[0]) & (ch[:, 1] < dn[1]) & (ch[:, 2] < dn[2])
                carry[ch[ok, 0], ch[ok, 1], ch[ok, 2]] = share[ok]
    return dx


def apr_conv_bwd_weight(apr: LinearAccess, x, dy, k: int, n_wlevels: Optional[int] = None,
                        tree: Optional[LinearAccess] = None, tvals=None) -> np.ndarray:
    """dW_l[co, ci, o] = sum_{p at level l} dY[p, co] V_l[ci](c_p + o).
    With one shared stencil (n_wlevels == 1) the levels are summed.  ``tvals``
    (tree values of x, e.g. as stored in a narrower type) replaces the FP64
    fill when given."""
    tree = tree_structure(apr) if tree is None else tree
    x2 = _as2d(x)
    g = _as2d(dy)
    t2 = _as2d(fill_tree(apr, tree, x2)) if tvals is None else _as2d(tvals)
    r = (k - 1) // 2
    nl = apr.l_max - apr.l_min + 1
    dW = np.zeros((nl, g.shape[1], x2.shape[1], k, k, k))
    for l in range(apr.l_min, apr.l_max + 1):
        b, e = apr.level_range(l)
        if e == b:
            continue
        V = level_grid(apr, tree, x2, t2, l)
        Vp = np.pad(V, ((r, r), (r, r), (r, r), (0, 0)))
        c = apr.cells(l)
        for (oz, ox, oy) in taps(k):
            v = Vp[c[:, 0] + oz + r, c[:, 1] + ox + r, c[:, 2] + oy + r]
            dW[l - apr.l_min, :, :, oz + r, ox + r, oy + r] = g[b:e].T @ v
    if n_wlevels == 1:
        dW = dW.sum(axis=0, keepdims=True)
    return dW


def abs_scale(apr: LinearAccess, x, w, tree=None) -> np.ndarray:
    """M_p = sum_o |W_l[o]| |V_l(c_p+o)| bounded above by the convolution of
    |x| with |W| (tree values of |x| dominate |tree values of x|)."""
    return apr_conv(apr, np.abs(np.asarray(x, np.float64)), np.abs(np.asarray(w, np.float64)), tree=tree)


def gradient_magnitude(apr: LinearAccess, x, w3, tree: Optional[LinearAccess] = None,
                       sample: Optional[np.ndarray] = None) -> np.ndarray:
    """|grad| from three stencils per level (Section 4.3, Eq. adapt_grad, with
    the per-level stencils w3 [n_levels or 1, 3, k, k, k]): the square root of
    the sum of the squares of the three APR convolutions; at the particles
    ``sample`` by keyed lookup when given."""
    w3 = np.asarray(w3, np.float64)
    tree = tree_structure(apr) if tree is None else tree
    x1 = np.asarray(x, np.float64).reshape(-1)
    tv = fill_tree(apr, tree, x1)
    sq = 0.0
    for j in range(3):
        wj = w3[:, j]
        if sample is None:
            g = apr_conv(apr, x1, wj, tree=tree, tvals=tv)
        else:
            g = apr_conv_keyed(apr, x1, wj, sample, tree=tree, tvals=tv)[:, 0]
        sq = sq + np.asarray(g).reshape(-1) ** 2
    return np.sqrt(sq)
