"""Shared helpers of the GPU parity tests: seeded cases and the comparison
rules.  Every expected value comes from the FP64 oracle on the same inputs."""
from __future__ import annotations

import numpy as np

from aprgen.apr_input import CONFIGS, cached_sphere_apr, dense_apr, random_apr, sphere_apr
from oracle import access as A

# (name, builder) pairs of small cases the oracle handles in seconds; they span
# several 4x4 tiles, ragged tails in z/x/y, non-power-of-two images, a single
# cell, one level only, and the 64^3 sphere field.
SMALL_CASES = {
    "rand8_l0": lambda: random_apr((8, 8, 8), l_min=0, seed=1, p_refine=0.3),
    "rand16_l1": lambda: random_apr((16, 16, 16), l_min=1, seed=2, p_refine=0.25),
    "rand9x12x7": lambda: random_apr((9, 12, 7), l_min=1, seed=3, p_refine=0.3),
    "rand5x16x3": lambda: random_apr((5, 16, 3), l_min=0, seed=4, p_refine=0.5),
    "rand33x20x70": lambda: random_apr((33, 20, 70), l_min=2, seed=5, p_refine=0.2),
    "rand_long_y": lambda: random_apr((6, 7, 300), l_min=3, seed=6, p_refine=0.3),
    "single_cell": lambda: random_apr((1, 1, 1), l_min=0, seed=7),
    "one_level": lambda: random_apr((12, 10, 9), l_min=4, seed=8, p_refine=0.0),
    "dense13x11x70": lambda: dense_apr((13, 11, 70), l_min=1, seed=9),
    "sphere32": lambda: sphere_apr(CONFIGS["sphere32"]),
    "sphere64": lambda: sphere_apr(CONFIGS["sphere64"]),
}


def linear_access(inp) -> A.LinearAccess:
    return A.LinearAccess(inp.dims, inp.l_min, inp.l_max, inp.y_idx, inp.xz_end)


def encode_oracle_map(src: np.ndarray, idx: np.ndarray) -> np.ndarray:
    """Oracle (source, index) pairs in the library's neighbour-map code."""
    out = np.where(src == 0, -1, (src.astype(np.int64) << 40) | idx.astype(np.int64))
    return out


def assert_close_scaled(got: np.ndarray, ref: np.ndarray, scale: np.ndarray, tol: float, what: str):
    """|got - ref| <= tol * scale elementwise, scale = sum |w||V| per output."""
    got = np.asarray(got, np.float64)
    err = np.abs(got - ref)
    bound = tol * np.maximum(scale, np.finfo(np.float64).tiny)
    bad = err > bound
    if bad.any():
        i = int(np.argmax(err / bound))
        raise AssertionError(f"{what}: {int(bad.sum())} of {got.size} outside {tol} x scale; worst at {i}: "
                             f"got {got.flat[i]!r} ref {ref.flat[i]!r} scale {scale.flat[i]!r}")
    return float((err / np.maximum(scale, 1e-300)).max()) if err.size else 0.0


def corner_block(dims, lmax_img: int, l_first: int, l_last: int, y_idx, xz_end, edge: int):
    """The cells of levels l_first..l_last (image finest level lmax_img) that
    lie in the corner cube [0, edge)^3, encoded as a LinearAccess of that cube
    (its levels shift down by lmax_img - log2(edge)); ``edge`` is a multiple
    of the coarsest cell, so no cell straddles the cube.  Returns
    (y_idx, xz_end, index of each kept element in the input arrays)."""
    y_all = np.asarray(y_idx)
    e_all = np.asarray(xz_end).astype(np.int64)
    ys, cnts, idxs = [], [], []
    row0 = 0
    for l in range(l_first, l_last + 1):
        s = 1 << (lmax_img - l)
        assert edge % s == 0
        dz, dx = -(-dims[0] // s), -(-dims[1] // s)
        lim = edge // s
        zz, xx = np.meshgrid(np.arange(min(lim, dz)), np.arange(min(lim, dx)), indexing="ij")
        rows = row0 + zz.ravel() * dx + xx.ravel()
        e = e_all[rows]
        b = np.where(rows > 0, e_all[np.maximum(rows - 1, 0)], 0)
        n = e - b
        first = np.repeat(b - np.concatenate([[0], np.cumsum(n)[:-1]]), n)
        idx = first + np.arange(int(n.sum()))
        y = y_all[idx]
        keep = y < lim
        rid = np.repeat(np.arange(rows.size), n)
        cnt = np.zeros((lim, lim), np.int64)
        cnt[:zz.shape[0], :zz.shape[1]] = np.bincount(rid[keep], minlength=rows.size).reshape(zz.shape)
        cnts.append(cnt.ravel())
        ys.append(y[keep])
        idxs.append(idx[keep])
        row0 += dz * dx
    return (np.concatenate(ys).astype(np.int64), np.cumsum(np.concatenate(cnts)).astype(np.int64),
            np.concatenate(idxs).astype(np.int64))
