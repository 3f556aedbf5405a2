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
