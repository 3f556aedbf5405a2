"""APR construction of a synthetic sphere-field image (Section 2.3), in FP64.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Section 2.3 builds an APR from a pixel image in three steps: a level function
says how fine the sampling must be at every location; the Pulling Scheme turns
it into the coarsest partition of the image into cells of the image pyramid
that honours it; the particle values are the means of the pixels each cell
covers (average downsampling).  This module states those steps for the
synthetic sphere fields used as inputs, where the level function is a rule on
the distance to the nearest sphere surface.  Readings, where the paper leaves
the details to its reference or is silent:

* Level rule.  A location at distance d from the nearest sphere surface asks
  for level ``l_max - floor(log2(1 + d/2))``; a cell of level l (side
  s = 2^(l_max - l) pixels) is therefore split when some point of the box
  spanned by its pixel centres lies at d < 2 (s - 1).  The distance from a box
  to a sphere surface is 0 when the box reaches both inside and outside the
  sphere, else the gap between the box's nearest (outside) or farthest
  (inside) point and the radius.
* Pulling Scheme output.  Split every cell the rule asks for; then, from fine
  to coarse, split the parent of every cell that touches (faces, edges or
  corners: 26-neighbourhood) a split cell of the same level, so that
  neighbouring particle cells differ by at most one level (Section 5.1).  The
  particles are the cells that are not split and whose parent is split (every
  cell of level l_min has a "split" parent).
* Image.  Background b, spheres of intensity f, the sphere indicator blurred
  by a normalised Gaussian (sigma pixels, truncated at 4 sigma, zero outside
  the image): clean = b + (f - b) * (G * 1_union).
* Noise.  The noisy sum over a cell of n pixels with clean sum S is taken as
  S + sqrt(S) Z, Z a standard-normal variate: the Gaussian limit of the
  Poisson law of the sum (S >= 100 n here).  Z is the sum of twelve uniforms
  minus six (Irwin-Hall), the uniforms drawn from Philox4x64-10 (Salmon et
  al., SC'11) keyed by the cell, so that any implementation reproduces it.
  The particle value is the noisy sum divided by n.

Every function works on small images: brute force over cells and spheres.
"""
from __future__ import annotations

from typing import Dict

import numpy as np

from .access import LinearAccess, finest_level, from_cells, level_dims

# ---------------------------------------------------------------------------
# Level rule and the Pulling Scheme's partition
# ---------------------------------------------------------------------------


def box_surface_distance(lo, hi, c, r):
    """Distance from the boxes [lo, hi] (arrays [..., 3]) to the surface of
    the sphere (centre c, radius r): 0 if the box holds points inside and
    outside the sphere."""
    near = np.maximum(np.maximum(lo - c, c - hi), 0.0)
    far = np.maximum(np.abs(c - lo), np.abs(c - hi))
    dmin = np.sqrt((near[..., 0] * near[..., 0] + near[..., 1] * near[..., 1]) + near[..., 2] * near[..., 2])
    dmax = np.sqrt((far[..., 0] * far[..., 0] + far[..., 1] * far[..., 1]) + far[..., 2] * far[..., 2])
    return np.where(r < dmin, dmin - r, np.where(r > dmax, r - dmax, 0.0))


def cell_boxes(dims, l_max: int, l: int):
    """Pixel-centre box [lo, hi] of every cell of level l, arrays [Dz, Dx, Dy, 3]."""
    s = 2 ** (l_max - l)
    d = level_dims(dims, l_max, l)
    lo = np.zeros(d + (3,))
    hi = np.zeros(d + (3,))
    for a in range(3):
        i = np.arange(d[a], dtype=np.float64)
        sh = [1, 1, 1]
        sh[a] = d[a]
        lo[..., a] = (i * s + 0.5).reshape(sh)
        hi[..., a] = (np.minimum((i + 1) * s, dims[a]) - 0.5).reshape(sh)
    return lo, hi


def split_by_rule(dims, l_min: int, l_max: int, centres, radii) -> Dict[int, np.ndarray]:
    """Cells of levels l_min .. l_max-1 that the distance rule splits."""
    out = {}
    for l in range(l_min, l_max):
        s = 2 ** (l_max - l)
        lo, hi = cell_boxes(dims, l_max, l)
        need = np.zeros(lo.shape[:3], bool)
        for c, r in zip(np.asarray(centres, np.float64), np.asarray(radii, np.float64)):
            need |= box_surface_distance(lo, hi, c, r) < 2.0 * (s - 1)
        out[l] = need
    return out


def _touching(mask: np.ndarray) -> np.ndarray:
    """Cells that touch (26-neighbourhood) or are a marked cell."""
    out = mask.copy()
    d = mask.shape
    for dz in (-1, 0, 1):
        for dx in (-1, 0, 1):
            for dy in (-1, 0, 1):
                src = tuple(slice(max(0, -o), n - max(0, o)) for o, n in zip((dz, dx, dy), d))
                dst = tuple(slice(max(0, o), n - max(0, -o)) for o, n in zip((dz, dx, dy), d))
                out[dst] |= mask[src]
    return out


def _parents(mask: np.ndarray, parent_dims) -> np.ndarray:
    """Parent cells (level l-1) of the marked cells of level l."""
    out = np.zeros(parent_dims, bool)
    z, x, y = np.nonzero(mask)
    out[z // 2, x // 2, y // 2] = True
    return out


def balanced_splits(dims, l_min: int, l_max: int, split: Dict[int, np.ndarray]) -> Dict[int, np.ndarray]:
    """Close the split sets for 2:1 balance, fine to coarse: the parent of
    every cell that touches a split cell is split."""
    out = {l: split[l].copy() for l in split}
    for l in range(l_max - 2, l_min - 1, -1):
        out[l] |= _parents(_touching(out[l + 1]), level_dims(dims, l_max, l))
    return out


def particle_cells(dims, l_min: int, l_max: int, split: Dict[int, np.ndarray]) -> Dict[int, np.ndarray]:
    """Particle cells per level, sorted (z, x, y): not split, parent split."""
    cells = {}
    for l in range(l_min, l_max + 1):
        d = level_dims(dims, l_max, l)
        if l == l_min:
            exists = np.ones(d, bool)
        else:
            z, x, y = np.meshgrid(np.arange(d[0]), np.arange(d[1]), np.arange(d[2]), indexing="ij")
            exists = split[l - 1][z // 2, x // 2, y // 2]
        leaf = exists & ~split[l] if l < l_max else exists
        cells[l] = np.argwhere(leaf).astype(np.int64)   # C order: sorted by (z, x, y)
    return cells


def sphere_partition(dims, l_min: int, centres, radii):
    """(LinearAccess, particle cells) of the sphere field's APR."""
    l_max = finest_level(dims)
    split = balanced_splits(dims, l_min, l_max, split_by_rule(dims, l_min, l_max, centres, radii))
    cells = particle_cells(dims, l_min, l_max, split)
    return from_cells(dims, l_min, l_max, cells), cells


# ---------------------------------------------------------------------------
# Image and particle values
# ---------------------------------------------------------------------------


def gaussian_taps(sigma: float) -> np.ndarray:
    """Normalised Gaussian of radius round(4 sigma)."""
    r = int(4.0 * sigma + 0.5)
    t = np.arange(-r, r + 1, dtype=np.float64)
    g = np.exp(-0.5 * (t / sigma) ** 2)
    return g / g.sum()


def sphere_image(dims, centres, radii, background: float, foreground: float, sigma: float) -> np.ndarray:
    """Clean image [N_z, N_x, N_y], FP64: a pixel (centre p + 1/2) is inside
    a sphere when |p + 1/2 - c|^2 <= r^2; the indicator is blurred axis by
    axis (z, x, y) with zeros outside the image."""
    nz, nx, ny = dims
    ind = np.zeros(dims)
    zz = np.arange(nz) + 0.5
    xx = np.arange(nx) + 0.5
    yy = np.arange(ny) + 0.5
    for c, r in zip(np.asarray(centres, np.float64), np.asarray(radii, np.float64)):
        d2 = ((zz - c[0]) ** 2)[:, None, None] + ((xx - c[1]) ** 2)[None, :, None]
        d2 = d2 + ((yy - c[2]) ** 2)[None, None, :]
        ind[d2 <= r * r] = 1.0
    if sigma > 0:
        g = gaussian_taps(sigma)
        h = g.shape[0] // 2
        for a in range(3):
            n = ind.shape[a]
            pad = [(0, 0)] * 3
            pad[a] = (h, h)
            p = np.pad(ind, pad)
            acc = np.zeros_like(ind)
            for j, w in enumerate(g):
                sl = [slice(None)] * 3
                sl[a] = slice(j, j + n)
                acc += w * p[tuple(sl)]
            ind = acc
    return background + (foreground - background) * ind


_M0, _M1 = np.uint64(0xD2E7470EE14C6C93), np.uint64(0xCA5A826395121157)
_W0, _W1 = np.uint64(0x9E3779B97F4A7C15), np.uint64(0xBB67AE8584CAA73B)
_LO32 = np.uint64(0xFFFFFFFF)
_S32 = np.uint64(32)


def _mulhilo64(a: np.ndarray, b: np.uint64):
    """(high, low) 64-bit halves of the 128-bit product a * b."""
    a0, a1 = a & _LO32, a >> _S32
    b0, b1 = b & _LO32, b >> _S32
    p00, p01, p10, p11 = a0 * b0, a0 * b1, a1 * b0, a1 * b1
    mid = (p00 >> _S32) + (p01 & _LO32) + (p10 & _LO32)
    hi = p11 + (p01 >> _S32) + (p10 >> _S32) + (mid >> _S32)
    return hi, a * b


def philox4x64(ctr, key):
    """Philox4x64-10 (Salmon et al., SC'11): counter words ctr[0..3] and key
    words key[0..1] (uint64 arrays, broadcast) -> four uint64 arrays."""
    with np.errstate(over="ignore"):
        c = [np.asarray(v, np.uint64) for v in ctr]
        k0, k1 = np.asarray(key[0], np.uint64), np.asarray(key[1], np.uint64)
        for rnd in range(10):
            if rnd:
                k0, k1 = k0 + _W0, k1 + _W1
            hi0, lo0 = _mulhilo64(c[0], _M0)
            hi1, lo1 = _mulhilo64(c[2], _M1)
            c = [hi1 ^ c[1] ^ k0, lo1, hi0 ^ c[3] ^ k1, lo0]
    return c


def cell_key(l, z, x, y) -> np.ndarray:
    """Counter word of a cell: level | z | x | y in 16-bit fields."""
    return ((np.asarray(l, np.uint64) << np.uint64(48)) | (np.asarray(z, np.uint64) << np.uint64(32))
            | (np.asarray(x, np.uint64) << np.uint64(16)) | np.asarray(y, np.uint64))


def cell_normal(keys: np.ndarray, seed: int) -> np.ndarray:
    """Z per cell: twelve uniforms (53-bit) from three Philox blocks
    (counter = key, block, 0, 0; key = seed, 0), summed in order, minus 6."""
    keys = np.asarray(keys, np.uint64)
    z = np.zeros(keys.shape)
    zero = np.zeros_like(keys)
    for b in range(3):
        out = philox4x64([keys, np.full_like(keys, b), zero, zero], [np.uint64(seed), np.uint64(0)])
        for w in out:
            z = z + (w >> np.uint64(11)).astype(np.float64) * 2.0 ** -53
    return z - 6.0


def cell_values(dims, l_min: int, l_max: int, cells: Dict[int, np.ndarray], image: np.ndarray,
                noise: bool, seed: int) -> np.ndarray:
    """Particle values in storage order: (S + sqrt(S) Z) / n, or S / n
    without noise; S the clean sum over the cell's pixels inside the image."""
    vals = []
    for l in range(l_min, l_max + 1):
        s = 2 ** (l_max - l)
        c = cells[l]
        if c.shape[0] == 0:
            continue
        S = np.empty(c.shape[0])
        n = np.empty(c.shape[0])
        for i, (z, x, y) in enumerate(c):
            blk = image[z * s:(z + 1) * s, x * s:(x + 1) * s, y * s:(y + 1) * s]
            S[i] = blk.sum()
            n[i] = blk.size
        if noise:
            Z = cell_normal(cell_key(l, c[:, 0], c[:, 1], c[:, 2]), seed)
            S = S + np.sqrt(S) * Z
        vals.append(S / n)
    return np.concatenate(vals) if vals else np.zeros(0)


def sphere_apr(dims, l_min: int, centres, radii, background=100.0, foreground=1000.0, sigma=1.0,
               noise=True, seed=0):
    """(LinearAccess, particle values) of the synthetic sphere field."""
    la, cells = sphere_partition(dims, l_min, centres, radii)
    img = sphere_image(dims, centres, radii, background, foreground, sigma)
    return la, cell_values(dims, l_min, la.l_max, cells, img, noise, seed)
