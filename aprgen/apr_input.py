"""Seeded synthetic APR inputs.

An APR (Section 2.1 of the paper) is a set of particle cells: leaves of a
pruned 2^d-tree over the image, each cell ``(l, z, x, y)`` at level ``l``
covering the pixel block ``[z*s, (z+1)*s) x [x*s, (x+1)*s) x [y*s, (y+1)*s)``
clipped to the image, with ``s = 2**(l_max - l)``.  The cells partition the
image.  Particle values are cell means of the pixel image (Section 2.3).

Two sources of inputs live here:

* ``sphere_apr`` -- the sphere-field workload: seeded spheres, a distance-based
  level request, 26-neighbour 2:1 balance, and Poisson-noisy cell means.
* ``random_apr`` -- tiny random balanced (or deliberately unbalanced) APRs for
  property tests.

``encode_cells`` writes the particle cells in the LinearAccess layout of
Algorithm 1 (y index per particle, inclusive end offset per (l, z, x) row);
that layout is the input format of both the oracle and the HIP library.
"""
from __future__ import annotations

import dataclasses
from dataclasses import dataclass
from typing import Dict, Optional, Sequence, Tuple

import numpy as np


def lmax_for(dims: Sequence[int]) -> int:
    """Finest level: the image edge extended to a power of two is 2**l_max."""
    m = int(max(dims))
    return max(0, (m - 1).bit_length())


def level_dims(dims: Sequence[int], l_max: int, l: int) -> Tuple[int, int, int]:
    """Grid size at level ``l``: ceil(N / 2**(l_max - l)) per axis."""
    s = 1 << (l_max - l)
    return tuple((int(n) + s - 1) // s for n in dims)


@dataclass
class AprInput:
    dims: Tuple[int, int, int]          # (N_z, N_x, N_y) pixels
    l_min: int
    l_max: int
    cells: Dict[int, np.ndarray]        # level -> int32 [n_l, 3] (z, x, y), sorted
    values: np.ndarray                  # float32 [N_p], particle order l->z->x->y
    y_idx: np.ndarray                   # uint16 [N_p]
    xz_end: np.ndarray                  # uint64 [n_rows], inclusive row ends
    meta: dict = dataclasses.field(default_factory=dict)

    @property
    def n_particles(self) -> int:
        return int(self.y_idx.shape[0])

    @property
    def n_pixels(self) -> int:
        return int(np.prod(self.dims))

    def level_counts(self) -> Dict[int, int]:
        return {l: int(c.shape[0]) for l, c in self.cells.items()}

    def particle_levels(self) -> np.ndarray:
        return np.concatenate([np.full(self.cells[l].shape[0], l, np.int32)
                               for l in range(self.l_min, self.l_max + 1)])

    def particle_coords(self) -> np.ndarray:
        return np.concatenate([self.cells[l] for l in range(self.l_min, self.l_max + 1)])

    def with_values(self, values: np.ndarray) -> "AprInput":
        return dataclasses.replace(self, values=np.ascontiguousarray(values))


# ----------------------------------------------------------------------------
# LinearAccess encoding of a particle cell set (Algorithm 1 layout)
# ----------------------------------------------------------------------------

def encode_cells(dims, l_min, l_max, cells: Dict[int, np.ndarray]):
    """Return (y_idx uint16, xz_end uint64) for per-level sorted cell lists.

    Rows are enumerated l -> z -> x for l in [l_min, l_max]; ``xz_end[row]``
    is the number of particles in all rows up to and including ``row``.
    """
    ys, counts = [], []
    for l in range(l_min, l_max + 1):
        dz, dx, _ = level_dims(dims, l_max, l)
        c = cells[l]
        rows = c[:, 0].astype(np.int64) * dx + c[:, 1]
        counts.append(np.bincount(rows, minlength=dz * dx).astype(np.uint64))
        ys.append(c[:, 2].astype(np.uint16))
    y_idx = np.concatenate(ys) if ys else np.zeros(0, np.uint16)
    xz_end = np.cumsum(np.concatenate(counts), dtype=np.uint64)
    return y_idx, xz_end


def _sorted_cells(mask: np.ndarray) -> np.ndarray:
    nz = np.nonzero(mask)          # C order == lexicographic (z, x, y)
    return np.stack(nz, axis=1).astype(np.int32) if len(nz[0]) else np.zeros((0, 3), np.int32)


# ----------------------------------------------------------------------------
# Refinement-set helpers (boolean grids per level)
# ----------------------------------------------------------------------------

def _parent_or(mask: np.ndarray) -> np.ndarray:
    """OR over 2x2x2 blocks (a coarse cell is marked if any child is)."""
    pads = [(0, d % 2) for d in mask.shape]
    m = np.pad(mask, pads) if any(p[1] for p in pads) else mask
    a, b, c = (d // 2 for d in m.shape)
    return m.reshape(a, 2, b, 2, c, 2).any(axis=(1, 3, 5))


def _children_of(mask: np.ndarray, child_dims) -> np.ndarray:
    up = mask.repeat(2, 0).repeat(2, 1).repeat(2, 2)
    return up[:child_dims[0], :child_dims[1], :child_dims[2]]


def _dilate26(mask: np.ndarray) -> np.ndarray:
    out = mask.copy()
    # separable 3-wide max along each axis == 26-neighbourhood dilation
    for ax in range(3):
        m = out
        o = m.copy()
        sl_lo = [slice(None)] * 3
        sl_hi = [slice(None)] * 3
        sl_lo[ax] = slice(0, -1)
        sl_hi[ax] = slice(1, None)
        o[tuple(sl_lo)] |= m[tuple(sl_hi)]
        o[tuple(sl_hi)] |= m[tuple(sl_lo)]
        out = o
    return out


def _leaves_from_refined(dims, l_min, l_max, refined: Dict[int, np.ndarray]):
    """Particle cells = cells whose parent is refined (or level l_min) and
    which are not refined themselves."""
    cells = {}
    for l in range(l_min, l_max + 1):
        d = level_dims(dims, l_max, l)
        exists = np.ones(d, bool) if l == l_min else _children_of(refined[l - 1], d)
        ref = refined.get(l)
        leaf = exists if ref is None else (exists & ~ref)
        cells[l] = _sorted_cells(leaf)
    return cells


def balance_refined(dims, l_min, l_max, refined: Dict[int, np.ndarray]) -> Dict[int, np.ndarray]:
    """One fine-to-coarse pass: S_l |= parent(dilate26(S_{l+1})).

    Guarantees that every refined cell's parent is refined and that leaf
    cells whose closures touch differ by at most one level.
    """
    out = dict(refined)
    for l in range(l_max - 2, l_min - 1, -1):
        out[l] = out[l] | _parent_or(_dilate26(out[l + 1]))
    return out


# ----------------------------------------------------------------------------
# Random tiny APRs for property tests
# ----------------------------------------------------------------------------

def random_apr(dims, l_min: int = 0, seed: int = 0, p_refine: float = 0.3,
               balanced: bool = True, value_range=(0.5, 2.0)) -> AprInput:
    dims = tuple(int(d) for d in dims)
    l_max = lmax_for(dims)
    l_min = min(l_min, l_max)
    rng = np.random.Generator(np.random.PCG64(seed))
    refined: Dict[int, np.ndarray] = {}
    for l in range(l_max - 1, l_min - 1, -1):
        d = level_dims(dims, l_max, l)
        r = rng.random(d) < p_refine
        if l + 1 <= l_max - 1:
            up = refined[l + 1]
            r |= _parent_or(_dilate26(up) if balanced else up)
        refined[l] = r
    cells = _leaves_from_refined(dims, l_min, l_max, refined)
    y_idx, xz_end = encode_cells(dims, l_min, l_max, cells)
    n = y_idx.shape[0]
    vals = rng.uniform(value_range[0], value_range[1], size=n).astype(np.float32)
    return AprInput(dims, l_min, l_max, cells, vals, y_idx, xz_end,
                    meta={"kind": "random", "seed": seed, "balanced": balanced})


def dense_apr(dims, l_min: int = 0, values: Optional[np.ndarray] = None, seed: int = 0) -> AprInput:
    """Every particle at the finest level (the APR of a pixel image at CR 1)."""
    dims = tuple(int(d) for d in dims)
    l_max = lmax_for(dims)
    refined = {l: np.ones(level_dims(dims, l_max, l), bool) for l in range(l_min, l_max)}
    cells = _leaves_from_refined(dims, l_min, l_max, refined)
    y_idx, xz_end = encode_cells(dims, l_min, l_max, cells)
    if values is None:
        rng = np.random.Generator(np.random.PCG64(seed))
        values = rng.uniform(0.5, 2.0, size=y_idx.shape[0]).astype(np.float32)
    else:
        values = np.ascontiguousarray(values, dtype=np.float32).reshape(-1)
    return AprInput(dims, l_min, l_max, cells, values, y_idx, xz_end,
                    meta={"kind": "dense"})


# ----------------------------------------------------------------------------
# Sphere-field workload
# ----------------------------------------------------------------------------

@dataclass(frozen=True)
class SphereConfig:
    dims: Tuple[int, int, int]
    n_spheres: int
    r_min: float
    r_max: float
    l_min: int = 2
    seed: int = 1000
    background: float = 100.0
    foreground: float = 1000.0
    edge_sigma: float = 1.0          # Gaussian blur of the sphere indicator
    psf_sigma: float = 0.0           # optional extra 5^3 Gaussian PSF blur
    psf_size: int = 5
    noise: bool = True               # Poisson noise on pixel intensities
    dense: bool = False              # every particle at the finest level


CONFIGS = {
    # 64^3, 8 spheres r in [4, 10], levels 2..6: small parity case.
    "sphere64": SphereConfig((64, 64, 64), 8, 4.0, 10.0, 2, 1000),
    # 512^3, r in [4, 24], levels 2..9; sphere count set so that the
    # pixels/particles ratio is ~20 (6.6M particles).
    "sphere512": SphereConfig((512, 512, 512), 320, 4.0, 24.0, 2, 2000),
    # the literal 200-sphere variant of the 512^3 field (ratio ~32)
    "sphere512_200": SphereConfig((512, 512, 512), 200, 4.0, 24.0, 2, 2000),
    # 256^3 with every particle at level 8 (dense-equivalence case)
    "dense256": SphereConfig((256, 256, 256), 40, 4.0, 24.0, 2, 2001, dense=True),
    # 32^3 sphere field (gradient checks)
    "sphere32": SphereConfig((32, 32, 32), 3, 3.0, 6.0, 1, 4000),
    # (N_z, N_x, N_y) = 1024 x 2048 x 2048, r in [4, 24], levels 2..11; sphere
    # counts set for pixels/particles ratios of ~50, ~100 and ~200 (86.6M,
    # 43.1M and 21.5M particles).  Generated slab by slab, never cached.
    "field2k_cr50": SphereConfig((1024, 2048, 2048), 3900, 4.0, 24.0, 2, 3000),
    "field2k_cr100": SphereConfig((1024, 2048, 2048), 1870, 4.0, 24.0, 2, 3000),
    "field2k_cr200": SphereConfig((1024, 2048, 2048), 890, 4.0, 24.0, 2, 3000),
    # 1024^3, r in [4, 24], levels 2..10, pixels/particles ~30 (35.8M
    # particles): the 16-channel layer field.
    "field1k_layer": SphereConfig((1024, 1024, 1024), 1660, 4.0, 24.0, 2, 4100),
}

# configurations generated slab by slab (too large to hold their pixel image)
SLAB_CONFIGS = {"field2k_cr50", "field2k_cr100", "field2k_cr200", "field1k_layer"}


def _sphere_params(cfg: SphereConfig):
    rng = np.random.Generator(np.random.PCG64(cfg.seed))
    centres = rng.uniform(0.0, 1.0, size=(cfg.n_spheres, 3)) * np.asarray(cfg.dims, np.float64)
    radii = rng.uniform(cfg.r_min, cfg.r_max, size=cfg.n_spheres)
    return centres, radii


def _axis_box(idx: np.ndarray, s: int, n: int):
    """Pixel-centre extent [lo, hi] of cells ``idx`` (cell side ``s``) along one axis."""
    lo = idx * s + 0.5
    hi = np.minimum((idx + 1) * s, n) - 0.5
    return lo, hi


def _rule_refined(cfg: SphereConfig, l_max: int, centres, radii) -> Dict[int, np.ndarray]:
    """Cells refined by the distance rule.

    A pixel at distance d from the nearest sphere surface requests level
    ``l_max - floor(log2(1 + d/2))``; a level-l cell is refined when a pixel
    inside it requests a finer level, i.e. when d < 2*(2**(l_max-l) - 1)
    somewhere in it.  "Somewhere" is evaluated on the continuous box spanned
    by the cell's pixel centres.
    """
    refined = {}
    for l in range(cfg.l_min, l_max):
        s = 1 << (l_max - l)
        thr = 2.0 * (s - 1)
        d = level_dims(cfg.dims, l_max, l)
        grid = np.zeros(d, bool)
        for c, r in zip(centres, radii):
            reach = r + thr
            sub = []
            near2 = []
            far2 = []
            for a in range(3):
                i0 = max(0, int(np.floor((c[a] - reach) / s)) - 1)
                i1 = min(d[a] - 1, int(np.floor((c[a] + reach) / s)) + 1)
                if i1 < i0:
                    sub = None
                    break
                idx = np.arange(i0, i1 + 1)
                lo, hi = _axis_box(idx, s, cfg.dims[a])
                near = np.maximum(np.maximum(lo - c[a], c[a] - hi), 0.0)
                far = np.maximum(np.abs(c[a] - lo), np.abs(c[a] - hi))
                sh = [1, 1, 1]
                sh[a] = idx.size
                near2.append((near ** 2).reshape(sh))
                far2.append((far ** 2).reshape(sh))
                sub.append(slice(i0, i1 + 1))
            if sub is None:
                continue
            dmin = np.sqrt(near2[0] + near2[1] + near2[2])
            dmax = np.sqrt(far2[0] + far2[1] + far2[2])
            dist = np.where(r < dmin, dmin - r, np.where(r > dmax, r - dmax, 0.0))
            grid[tuple(sub)] |= dist < thr
        refined[l] = grid
    return refined


def _blur_radius(cfg: SphereConfig) -> int:
    """Rows of context a clean-image row depends on along each axis: the edge
    blur's support (scipy's radius for truncate=4) plus the PSF's half size."""
    h = int(4.0 * cfg.edge_sigma + 0.5) if cfg.edge_sigma > 0 else 0
    if cfg.psf_sigma > 0:
        h += cfg.psf_size // 2
    return h


def _clean_rows(cfg: SphereConfig, centres, radii, z0: int, z1: int) -> np.ndarray:
    """Rows ``z0 <= z < z1`` (all x, y) of the clean image.

    The rows are computed on a block widened by the blur radius on both sides
    (clipped to the image), so each returned row equals the same row of the
    whole-image computation: zero padding acts only at the image border.
    """
    from scipy import ndimage
    nz, nx, ny = cfg.dims
    h = _blur_radius(cfg)
    a0, a1 = max(0, z0 - h), min(nz, z1 + h)
    union = np.zeros((a1 - a0, nx, ny), np.float32)
    for c, r in zip(centres, radii):
        lo = [max(0, int(np.floor(c[a] - r - 1))) for a in range(3)]
        hi = [min(cfg.dims[a], int(np.ceil(c[a] + r + 1))) for a in range(3)]
        lo[0], hi[0] = max(lo[0], a0), min(hi[0], a1)
        if any(h_ <= l_ for l_, h_ in zip(lo, hi)):
            continue
        zz = (np.arange(lo[0], hi[0]) + 0.5 - c[0]) ** 2
        xx = (np.arange(lo[1], hi[1]) + 0.5 - c[1]) ** 2
        yy = (np.arange(lo[2], hi[2]) + 0.5 - c[2]) ** 2
        inside = (zz[:, None, None] + xx[None, :, None] + yy[None, None, :]) <= r * r
        view = union[lo[0] - a0:hi[0] - a0, lo[1]:hi[1], lo[2]:hi[2]]
        view[inside] = 1.0
    if cfg.edge_sigma > 0:
        union = ndimage.gaussian_filter(union, cfg.edge_sigma, mode="constant", truncate=4.0)
    img = (cfg.background + (cfg.foreground - cfg.background) * union).astype(np.float32)
    del union
    if cfg.psf_sigma > 0:
        k = cfg.psf_size
        t = np.arange(k) - (k - 1) / 2.0
        g = np.exp(-0.5 * (t / cfg.psf_sigma) ** 2)
        g /= g.sum()
        for a in range(3):
            img = ndimage.correlate1d(img, g.astype(np.float32), axis=a, mode="constant")
    if a0 == z0 and a1 == z1:
        return img
    return np.ascontiguousarray(img[z0 - a0:z1 - a0])


def _clean_image(cfg: SphereConfig, centres, radii) -> np.ndarray:
    return _clean_rows(cfg, centres, radii, 0, cfg.dims[0])


def _block_sums(img: np.ndarray, l_max: int, l_min: int):
    """Pixel sums and pixel counts of every cell at every level l_min..l_max."""
    sums = {l_max: img}
    cur = img.astype(np.float64) if img.dtype != np.float64 else img
    for l in range(l_max - 1, l_min - 1, -1):
        pads = [(0, d % 2) for d in cur.shape]
        if any(p[1] for p in pads):
            cur = np.pad(cur, pads)
        a, b, c = (d // 2 for d in cur.shape)
        cur = cur.reshape(a, 2, b, 2, c, 2).sum(axis=(1, 3, 5))
        sums[l] = cur
    return sums


def _cell_counts(dims, l_max, l, cells: np.ndarray) -> np.ndarray:
    s = 1 << (l_max - l)
    cnt = np.ones(cells.shape[0], np.float64)
    for a in range(3):
        i = cells[:, a].astype(np.int64)
        cnt *= np.minimum((i + 1) * s, dims[a]) - i * s
    return cnt


def sphere_apr(cfg: SphereConfig, return_image: bool = False):
    """Generate the APR of a seeded sphere-field image (see module doc)."""
    dims = tuple(int(d) for d in cfg.dims)
    l_max = lmax_for(dims)
    centres, radii = _sphere_params(cfg)
    if cfg.dense:
        refined = {l: np.ones(level_dims(dims, l_max, l), bool) for l in range(cfg.l_min, l_max)}
    else:
        refined = balance_refined(dims, cfg.l_min, l_max, _rule_refined(cfg, l_max, centres, radii))
    cells = _leaves_from_refined(dims, cfg.l_min, l_max, refined)
    del refined
    y_idx, xz_end = encode_cells(dims, cfg.l_min, l_max, cells)
    img = _clean_image(cfg, centres, radii)
    sums = _block_sums(img, l_max, cfg.l_min)
    noise_rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([cfg.seed, 1])))
    vals = []
    for l in range(cfg.l_min, l_max + 1):
        c = cells[l]
        if c.shape[0] == 0:
            continue
        lam = sums[l][c[:, 0], c[:, 1], c[:, 2]].astype(np.float64)
        cnt = _cell_counts(dims, l_max, l, c)
        if cfg.noise:
            v = noise_rng.poisson(lam) / cnt
        else:
            v = lam / cnt
        vals.append(v.astype(np.float32))
    values = np.concatenate(vals) if vals else np.zeros(0, np.float32)
    meta = {"kind": "sphere", "config": dataclasses.asdict(cfg), "l_max": l_max,
            "n_particles": int(values.shape[0]),
            "cr": float(np.prod(dims)) / max(1, values.shape[0])}
    out = AprInput(dims, cfg.l_min, l_max, cells, values, y_idx, xz_end, meta)
    if return_image:
        return out, img
    return out


# ----------------------------------------------------------------------------
# Slab-wise generation of large sphere fields
# ----------------------------------------------------------------------------

def _sphere_refined(cfg: SphereConfig, l_max: int, centres, radii) -> Dict[int, np.ndarray]:
    dims = tuple(int(d) for d in cfg.dims)
    if cfg.dense:
        return {l: np.ones(level_dims(dims, l_max, l), bool) for l in range(cfg.l_min, l_max)}
    return balance_refined(dims, cfg.l_min, l_max, _rule_refined(cfg, l_max, centres, radii))


def _leaf_rows(dims, l_min, l_max, l, zl0, zl1, parent, ref):
    """Leaf mask of level-l rows zl0 <= z < zl1.  ``parent`` holds the
    level-(l-1) refinement rows zl0//2 .. (zl1+1)//2 (None at l_min), ``ref``
    the level-l refinement rows zl0..zl1 (None at l_max)."""
    d = level_dims(dims, l_max, l)
    if parent is None:
        exists = np.ones((zl1 - zl0, d[1], d[2]), bool)
    else:
        up = parent.repeat(2, 0).repeat(2, 1).repeat(2, 2)
        off = zl0 - 2 * (zl0 // 2)
        exists = up[off:off + (zl1 - zl0), :d[1], :d[2]]
    return exists if ref is None else (exists & ~ref)


def _slab_job(args):
    """One z-slab: clean rows, block sums for the levels whose cells fit in
    the slab, leaves, Poisson-noisy means.  Returns, per level, the leaves'
    y (uint16), the per-row counts of the slab's rows (uint64) and the values
    (float32), plus the block sums of the slab-sized cells."""
    cfg, l_max, centres, radii, j, slab, l_c, slices = args
    dims = tuple(int(d) for d in cfg.dims)
    z0, z1 = j * slab, min(dims[0], (j + 1) * slab)
    img = _clean_rows(cfg, centres, radii, z0, z1)
    sums = _block_sums(img, l_max, l_c)
    del img
    rng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([cfg.seed, 1, j])))
    out = {}
    for l in range(max(l_c, cfg.l_min), l_max + 1):
        s = 1 << (l_max - l)
        zl0, zl1 = z0 // s, (z1 + s - 1) // s
        leaf = _leaf_rows(dims, cfg.l_min, l_max, l, zl0, zl1, *slices[l])
        dz, dx, dy = leaf.shape
        c = _sorted_cells(leaf)
        del leaf
        lam = sums[l][c[:, 0], c[:, 1], c[:, 2]].astype(np.float64)
        c[:, 0] += zl0
        cnt = _cell_counts(dims, l_max, l, c)
        v = rng.poisson(lam) / cnt if cfg.noise else lam / cnt
        counts = np.bincount((c[:, 0] - zl0).astype(np.int64) * dx + c[:, 1], minlength=dz * dx)
        out[l] = (c[:, 2].astype(np.uint16), counts.astype(np.uint64), v.astype(np.float32))
    return j, out, np.asarray(sums[l_c], np.float64)


class _AccessCells(dict):
    """Per-level (z, x, y) cell lists of a LinearAccess, decoded on first use."""

    def __init__(self, dims, l_min, l_max, y_idx, xz_end):
        super().__init__()
        self._a = (dims, l_min, l_max, y_idx, xz_end)

    def __missing__(self, l):
        dims, l_min, l_max, y_idx, xz_end = self._a
        if not l_min <= l <= l_max:
            raise KeyError(l)
        c = _level_cells(dims, l_min, l_max, y_idx, xz_end, l)
        self[l] = c
        return c

    def items(self):
        return [(l, self[l]) for l in range(self._a[1], self._a[2] + 1)]

    def keys(self):
        return list(range(self._a[1], self._a[2] + 1))

    def __iter__(self):
        return iter(self.keys())

    def __len__(self):
        return self._a[2] - self._a[1] + 1


def sphere_apr_slabs(cfg: SphereConfig, slab: int = 32, workers: int = 1, progress=None) -> AprInput:
    """The sphere-field APR generated one z-slab at a time.

    The cell structure is that of ``sphere_apr`` (same rule, same balance).
    The clean image is only ever held ``slab`` (+ blur radius) rows at a time;
    each slab's rows equal the whole-image computation, so without noise the
    values equal ``sphere_apr``'s.  Noise is drawn from one seeded stream per
    slab (and one for the cells larger than a slab): the same distribution as
    ``sphere_apr`` (a Poisson draw of each cell's intensity sum), a different
    realisation.  ``slab`` is a power of two; ``progress(done, total)`` is
    called as slabs finish.  ``cells`` of the result are decoded lazily.
    """
    dims = tuple(int(d) for d in cfg.dims)
    l_max = lmax_for(dims)
    if slab & (slab - 1) or slab < 1:
        raise ValueError("slab must be a power of two")
    centres, radii = _sphere_params(cfg)
    refined = _sphere_refined(cfg, l_max, centres, radii)
    l_c = max(cfg.l_min, l_max - (slab.bit_length() - 1))   # coarsest level done per slab
    n_slab = (dims[0] + slab - 1) // slab
    jobs = []
    for j in range(n_slab):
        z0, z1 = j * slab, min(dims[0], (j + 1) * slab)
        sl = {}
        for l in range(max(l_c, cfg.l_min), l_max + 1):
            s = 1 << (l_max - l)
            zl0, zl1 = z0 // s, (z1 + s - 1) // s
            par = None if l == cfg.l_min else refined[l - 1][zl0 // 2:(zl1 + 1) // 2]
            ref = refined[l][zl0:zl1] if l < l_max else None
            sl[l] = (par, ref)
        jobs.append((cfg, l_max, centres, radii, j, slab, l_c, sl))
    res = [None] * n_slab
    if workers <= 1 or n_slab <= 1:
        for k, jb in enumerate(jobs):
            j, o, cs = _slab_job(jb)
            res[j] = (o, cs)
            if progress:
                progress(k + 1, n_slab)
    else:
        import concurrent.futures as cf
        import multiprocessing as mp
        with cf.ProcessPoolExecutor(max_workers=min(workers, n_slab), mp_context=mp.get_context("spawn")) as ex:
            futs = [ex.submit(_slab_job, jb) for jb in jobs]
            del jobs
            for k, f in enumerate(cf.as_completed(futs)):
                j, o, cs = f.result()
                res[j] = (o, cs)
                if progress:
                    progress(k + 1, n_slab)
    # cells larger than a slab: sums of the slab-sized cells, reduced further
    coarse = {}
    if l_c > cfg.l_min:
        cur = np.concatenate([r[1] for r in res], axis=0)
        crng = np.random.Generator(np.random.PCG64(np.random.SeedSequence([cfg.seed, 2])))
        csum = {l_c: cur}
        for l in range(l_c - 1, cfg.l_min - 1, -1):
            pads = [(0, d % 2) for d in cur.shape]
            if any(p[1] for p in pads):
                cur = np.pad(cur, pads)
            a, b, c = (d // 2 for d in cur.shape)
            cur = cur.reshape(a, 2, b, 2, c, 2).sum(axis=(1, 3, 5))
            csum[l] = cur
        for l in range(cfg.l_min, l_c):
            d = level_dims(dims, l_max, l)
            par = None if l == cfg.l_min else refined[l - 1]
            leaf = _leaf_rows(dims, cfg.l_min, l_max, l, 0, d[0], par, refined[l])
            c = _sorted_cells(leaf)
            lam = csum[l][c[:, 0], c[:, 1], c[:, 2]].astype(np.float64)
            cnt = _cell_counts(dims, l_max, l, c)
            v = crng.poisson(lam) / cnt if cfg.noise else lam / cnt
            counts = np.bincount(c[:, 0].astype(np.int64) * d[1] + c[:, 1], minlength=d[0] * d[1])
            coarse[l] = (c[:, 2].astype(np.uint16), counts.astype(np.uint64), v.astype(np.float32))
    del refined
    ys, cnts, vals = [], [], []
    for l in range(cfg.l_min, l_max + 1):
        parts = [coarse[l]] if l in coarse else [r[0][l] for r in res]
        for y, cn, v in parts:
            ys.append(y)
            cnts.append(cn)
            vals.append(v)
    del res
    y_idx = np.concatenate(ys)
    xz_end = np.cumsum(np.concatenate(cnts), dtype=np.uint64)
    values = np.concatenate(vals)
    meta = {"kind": "sphere", "config": dataclasses.asdict(cfg), "l_max": l_max, "slab": slab,
            "n_particles": int(values.shape[0]), "cr": float(np.prod(dims)) / max(1, values.shape[0])}
    cells = _AccessCells(dims, cfg.l_min, l_max, y_idx, xz_end)
    return AprInput(dims, cfg.l_min, l_max, cells, values, y_idx, xz_end, meta)


def sphere_level_counts(cfg: SphereConfig) -> Dict[int, int]:
    """Particles per level of the sphere-field APR (structure only, no image)."""
    dims = tuple(int(d) for d in cfg.dims)
    l_max = lmax_for(dims)
    centres, radii = _sphere_params(cfg)
    refined = _sphere_refined(cfg, l_max, centres, radii)
    out = {}
    for l in range(cfg.l_min, l_max + 1):
        d = level_dims(dims, l_max, l)
        n = 0
        step = max(1, (1 << 26) // max(1, d[1] * d[2]))
        for z0 in range(0, d[0], step):
            z1 = min(d[0], z0 + step)
            par = None if l == cfg.l_min else refined[l - 1][z0 // 2:(z1 + 1) // 2]
            ref = refined[l][z0:z1] if l < l_max else None
            n += int(_leaf_rows(dims, cfg.l_min, l_max, l, z0, z1, par, ref).sum())
        out[l] = n
    return out


def _level_cells(dims, l_min, l_max, y_idx, xz_end, l) -> np.ndarray:
    ends = np.asarray(xz_end, np.int64)
    row0 = 0
    for m in range(l_min, l):
        dz, dx, _ = level_dims(dims, l_max, m)
        row0 += dz * dx
    dz, dx, _ = level_dims(dims, l_max, l)
    nrow = dz * dx
    e = ends[row0:row0 + nrow]
    b = np.concatenate([[ends[row0 - 1] if row0 > 0 else 0], e[:-1]])
    rows = np.repeat(np.arange(nrow, dtype=np.int64), e - b)
    p0 = int(ends[row0 - 1]) if row0 > 0 else 0
    ys = np.asarray(y_idx[p0:p0 + rows.size], np.int32)
    return np.stack([(rows // dx).astype(np.int32), (rows % dx).astype(np.int32), ys], axis=1)


def cells_from_access(dims, l_min, l_max, y_idx, xz_end) -> Dict[int, np.ndarray]:
    """Per-level (z, x, y) cell lists of a LinearAccess (inverse of encode_cells)."""
    cells = {}
    row0 = 0
    ends = np.asarray(xz_end, np.int64)
    for l in range(l_min, l_max + 1):
        dz, dx, _ = level_dims(dims, l_max, l)
        nrow = dz * dx
        e = ends[row0:row0 + nrow]
        b = np.concatenate([[ends[row0 - 1] if row0 > 0 else 0], e[:-1]])
        rows = np.repeat(np.arange(nrow, dtype=np.int64), e - b)
        p0 = int(ends[row0 - 1]) if row0 > 0 else 0
        ys = np.asarray(y_idx[p0:p0 + rows.size], np.int32)
        cells[l] = np.stack([(rows // dx).astype(np.int32), (rows % dx).astype(np.int32), ys], axis=1)
        row0 += nrow
    return cells


def cached_sphere_apr(name: str, cache_dir: Optional[str] = None) -> AprInput:
    """``sphere_apr(CONFIGS[name])`` memoised as an .npz file (y_idx, xz_end,
    values; the cell lists are rebuilt from them)."""
    import hashlib
    import os
    cfg = CONFIGS[name]
    if cache_dir is None:
        cache_dir = os.environ.get("APRGEN_CACHE",
                                   os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "_cache"))
    os.makedirs(cache_dir, exist_ok=True)
    key = hashlib.sha1(repr(dataclasses.astuple(cfg)).encode()).hexdigest()[:10]
    path = os.path.join(cache_dir, f"{name}_{key}.npz")
    l_max = lmax_for(cfg.dims)
    if os.path.exists(path):
        z = np.load(path, allow_pickle=False)
        y_idx, xz_end, values = z["y_idx"], z["xz_end"], z["values"]
        cells = cells_from_access(cfg.dims, cfg.l_min, l_max, y_idx, xz_end)
        return AprInput(tuple(cfg.dims), cfg.l_min, l_max, cells, values, y_idx, xz_end,
                        meta={"kind": "sphere", "name": name, "n_particles": int(values.shape[0]),
                              "cr": float(np.prod(cfg.dims)) / max(1, values.shape[0])})
    a = sphere_apr(cfg)
    tmp = path + f".{os.getpid()}.tmp.npz"
    np.savez(tmp, values=a.values, y_idx=a.y_idx, xz_end=a.xz_end)
    os.replace(tmp, path)
    a.meta["name"] = name
    return a


def load_sphere_apr(name: str, workers: Optional[int] = None, progress=None,
                    cache_dir: Optional[str] = None) -> AprInput:
    """The named configuration: slab-wise generation (``workers`` processes,
    default the CPUs available up to 16) for the large fields,
    ``cached_sphere_apr`` for the rest.  A large field is cached only when a
    cache directory is given (``cache_dir`` or the ``APRGEN_LARGE_CACHE``
    environment variable): an uncompressed .npz of y_idx, xz_end, values."""
    if name not in SLAB_CONFIGS:
        return cached_sphere_apr(name)
    import hashlib
    import os
    cfg = CONFIGS[name]
    cache_dir = cache_dir or os.environ.get("APRGEN_LARGE_CACHE")
    path = None
    if cache_dir:
        key = hashlib.sha1(repr(dataclasses.astuple(cfg)).encode()).hexdigest()[:10]
        path = os.path.join(cache_dir, f"{name}_{key}.npz")
        if os.path.exists(path):
            z = np.load(path, allow_pickle=False)
            y_idx, xz_end, values = z["y_idx"], z["xz_end"], z["values"]
            l_max = lmax_for(cfg.dims)
            return AprInput(tuple(cfg.dims), cfg.l_min, l_max,
                            _AccessCells(tuple(cfg.dims), cfg.l_min, l_max, y_idx, xz_end), values, y_idx, xz_end,
                            meta={"kind": "sphere", "name": name, "n_particles": int(values.shape[0]),
                                  "cr": float(np.prod(cfg.dims)) / max(1, values.shape[0])})
    if workers is None:
        workers = min(16, len(os.sched_getaffinity(0)))
    a = sphere_apr_slabs(cfg, slab=32, workers=workers, progress=progress)
    a.meta["name"] = name
    if path:
        os.makedirs(cache_dir, exist_ok=True)
        tmp = path + f".{os.getpid()}.tmp.npz"
        np.savez(tmp, values=a.values, y_idx=a.y_idx, xz_end=a.xz_end)
        os.replace(tmp, path)
    return a


def gaussian_stencil(k: int, sigma: float) -> np.ndarray:
    """Normalised separable Gaussian filter [k, k, k] (FP64), a filter input."""
    t = np.arange(k) - (k - 1) / 2.0
    g = np.exp(-0.5 * (t / sigma) ** 2)
    g = g / g.sum()
    return np.einsum("i,j,k->ijk", g, g, g)


def sobel_stencils() -> np.ndarray:
    """The three 3^3 Sobel filters [3, 3, 3, 3] (d/dz, d/dx, d/dy), a filter
    input: a central difference along one axis times [1, 2, 1] smoothing along
    the other two, scaled by 1/32 so that a unit-slope ramp on pixels gives 1."""
    d = np.array([-1.0, 0.0, 1.0])
    sm = np.array([1.0, 2.0, 1.0])
    out = np.stack([np.einsum("i,j,k->ijk", d, sm, sm), np.einsum("i,j,k->ijk", sm, d, sm),
                    np.einsum("i,j,k->ijk", sm, sm, d)])
    return out / 32.0


# ----------------------------------------------------------------------------
# Deconvolution workload: sphere fields blurred by a 5^3 Gaussian PSF
# (sigma 1.5) and corrupted by Poisson noise.  Sphere count scales with the
# volume (320 spheres per 512^3, radii 4-16 px).
# ----------------------------------------------------------------------------

DECONV_PSF_SIGMA = 1.5
DECONV_PSF_SIZE = 5


def deconv_config(edge: int, seed: int, r_max: float = 16.0) -> SphereConfig:
    n_spheres = max(2, int(round(320 * (edge / 512.0) ** 3)))
    return SphereConfig((edge, edge, edge), n_spheres, 4.0, r_max, 2, seed, psf_sigma=DECONV_PSF_SIGMA,
                        psf_size=DECONV_PSF_SIZE)


def deconv_psf() -> np.ndarray:
    return gaussian_stencil(DECONV_PSF_SIZE, DECONV_PSF_SIGMA)


def _deconv_job(args):
    edge, seed = args
    a = sphere_apr(deconv_config(edge, seed))
    return a


def input_digest(inp) -> str:
    """SHA-256 of an APR input's LinearAccess and values (pairs stored results
    with the input they were computed from)."""
    import hashlib
    h = hashlib.sha256()
    for a in (np.asarray(inp.y_idx, np.uint16), np.asarray(inp.xz_end, np.uint64),
              np.asarray(inp.values, np.float32)):
        h.update(np.ascontiguousarray(a).tobytes())
    return h.hexdigest()


def deconv_set(edges: Sequence[int], seed0: int, workers: int = 1, progress=None):
    """APRs of the deconvolution workload with seeds seed0, seed0 + 1, ...;
    generated in ``workers`` processes; ``progress(edge, n_particles)`` is
    called as each one is done."""
    jobs = [(int(e), seed0 + i) for i, e in enumerate(edges)]
    if workers <= 1 or len(jobs) <= 1:
        out = []
        for j in jobs:
            out.append(_deconv_job(j))
            if progress:
                progress(j[0], out[-1].n_particles)
        return out
    import concurrent.futures as cf
    import multiprocessing as mp
    with cf.ProcessPoolExecutor(max_workers=min(workers, len(jobs)), mp_context=mp.get_context("spawn")) as ex:
        futs = [ex.submit(_deconv_job, j) for j in jobs]
        for f, j in zip(cf.as_completed(futs), jobs):
            if progress:
                a = f.result()
                progress(a.dims[0], a.n_particles)
        return [f.result() for f in futs]
