"""LinearAccess and the APR tree structure, written from the definitions.

Test infrastructure only (see the package docstring).
"""
from __future__ import annotations

from typing import Dict, Tuple

import numpy as np


def finest_level(dims) -> int:
    """l_max: the smallest l with 2**l >= the largest image edge (Section 2.1:
    a non-power-of-two domain is extended to the next power of two)."""
    m = int(max(dims))
    l = 0
    while (1 << l) < m:
        l += 1
    return l


def level_dims(dims, l_max: int, l: int) -> Tuple[int, int, int]:
    """Grid size at level l.  The paper leaves it implicit (Section 3.1 names
    per-level dims only); reading: ceil(N / 2**(l_max - l)) per axis, so that a
    boundary cell may be partial."""
    s = 2 ** (l_max - l)
    return tuple(-(-int(n) // s) for n in dims)


class LinearAccess:
    """The sparse access structure of Algorithm 1.

    Particles are ordered l -> z -> x -> y.  ``xz_end[row]`` holds the end
    (exclusive) of the particles of ``row = level_offset[l] + z*x_dim[l] + x``;
    the row begins where the previous row ends, and row 0 begins at 0 (the
    algorithm reads ``xz_end[row-1]`` without defining it for row 0).
    """

    def __init__(self, dims, l_min, l_max, y_idx, xz_end):
        self.dims = tuple(int(d) for d in dims)
        self.l_min = int(l_min)
        self.l_max = int(l_max)
        self.y_idx = np.asarray(y_idx).astype(np.int64)
        self.xz_end = np.asarray(xz_end).astype(np.int64)
        self.z_dim, self.x_dim, self.y_dim, self.level_offset = {}, {}, {}, {}
        off = 0
        for l in range(self.l_min, self.l_max + 1):
            dz, dx, dy = level_dims(self.dims, self.dims_lmax, l)
            self.z_dim[l], self.x_dim[l], self.y_dim[l] = dz, dx, dy
            self.level_offset[l] = off
            off += dz * dx
        self.n_rows = off
        if self.xz_end.shape[0] != off:
            raise ValueError(f"xz_end has {self.xz_end.shape[0]} rows, expected {off}")

    @property
    def dims_lmax(self) -> int:
        # the grid levels are relative to the image's own finest level
        return finest_level(self.dims)

    @property
    def n(self) -> int:
        return int(self.y_idx.shape[0])

    def get_row(self, l, z, x):
        """Algorithm 1, get_row."""
        row = self.level_offset[l] + z * self.x_dim[l] + x
        begin = int(self.xz_end[row - 1]) if row > 0 else 0
        end = int(self.xz_end[row])
        return begin, end

    def iterate(self):
        """Algorithm 2: yields (l, z, x, y, i) in storage order (small inputs)."""
        for l in range(self.l_min, self.l_max + 1):
            for z in range(self.z_dim[l]):
                for x in range(self.x_dim[l]):
                    b, e = self.get_row(l, z, x)
                    for i in range(b, e):
                        yield l, z, x, int(self.y_idx[i]), i

    def level_range(self, l) -> Tuple[int, int]:
        """[first, last) particle index of level l."""
        r0 = self.level_offset[l]
        r1 = r0 + self.z_dim[l] * self.x_dim[l]
        b = int(self.xz_end[r0 - 1]) if r0 > 0 else 0
        e = int(self.xz_end[r1 - 1]) if r1 > 0 else 0
        return b, e

    def cells(self, l) -> np.ndarray:
        """(z, x, y) of the level-l particles in storage order, int64 [n_l, 3]."""
        cache = self.__dict__.setdefault("_cells", {})
        if l not in cache:
            cache[l] = self._decode(l)
        return cache[l]

    def _decode(self, l) -> np.ndarray:
        r0 = self.level_offset[l]
        nrow = self.z_dim[l] * self.x_dim[l]
        ends = self.xz_end[r0:r0 + nrow]
        begins = np.concatenate([[self.xz_end[r0 - 1] if r0 > 0 else 0], ends[:-1]])
        counts = ends - begins
        rows = np.repeat(np.arange(nrow, dtype=np.int64), counts)
        b, e = self.level_range(l)
        z = rows // self.x_dim[l]
        x = rows % self.x_dim[l]
        return np.stack([z, x, self.y_idx[b:e]], axis=1)

    def keys(self, l) -> np.ndarray:
        """Linearised cell index (z*x_dim + x)*y_dim + y of the level-l particles;
        sorted ascending because storage order is lexicographic."""
        cache = self.__dict__.setdefault("_keys", {})
        if l not in cache:
            c = self.cells(l)
            cache[l] = (c[:, 0] * self.x_dim[l] + c[:, 1]) * self.y_dim[l] + c[:, 2]
        return cache[l]

    def lookup(self, l, cells: np.ndarray) -> np.ndarray:
        """Global index of the element at level l and cell (z,x,y), or -1."""
        if l < self.l_min or l > self.l_max or cells.shape[0] == 0:
            return np.full(cells.shape[0], -1, np.int64)
        keys = self.keys(l)
        dz, dx, dy = self.z_dim[l], self.x_dim[l], self.y_dim[l]
        ok = ((cells >= 0).all(axis=1) & (cells[:, 0] < dz) & (cells[:, 1] < dx) & (cells[:, 2] < dy))
        q = (cells[:, 0] * dx + cells[:, 1]) * dy + cells[:, 2]
        pos = np.searchsorted(keys, q)
        hit = ok & (pos < keys.shape[0])
        hit[hit] = keys[pos[hit]] == q[hit]
        b, _ = self.level_range(l)
        return np.where(hit, b + pos, -1)


def from_cells(dims, l_min, l_max, cells: Dict[int, np.ndarray]) -> LinearAccess:
    """Encode per-level cell sets as a LinearAccess (sorting them l->z->x->y)."""
    ys, counts = [], []
    for l in range(l_min, l_max + 1):
        dz, dx, dy = level_dims(dims, finest_level(dims), l)
        c = np.asarray(cells.get(l, np.zeros((0, 3), np.int64)), np.int64).reshape(-1, 3)
        order = np.lexsort((c[:, 2], c[:, 1], c[:, 0]))
        c = c[order]
        rows = c[:, 0] * dx + c[:, 1]
        counts.append(np.bincount(rows, minlength=dz * dx))
        ys.append(c[:, 2])
    y_idx = np.concatenate(ys) if ys else np.zeros(0, np.int64)
    xz_end = np.cumsum(np.concatenate(counts)) if counts else np.zeros(0, np.int64)
    return LinearAccess(dims, l_min, l_max, y_idx, xz_end)


def tree_levels(apr: LinearAccess) -> Tuple[int, int]:
    """Tree level range [max(l_min-1, 0), l_max-1]: every particle has a
    parent node (the footnote to Algorithm 3 assumes the parent exists)."""
    return max(apr.l_min - 1, 0), apr.l_max - 1


def tree_structure(apr: LinearAccess) -> LinearAccess:
    """The APR tree (Section 3.4): all interior nodes, i.e. every ancestor of a
    particle, stored as a second LinearAccess over the tree levels."""
    t_lo, t_hi = tree_levels(apr)
    nodes: Dict[int, np.ndarray] = {}
    for L in range(t_hi, t_lo - 1, -1):
        kids = []
        if apr.l_min <= L + 1 <= apr.l_max:
            kids.append(apr.cells(L + 1))
        if L + 1 <= t_hi:
            kids.append(nodes[L + 1])
        allk = np.concatenate(kids) if kids else np.zeros((0, 3), np.int64)
        par = allk // 2
        # distinct parents, via their linear index at level L
        dz, dx, dy = level_dims(apr.dims, apr.dims_lmax, L)
        key = np.unique((par[:, 0] * dx + par[:, 1]) * dy + par[:, 2])
        nodes[L] = np.stack([key // (dx * dy), (key // dy) % dx, key % dy], axis=1)
    if t_hi < t_lo:
        return from_cells(apr.dims, t_lo, t_lo - 1, {})
    return from_cells(apr.dims, t_lo, t_hi, nodes)


def covered_index(apr: LinearAccess, l: int) -> np.ndarray:
    """Dense grid at level l holding, for every cell, the index of the
    particle at a level <= l whose cell contains it, or -1 (Section 3.5,
    case 1).  Painting; meant for small images."""
    d = level_dims(apr.dims, apr.dims_lmax, l)
    out = np.full(d, -1, np.int64)
    for lq in range(apr.l_min, min(l, apr.l_max) + 1):
        b, e = apr.level_range(lq)
        if b == e:
            continue
        c = apr.cells(lq)
        f = 2 ** (l - lq)
        for a0 in range(f):
            for a1 in range(f):
                for a2 in range(f):
                    z = c[:, 0] * f + a0
                    x = c[:, 1] * f + a1
                    y = c[:, 2] * f + a2
                    ok = (z < d[0]) & (x < d[1]) & (y < d[2])
                    out[z[ok], x[ok], y[ok]] = b + np.nonzero(ok)[0]
    return out


def tree_structure_by_painting(apr: LinearAccess) -> LinearAccess:
    """Second derivation of the tree (Section 3.5, case 2): a level-l grid cell
    is a tree node iff it lies in the image and no particle at a level <= l
    contains it.  Painting; meant for small images."""
    t_lo, t_hi = tree_levels(apr)
    nodes = {}
    for L in range(t_lo, t_hi + 1):
        cov = covered_index(apr, L)
        nodes[L] = np.argwhere(cov < 0)
    if t_hi < t_lo:
        return from_cells(apr.dims, t_lo, t_lo - 1, {})
    return from_cells(apr.dims, t_lo, t_hi, nodes)


def check_parents_by_synchronized_iteration(apr: LinearAccess, tree: LinearAccess) -> bool:
    """Algorithm 3: walk each particle row with a parent pointer into the tree
    row (l-1, z/2, x/2), advancing it while the parent's y is below y/2; the
    node reached must be the parent.  Pure Python; small inputs only."""
    t_lo, _ = tree_levels(apr)
    for l in range(max(apr.l_min, t_lo + 1), apr.l_max + 1):
        for z in range(apr.z_dim[l]):
            for x in range(apr.x_dim[l]):
                rb, re = apr.get_row(l, z, x)
                if rb == re:
                    continue
                pb, pe = tree.get_row(l - 1, z // 2, x // 2)
                j = pb
                for i in range(rb, re):
                    half = int(apr.y_idx[i]) // 2
                    while j < pe and tree.y_idx[j] < half:
                        j += 1
                    if j >= pe or tree.y_idx[j] != half:
                        return False
    return True


def pixel_level_map(apr: LinearAccess) -> Tuple[np.ndarray, np.ndarray]:
    """Paint every pixel with the level and index of the particle covering it;
    returns (level map, cover count).  Small images only."""
    lmax = apr.dims_lmax
    lev = np.full(apr.dims, -1, np.int64)
    idx = np.full(apr.dims, -1, np.int64)
    cnt = np.zeros(apr.dims, np.int64)
    for l in range(apr.l_min, apr.l_max + 1):
        c = apr.cells(l)
        b, _ = apr.level_range(l)
        s = 2 ** (lmax - l)
        for k in range(c.shape[0]):
            z, x, y = c[k]
            sl = (slice(z * s, min((z + 1) * s, apr.dims[0])),
                  slice(x * s, min((x + 1) * s, apr.dims[1])),
                  slice(y * s, min((y + 1) * s, apr.dims[2])))
            lev[sl] = l
            idx[sl] = b + k
            cnt[sl] += 1
    return lev, idx, cnt


def check_partition(apr: LinearAccess) -> bool:
    """The particle cells partition the image (Section 3.1): every pixel is
    covered exactly once."""
    _, _, cnt = pixel_level_map(apr)
    return bool((cnt == 1).all())


def check_balance(apr: LinearAccess) -> bool:
    """Levels of neighbouring particle cells differ by at most one (footnote in
    Section 5.1, the CPU implementation).  Reading: neighbours are cells whose
    closures touch (26-neighbourhood); equivalently, 26-adjacent pixels belong
    to cells whose levels differ by at most one."""
    lev, _, _ = pixel_level_map(apr)
    D = np.asarray(apr.dims)
    for dz in (-1, 0, 1):
        for dx in (-1, 0, 1):
            for dy in (-1, 0, 1):
                if (dz, dx, dy) == (0, 0, 0):
                    continue
                a = [slice(max(0, -d), n - max(0, d)) for d, n in zip((dz, dx, dy), D)]
                b = [slice(max(0, d), n - max(0, -d)) for d, n in zip((dz, dx, dy), D)]
                if np.abs(lev[tuple(a)] - lev[tuple(b)]).max(initial=0) > 1:
                    return False
    return True
