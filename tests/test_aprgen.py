"""The input generator (CPU): slab-wise generation of the sphere field gives
the whole-image generator's cells exactly and, without noise, its values
exactly; with noise, the same structure and Poisson-distributed cell sums."""
import dataclasses

import numpy as np
import pytest

from aprgen.apr_input import (CONFIGS, SphereConfig, deconv_config, sphere_apr, sphere_apr_slabs,
                              sphere_level_counts)

CASES = {
    "sphere64": CONFIGS["sphere64"],
    "odd_dims": SphereConfig((40, 72, 100), 6, 3.0, 9.0, 1, 77),
    "deconv96": deconv_config(96, 5),
    "sphere32": CONFIGS["sphere32"],
}


@pytest.mark.parametrize("name", sorted(CASES))
@pytest.mark.parametrize("slab", [4, 16])
def test_slabs_equal_whole_image_without_noise(name, slab):
    cfg = dataclasses.replace(CASES[name], noise=False)
    a = sphere_apr(cfg)
    b = sphere_apr_slabs(cfg, slab=slab)
    assert np.array_equal(a.y_idx, b.y_idx)
    assert np.array_equal(a.xz_end, b.xz_end)
    for l in range(a.l_min, a.l_max + 1):
        assert np.array_equal(a.cells[l], b.cells[l])
    assert np.array_equal(a.values, b.values)
    assert sum(sphere_level_counts(cfg).values()) == a.n_particles


def test_slabs_noise_statistics():
    """Cell sums are Poisson(lambda): (sum - lambda) / sqrt(lambda) has mean
    ~0 and variance ~1 over the ~30k cells."""
    cfg = CONFIGS["sphere64"]
    clean = sphere_apr(dataclasses.replace(cfg, noise=False))
    b = sphere_apr_slabs(cfg, slab=16, workers=2)
    assert np.array_equal(clean.y_idx, b.y_idx)
    cnt = np.concatenate([np.prod(np.minimum((clean.cells[l] + 1) * (1 << (clean.l_max - l)), 64)
                                  - clean.cells[l] * (1 << (clean.l_max - l)), axis=1)
                          for l in range(clean.l_min, clean.l_max + 1)]).astype(np.float64)
    lam = clean.values.astype(np.float64) * cnt
    z = (b.values.astype(np.float64) * cnt - lam) / np.sqrt(lam)
    assert abs(z.mean()) < 0.03 and abs(z.var() - 1.0) < 0.05, (z.mean(), z.var())
    # integer cell sums, and a different realisation per slab seed
    assert np.allclose(b.values * cnt, np.round(b.values * cnt), rtol=0, atol=1e-3 * cnt.max())
