"""Pins for the oracle's APR construction of the sphere fields (CPU only):
the counter-based generator against numpy's Philox, the partition against a
fully refined hand case, the validity and minimality of the partition, the
independent generator in ``aprgen`` on the small configurations, the image
blur against the separable kernel, and the noise statistics."""
import numpy as np
import pytest

from aprgen.apr_input import CONFIGS, SphereConfig, _sphere_params, sphere_apr
from oracle import access as A
from oracle import construct as K


def test_philox_matches_numpy_bit_generator():
    # numpy's Philox (4 x 64 bit, 10 rounds) increments its counter before
    # each block: its first block is the counter + 1
    rng = np.random.default_rng(3)
    for _ in range(5):
        key = rng.integers(0, 2**63, size=2, dtype=np.uint64)
        ctr = rng.integers(0, 2**63, size=4, dtype=np.uint64)
        bg = np.random.Philox(key=key, counter=ctr)
        want = bg.random_raw(4)
        c1 = ctr.copy()
        c1[0] += np.uint64(1)
        got = K.philox4x64([c1[0], c1[1], c1[2], c1[3]], [key[0], key[1]])
        assert [int(g) for g in got] == [int(w) for w in want]


def test_cell_normal_is_standard_and_keyed():
    keys = K.cell_key(np.full(20000, 7), np.arange(20000) // 100, np.arange(20000) % 100, 5)
    z = K.cell_normal(keys, seed=11)
    assert abs(z.mean()) < 0.03 and abs(z.std() - 1.0) < 0.03
    assert np.all(np.abs(z) <= 6.0)
    assert np.array_equal(z, K.cell_normal(keys, seed=11))
    assert not np.array_equal(z, K.cell_normal(keys, seed=12))


def test_fully_refined_hand_case():
    # one sphere (r = 1) at the centre of a 4^3 image: every level-0 and
    # level-1 cell box straddles the surface, so every pixel is a particle
    la, cells = K.sphere_partition((4, 4, 4), 0, [[2.0, 2.0, 2.0]], [1.0])
    assert la.l_max == 2
    assert la.y_idx.tolist() == [0, 1, 2, 3] * 16
    assert la.xz_end.tolist() == [0] + [0] * 4 + list(range(4, 68, 4))


def test_far_sphere_leaves_coarse_cells():
    # a sphere in a corner of a 64^3 image: coarse cells survive far from it
    la, cells = K.sphere_partition((64, 64, 64), 2, [[2.0, 2.0, 2.0]], [1.5])
    lv = {l: cells[l].shape[0] for l in cells}
    assert lv[2] > 0 and lv[la.l_max] > 0
    assert A.check_partition(la) and A.check_balance(la)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_partition_valid_and_minimal(seed):
    rng = np.random.default_rng(seed)
    dims = (20, 13, 24)
    cen = rng.uniform(0, 1, (3, 3)) * np.asarray(dims)
    rad = rng.uniform(1.5, 4.0, 3)
    l_max = A.finest_level(dims)
    rule = K.split_by_rule(dims, 1, l_max, cen, rad)
    split = K.balanced_splits(dims, 1, l_max, rule)
    la, cells = K.sphere_partition(dims, 1, cen, rad)
    assert A.check_partition(la) and A.check_balance(la)
    for l in range(1, l_max):
        # every split is asked for by the rule or by balance with level l+1
        if l + 1 < l_max:
            need = K._parents(K._touching(split[l + 1]), split[l].shape)
        else:
            need = np.zeros_like(split[l])
        assert not np.any(split[l] & ~(rule[l] | need))
        # no particle cell is one the rule splits
        c = cells[l]
        assert not np.any(rule[l][c[:, 0], c[:, 1], c[:, 2]])


@pytest.mark.parametrize("name", ["sphere32", "sphere64"])
def test_matches_independent_generator(name):
    cfg = CONFIGS[name]
    cen, rad = _sphere_params(cfg)
    la, cells = K.sphere_partition(cfg.dims, cfg.l_min, cen, rad)
    ref = sphere_apr(SphereConfig(cfg.dims, cfg.n_spheres, cfg.r_min, cfg.r_max, cfg.l_min, cfg.seed, noise=False))
    assert np.array_equal(la.y_idx, ref.y_idx.astype(np.int64))
    assert np.array_equal(la.xz_end, ref.xz_end.astype(np.int64))
    img = K.sphere_image(cfg.dims, cen, rad, 100.0, 1000.0, 1.0)
    v = K.cell_values(cfg.dims, cfg.l_min, la.l_max, cells, img, False, 0)
    # aprgen stores FP32 values
    np.testing.assert_allclose(v, ref.values, rtol=3e-7)


def test_image_blur_is_the_separable_gaussian():
    # one voxel of a tiny sphere: the blur is the outer product of the taps
    dims = (15, 15, 15)
    img = K.sphere_image(dims, [[7.5, 7.5, 7.5]], [0.1], 0.0, 1.0, 1.0)
    g = K.gaussian_taps(1.0)
    assert g.shape == (9,) and abs(g.sum() - 1.0) < 1e-15
    want = np.zeros(dims)
    want[3:12, 3:12, 3:12] = g[:, None, None] * g[None, :, None] * g[None, None, :]
    np.testing.assert_allclose(img, want, atol=1e-16)
    # zeros outside the image: a voxel at the corner loses the outside mass
    img = K.sphere_image(dims, [[0.5, 0.5, 0.5]], [0.1], 0.0, 1.0, 1.0)
    assert abs(img.sum() - g[4:].sum() ** 3) < 1e-14


def test_values_are_means_and_noise_scales_with_sqrt_sum():
    dims = (16, 16, 16)
    la, cells = K.sphere_partition(dims, 1, [[8.0, 8.0, 8.0]], [3.0])
    flat = np.full(dims, 250.0)
    v = K.cell_values(dims, 1, la.l_max, cells, flat, False, 0)
    assert np.all(v == 250.0)
    vn = K.cell_values(dims, 1, la.l_max, cells, flat, True, 5)
    n = np.concatenate([np.full(cells[l].shape[0], 8.0 ** (la.l_max - l)) for l in range(1, la.l_max + 1)])
    z = (vn - v) * n / np.sqrt(250.0 * n)   # the Z of each cell
    assert abs(z.mean()) < 0.1 and abs(z.std() - 1.0) < 0.1
