"""APR construction on the device (``apr_sphere_field``) against the oracle's
construction (``oracle.construct``): the LinearAccess bit for bit, the
particle values (with and without noise) within the FP32-image bound; at
512^3 the partition against the independent input generator (``aprgen``)."""
import sys

import numpy as np
import pytest
import torch

from aprgen.apr_input import CONFIGS, SphereConfig, _sphere_params, sphere_apr
from oracle import access as A
from oracle import construct as K
from paper_2112_03592_amd import apr as G

pytestmark = pytest.mark.gpu

# the clean image is stored in FP32 between blur passes (three roundings of
# values <= 1000) and the block sums are FP64: relative error well below 1e-6
RTOL = 1e-6


def _random_case(seed, dims, n, rmin, rmax):
    rng = np.random.default_rng(seed)
    return dims, rng.uniform(0, 1, (n, 3)) * np.asarray(dims, np.float64), rng.uniform(rmin, rmax, n)


CASES = {
    "sphere32": lambda: (CONFIGS["sphere32"].dims, *_sphere_params(CONFIGS["sphere32"])),
    "sphere64": lambda: (CONFIGS["sphere64"].dims, *_sphere_params(CONFIGS["sphere64"])),
    "ragged40x33x50": lambda: _random_case(1, (40, 33, 50), 5, 2.0, 7.0),
    "ragged17x70x9": lambda: _random_case(2, (17, 70, 9), 4, 1.5, 5.0),
    "one_sphere_8": lambda: ((8, 8, 8), np.array([[4.0, 4.0, 4.0]]), np.array([2.0])),
    "no_sphere": lambda: ((12, 20, 16), np.zeros((0, 3)), np.zeros(0)),
}


def say(*a):
    print(*a, flush=True, file=sys.stderr)


@pytest.mark.parametrize("name", list(CASES))
@pytest.mark.parametrize("noise", [False, True])
def test_device_construction_matches_oracle(name, noise):
    dims, cen, rad = CASES[name]()
    l_min = 1
    say(f"construct {name} dims={dims} spheres={len(rad)} noise={noise}")
    la, cells = K.sphere_partition(dims, l_min, cen, rad)
    img = K.sphere_image(dims, cen, rad, 100.0, 1000.0, 1.0)
    want = K.cell_values(dims, l_min, la.l_max, cells, img, noise, 17)
    f = G.sphere_field(dims, l_min, cen, rad, edge_sigma=1.0, noise=noise, seed=17)
    assert f.l_max == la.l_max and f.n_particles == la.n
    assert np.array_equal(f.y_idx.astype(np.int64), la.y_idx)
    assert np.array_equal(f.xz_end.astype(np.int64), la.xz_end)
    got = f.values.cpu().numpy().astype(np.float64)
    np.testing.assert_allclose(got, want, rtol=RTOL)


def test_device_construction_builds_a_valid_access():
    dims, cen, rad = CASES["sphere64"]()
    f = G.sphere_field(dims, 2, cen, rad)
    la = A.LinearAccess(f.dims, f.l_min, f.l_max, f.y_idx, f.xz_end)
    assert A.check_partition(la) and A.check_balance(la)
    with G.AprAccess.from_input(f) as acc:   # validates partition and balance on the device
        assert acc.n_particles == f.n_particles


def test_device_partition_matches_generator_512():
    # the 512^3 bench field: the device partition equals the independent
    # slab generator's (same sphere list, same rule)
    cfg = CONFIGS["sphere512"]
    cen, rad = _sphere_params(cfg)
    say("generating sphere512 structure with aprgen (noise-free)")
    ref = sphere_apr(SphereConfig(cfg.dims, cfg.n_spheres, cfg.r_min, cfg.r_max, cfg.l_min, cfg.seed, noise=False))
    f = G.sphere_field(cfg.dims, cfg.l_min, cen, rad, noise=False)
    assert f.n_particles == ref.n_particles
    assert np.array_equal(f.y_idx, ref.y_idx)
    assert np.array_equal(f.xz_end, ref.xz_end.astype(np.uint64))
    # noise-free values: the two generators blur in FP32 with different
    # summation orders
    np.testing.assert_allclose(f.values.cpu().numpy(), ref.values, rtol=2e-6)
