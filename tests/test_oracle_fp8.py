"""Pins of the oracle's FP8 E4M3 rounding (oracle/fp8.py): the format's grid
from its definition, torch's own float8_e4m3fn conversion on the finite
range, hand-checked ties and the saturation reading."""
import numpy as np
import torch

from oracle.fp8 import e4m3_values, round_e4m3, round_e4m3_codes


def test_grid():
    v = e4m3_values()
    assert np.isnan(v[0x7F]) and np.isnan(v[0xFF])
    pos = v[:127]
    assert np.all(np.diff(pos) > 0)
    assert pos[126] == 448.0 and pos[1] == 2.0 ** -9 and pos[8] == 2.0 ** -6
    assert np.array_equal(v[128:255], -pos)
    # the codes read as torch reads them
    t = torch.arange(256, dtype=torch.int32).to(torch.uint8).view(torch.float8_e4m3fn).float().numpy()
    assert np.array_equal(np.nan_to_num(t.astype(np.float64), nan=1e9), np.nan_to_num(v, nan=1e9))


def test_matches_torch_on_the_finite_range():
    rng = np.random.default_rng(3)
    x = rng.normal(size=100000) * 10.0 ** rng.uniform(-4, 2.6, 100000)
    mid = (e4m3_values()[:126] + e4m3_values()[1:127]) / 2          # every tie
    x = np.concatenate([x, mid, -mid, e4m3_values()[:127]]).astype(np.float32)
    x = x[np.abs(x) < 464]
    t = torch.from_numpy(x).to(torch.float8_e4m3fn).view(torch.uint8).numpy()
    assert np.array_equal(round_e4m3_codes(x.astype(np.float64)), t)


def test_ties_saturation_nan():
    assert round_e4m3([1.0625])[0] == 1.0          # between codes 56 and 57: even 56
    assert round_e4m3([1.1875])[0] == 1.25         # between codes 57 and 58: even 58
    assert round_e4m3([2.0 ** -10])[0] == 0.0      # half the smallest subnormal: even code 0
    assert round_e4m3([3 * 2.0 ** -10])[0] == 2.0 ** -8
    assert np.array_equal(round_e4m3([463.9, 464.0, 500.0, 1e30, np.inf, -np.inf]),
                          [448.0, 448.0, 448.0, 448.0, 448.0, -448.0])
    assert np.isnan(round_e4m3([np.nan])[0])
    c = round_e4m3_codes([-0.0, 0.0])
    assert c[0] == 0x80 and c[1] == 0


def test_idempotent_and_monotone():
    x = np.sort(np.random.default_rng(4).normal(size=20000) * 50)
    r = round_e4m3(x)
    assert np.array_equal(round_e4m3(r), r)
    assert np.all(np.diff(r) >= 0)
    # relative error bounded by half an ulp (2^-4) on the normal range
    n = (np.abs(x) >= 2.0 ** -6) & (np.abs(x) <= 448)
    assert np.all(np.abs(r[n] - x[n]) <= np.abs(x[n]) * 2.0 ** -4 + 1e-15)


def test_store_mean():
    from oracle.fp8 import store_mean_e4m3
    # (1 + 1.125 + 1.25) / 3 = 1.125 exactly; 7 / 3 = 2.333.. -> 2.25; a tie 2.125 -> 2.0 (even)
    got = store_mean_e4m3(np.array([[3.375], [7.0], [8.5]]), np.array([[3], [3], [4]]))
    assert np.array_equal(got[:, 0], [1.125, 2.25, 2.0])
