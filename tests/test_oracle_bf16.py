"""Pins of the oracle's BF16 rounding and its stored tree mean
(oracle/bf16.py): torch's own float32 -> bfloat16 conversion on FP32 values
of every magnitude, hand-checked ties, and the stored mean on hand cases and
through the tree fill."""
import numpy as np
import torch

from oracle.bf16 import round_bf16, store_mean_bf16


def _torch_bf16(x32):
    return torch.from_numpy(x32).to(torch.bfloat16).float().numpy().astype(np.float64)


def test_matches_torch_conversion():
    rng = np.random.default_rng(5)
    x = rng.normal(size=200000) * 10.0 ** rng.uniform(-40, 38, 200000)
    # every tie between neighbouring BF16 values on a few binades, and the
    # subnormal range
    g = np.arange(0, 257, dtype=np.float64)
    ties = np.concatenate([(1.0 + (g + 0.5) / 128) * 2.0 ** e for e in (-130, -20, 0, 7, 100)])
    sub = np.arange(1, 300, dtype=np.float64) * 2.0 ** -140
    x = np.concatenate([x, ties, -ties, sub, -sub, [0.0, -0.0, 3.0e38, -3.3e38]]).astype(np.float32)
    got = round_bf16(x.astype(np.float64))
    want = _torch_bf16(x)
    assert np.array_equal(got, want)
    assert np.array_equal(np.signbit(got), np.signbit(want))


def test_hand_ties_and_limits():
    # 1 + 2^-8 lies halfway between 1 (fraction 0) and 1 + 2^-7 (fraction 1): even -> 1
    assert round_bf16([1.0 + 2.0 ** -8])[0] == 1.0
    # 1 + 3*2^-8 lies halfway between fractions 1 and 2: even -> 1 + 2^-6
    assert round_bf16([1.0 + 3 * 2.0 ** -8])[0] == 1.0 + 2.0 ** -6
    assert round_bf16([1.0 + 2.0 ** -8 + 2.0 ** -20])[0] == 1.0 + 2.0 ** -7
    # 255.5 -> 256 (rounds into the next binade); 0.1 -> 0.10009765625
    assert round_bf16([255.5])[0] == 256.0
    assert round_bf16([0.1])[0] == 0.10009765625
    assert np.isinf(round_bf16([3.4e38])[0]) and round_bf16([3.389e38])[0] == (2 - 2.0 ** -7) * 2.0 ** 127
    assert np.isnan(round_bf16([np.nan])[0])


def test_idempotent_monotone_half_unit():
    x = np.sort(np.random.default_rng(6).normal(size=50000) * 1e3).astype(np.float32).astype(np.float64)
    r = round_bf16(x)
    assert np.array_equal(round_bf16(r), r)
    assert np.all(np.diff(r) >= 0)
    assert np.all(np.abs(r - x) <= np.abs(x) * 2.0 ** -8)


def test_store_mean():
    # (1 + 1.5 + 2) / 3 = 1.5 exactly; 10 / 3 = 3.333.. -> FP32 3.3333333 -> BF16 213 * 2^-6 = 3.328125;
    # 1.00390625 = 1 + 2^-8 is a tie -> 1.0 (even)
    got = store_mean_bf16(np.array([[4.5], [10.0], [2.0078125]]), np.array([[3], [3], [2]]))
    assert np.array_equal(got[:, 0], [1.5, 3.328125, 1.0])
    try:
        store_mean_bf16(np.array([[1.0 + 2.0 ** -30]]), np.array([[1]]))
    except ValueError:
        pass
    else:
        raise AssertionError("an inexact FP32 sum must be rejected")


def test_store_mean_through_the_fill():
    """With BF16 storage every tree value is a BF16 number, and a node whose
    children are all particles holds the BF16-rounded FP32 mean of them."""
    from aprgen.apr_input import random_apr
    from oracle import access as A
    from oracle.tree import fill_tree
    inp = random_apr((16, 16, 16), l_min=1, seed=2, p_refine=0.25)
    la = A.LinearAccess(inp.dims, inp.l_min, inp.l_max, inp.y_idx, inp.xz_end)
    tr = A.tree_structure(la)
    x = round_bf16(np.random.default_rng(1).uniform(1, 4, la.n))
    t = fill_tree(la, tr, x, store=store_mean_bf16)
    assert np.array_equal(round_bf16(t), t)
    exact = fill_tree(la, tr, x)
    # one rounding per level: at most (levels) BF16 half-units apart from the exact mean
    nl = la.l_max - la.l_min + 1
    assert np.all(np.abs(t - exact) <= exact * nl * 2.0 ** -8)
    # finest tree level: children are particles only, one rounding of the FP32 mean
    lt = la.l_max - 1
    b, e = tr.level_range(lt)
    cells = tr.cells(lt)
    for i in range(b, min(e, b + 50)):
        c = cells[i - b]
        vals = []
        for dz in (0, 1):
            for dx in (0, 1):
                for dy in (0, 1):
                    j = la.lookup(lt + 1, (2 * c + np.array([dz, dx, dy]))[None, :])[0]
                    if j >= 0:
                        vals.append(x[j])
        m32 = np.float32(np.float32(np.sum(vals)) / np.float32(len(vals)))
        assert t[i] == round_bf16([float(m32)])[0]
