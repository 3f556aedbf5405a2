"""Pins for the oracle's LinearAccess and tree structure (CPU only)."""
import json
import os

import numpy as np
import pytest

from aprgen.apr_input import CONFIGS, random_apr, sphere_apr, dense_apr
from oracle import access as A
from oracle.tree import fill_tree

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _gold(name):
    with open(os.path.join(GOLD, name)) as f:
        return json.load(f)


def _la(inp):
    return A.LinearAccess(inp.dims, inp.l_min, inp.l_max, inp.y_idx, inp.xz_end)


def test_golden_tiny4_encoding_and_tree():
    g = _gold("tiny4.json")
    cells = {int(k): np.array(v) for k, v in g["cells"].items()}
    la = A.from_cells(g["dims"], g["l_min"], g["l_max"], cells)
    assert la.y_idx.tolist() == g["y_idx"]
    assert la.xz_end.tolist() == g["xz_end"]
    # get_row of Algorithm 1 reproduces the rows
    assert la.get_row(1, 0, 0) == (0, 1)
    assert la.get_row(2, 1, 1) == (13, 15)
    assert la.get_row(2, 3, 3) == (15, 15)
    tr = A.tree_structure(la)
    assert (tr.l_min, tr.l_max) == (g["tree_l_min"], g["tree_l_max"])
    assert tr.y_idx.tolist() == g["tree_y_idx"]
    assert tr.xz_end.tolist() == g["tree_xz_end"]
    t = fill_tree(la, tr, np.array(g["values"], float))
    assert t.tolist() == g["tree_values"]


def test_golden_partial_boundary_tree_values():
    g = _gold("partial3.json")
    inp = dense_apr(g["dims"], l_min=g["l_min"], values=np.array(g["values"], np.float32))
    la = _la(inp)
    tr = A.tree_structure(la)
    t = fill_tree(la, tr, inp.values)
    assert t.tolist() == g["tree_values"]


def test_generator_encoding_matches_oracle_encoding():
    inp = random_apr((9, 12, 7), l_min=1, seed=3)
    la = A.from_cells(inp.dims, inp.l_min, inp.l_max, {l: inp.cells[l] for l in inp.cells})
    assert np.array_equal(la.y_idx, inp.y_idx.astype(np.int64))
    assert np.array_equal(la.xz_end, inp.xz_end.astype(np.int64))


def test_iteration_order_is_l_z_x_y():
    inp = random_apr((8, 8, 8), l_min=1, seed=5)
    la = _la(inp)
    seq = list(la.iterate())
    assert [s[4] for s in seq] == list(range(la.n))
    keys = [(l, z, x, y) for (l, z, x, y, _) in seq]
    assert keys == sorted(keys)
    for l in range(la.l_min, la.l_max + 1):
        c = la.cells(l)
        ref = [k[1:] for k in keys if k[0] == l]
        assert [tuple(r) for r in c.tolist()] == ref


@pytest.mark.parametrize("dims,l_min,seed,p", [
    ((8, 8, 8), 0, 0, 0.3), ((16, 16, 16), 1, 1, 0.2), ((9, 12, 7), 1, 2, 0.3),
    ((5, 16, 3), 0, 3, 0.5), ((16, 8, 32), 2, 4, 0.15), ((1, 1, 1), 0, 5, 0.5),
])
def test_tree_three_ways_and_validity(dims, l_min, seed, p):
    inp = random_apr(dims, l_min=l_min, seed=seed, p_refine=p)
    la = _la(inp)
    assert A.check_partition(la)
    assert A.check_balance(la)
    t1 = A.tree_structure(la)
    t2 = A.tree_structure_by_painting(la)
    assert np.array_equal(t1.y_idx, t2.y_idx)
    assert np.array_equal(t1.xz_end, t2.xz_end)
    assert A.check_parents_by_synchronized_iteration(la, t1)


def test_unbalanced_apr_is_detected():
    found = False
    for seed in range(20):
        inp = random_apr((16, 16, 16), l_min=0, seed=seed, p_refine=0.08, balanced=False)
        la = _la(inp)
        assert A.check_partition(la)
        if not A.check_balance(la):
            found = True
            break
    assert found


def test_sphere64_is_a_balanced_partition():
    inp = sphere_apr(CONFIGS["sphere64"])
    la = _la(inp)
    assert A.check_partition(la)
    assert A.check_balance(la)
    assert 0.9 * 29695 < la.n < 1.1 * 29695
