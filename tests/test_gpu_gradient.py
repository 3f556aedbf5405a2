"""The resolution-adaptive gradient magnitude (Section 4.3, Eq. adapt_grad,
Sobel filters; ``apr_conv`` with APR_EPI_GRADMAG, three stencils on one LDS
patch) against the FP64 oracle: small cases in full, the 512^3 field on a
seeded sample, BF16 values."""
import sys

import numpy as np
import pytest
import torch

from aprgen.apr_input import cached_sphere_apr, sobel_stencils
from oracle import access as A
from oracle import conv as C
from oracle import stencil as S
from oracle.tree import fill_tree as oracle_fill
from paper_2112_03592_amd import apr as G
from tests.gpu_common import SMALL_CASES, linear_access

pytestmark = pytest.mark.gpu


def _scale(la, tr, x64, w3, sample=None):
    """sqrt(sum_j M_j^2), M_j = sum_o |w_j[o]| |V(c_p + o)|: bounds the
    rounding of each component and hence of the magnitude."""
    xa = np.abs(x64)
    tva = oracle_fill(la, tr, xa)
    sq = 0.0
    for j in range(3):
        wj = np.abs(w3[:, j])
        if sample is None:
            m = C.apr_conv(la, xa, wj, tree=tr, tvals=tva)
        else:
            m = C.apr_conv_keyed(la, xa, wj, sample, tree=tr, tvals=tva)[:, 0]
        sq = sq + np.asarray(m).reshape(-1) ** 2
    return np.sqrt(sq)


def _oracle_sobel_levels(la):
    """The reference side's per-level Sobel stencils [nl, 3, 3, 3, 3], built by
    the oracle (Eq. adapt_grad), independently of the library's."""
    return np.moveaxis(np.stack([S.level_stencils(s_, S.ADAPTIVE, la.l_min, la.l_max) for s_ in sobel_stencils()]),
                       0, 1)


@pytest.mark.parametrize("name", ["rand16_l1", "rand33x20x70", "rand_long_y", "sphere32", "sphere64",
                                  "dense13x11x70", "single_cell"])
@pytest.mark.parametrize("storage", ["f32", "bf16"])
def test_gradient_magnitude(name, storage):
    inp = SMALL_CASES[name]()
    la = linear_access(inp)
    tr = A.tree_structure(la)
    w3 = G.stencil_levels(sobel_stencils(), "adaptive", 3, la.l_min, la.l_max)     # [nl, 3, 3, 3, 3]
    x = torch.from_numpy(inp.values).cuda()
    if storage == "bf16":
        x = x.to(torch.bfloat16)
    x64 = x.float().cpu().numpy().astype(np.float64)
    w64 = _oracle_sobel_levels(la)
    ref = C.gradient_magnitude(la, x64, w64, tree=tr)
    scale = _scale(la, tr, x64, w64)
    with G.AprAccess.from_input(inp) as acc:
        t = G.fill_tree(acc, x)
        y = G.gradient_magnitude(acc, x, t, torch.from_numpy(w3).cuda()).cpu().numpy().astype(np.float64)
    tol = 1e-5 if storage == "f32" else 1e-2
    assert np.all(np.abs(y - ref) <= tol * scale + 1e-30), float(np.max(np.abs(y - ref) / np.maximum(scale, 1e-30)))


def test_gradient_magnitude_sphere512_sampled():
    print("sphere512 gradient magnitude", flush=True, file=sys.stderr)
    inp = cached_sphere_apr("sphere512")
    la = linear_access(inp)
    tr = A.tree_structure(la)
    w3 = G.stencil_levels(sobel_stencils(), "adaptive", 3, la.l_min, la.l_max)
    smp = np.sort(np.random.default_rng(11).choice(la.n, 4096, replace=False))
    x64 = inp.values.astype(np.float64)
    w64 = _oracle_sobel_levels(la)
    ref = C.gradient_magnitude(la, x64, w64, tree=tr, sample=smp)
    scale = _scale(la, tr, x64, w64, sample=smp)
    with G.AprAccess.from_input(inp) as acc:
        x = torch.from_numpy(inp.values).cuda()
        t = G.fill_tree(acc, x)
        y = G.gradient_magnitude(acc, x, t, torch.from_numpy(w3).cuda()).cpu().numpy()
    assert np.all(np.abs(y[smp] - ref) <= 1e-5 * scale)


def test_gradient_magnitude_rejects():
    inp = SMALL_CASES["sphere32"]()
    with G.AprAccess.from_input(inp) as acc:
        x = torch.zeros(acc.n_particles, device="cuda")
        t = G.fill_tree(acc, x)
        with pytest.raises(ValueError):
            G.gradient_magnitude(acc, x, t, torch.zeros(acc.n_levels, 3, 5, 5, 5, device="cuda"))
