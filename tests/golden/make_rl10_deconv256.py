"""Writes rl10_deconv256.npz: the FP64 oracle's 10-iteration APR
Richardson-Lucy (Section 6.2, restricted 5^3 PSF, i_0 = u) on the 256^3
deconvolution APR of seed 7000 (the first APR of the surrogate benchmark
batch), stored rounded to FP32, with a digest of the input it was computed
from.  Calls only the oracle and the seeded input generator; about three
minutes on one core.

    python tests/golden/make_rl10_deconv256.py
"""
import os
import sys

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

from aprgen.apr_input import deconv_psf, deconv_set, input_digest  # noqa: E402
from oracle import access as A  # noqa: E402
from oracle import rl as RL  # noqa: E402

EDGE, SEED, N_ITER = 256, 7000, 10
OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "rl10_deconv256.npz")


def main():
    inp = deconv_set([EDGE], SEED)[0]
    la = A.LinearAccess(inp.dims, inp.l_min, inp.l_max, inp.y_idx, inp.xz_end)
    u = np.maximum(np.asarray(inp.values, np.float64), 0.0)
    out = RL.richardson_lucy(la, u, deconv_psf(), N_ITER)
    np.savez_compressed(OUT, rl10=out.astype(np.float32), digest=np.array(input_digest(inp)),
                        edge=EDGE, seed=SEED, n_iter=N_ITER)
    print("wrote", OUT, out.shape)


if __name__ == "__main__":
    main()
