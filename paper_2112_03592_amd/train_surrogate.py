"""Train the Richardson-Lucy surrogate on the GPU and store it.

    python -m paper_2112_03592_amd.train_surrogate [--steps N] [--out PATH]

Training pairs come from the plain method: sphere-field APRs blurred by the
5^3 Gaussian PSF (sigma 1.5) with Poisson noise, and 10 iterations of APR
Richardson-Lucy computed by ``apr_richardson_lucy``.  Steps:
  1. the start exponent p of the over-relaxed iterations on a grid,
  2. the network by Adam on (start, target) pairs, one APR per step,
  3. the monitor threshold tau on held-out APRs (every held-out APR with
     monitor <= tau has relative error <= the target).
"""
from __future__ import annotations

import argparse
import os
import sys
import time

import numpy as np
import torch

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

from aprgen.apr_input import deconv_psf, deconv_set  # noqa: E402
from paper_2112_03592_amd import apr as G  # noqa: E402
from paper_2112_03592_amd import surrogate as N  # noqa: E402

DEFAULT_OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "weights", "rl10_surrogate.npz")
TRAIN_EDGES = (64, 80, 96, 112, 128, 144, 160, 176, 192, 208, 224, 240, 256, 112, 160, 208)
TRAIN_SEED = 5000
CAL_EDGES = (72, 96, 112, 128, 160, 192, 224, 256, 288, 128)
CAL_SEED = 6000
TARGET = 2e-2


def say(*a):
    print(*a, flush=True)


def device_cases(apr_inputs, rl: N.RichardsonLucy, n_iter: int):
    out = []
    for inp in apr_inputs:
        acc = G.AprAccess.from_input(inp, gather=(3,))
        u = torch.from_numpy(np.maximum(inp.values, 0).astype(np.float32)).cuda()
        out.append((acc, u, rl(acc, u, n_iter)))
    return out


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--steps", type=int, default=20000)
    ap.add_argument("--lr", type=float, default=2e-3)
    ap.add_argument("--n-pre", type=int, default=2)
    ap.add_argument("--layers", type=int, default=4)
    ap.add_argument("--channels", type=int, default=16)
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--workers", type=int, default=8)
    ap.add_argument("--out", default=DEFAULT_OUT)
    ap.add_argument("--train-edges", default=",".join(map(str, TRAIN_EDGES)), help="edges of the training APRs")
    ap.add_argument("--cal-edges", default=",".join(map(str, CAL_EDGES)), help="edges of the held-out APRs")
    a = ap.parse_args(argv)
    t0 = time.time()
    psf = deconv_psf()
    # generated in worker processes before this process touches the GPU
    train_edges = tuple(int(e) for e in a.train_edges.split(","))
    cal_edges = tuple(int(e) for e in a.cal_edges.split(","))
    train_in = deconv_set(train_edges, TRAIN_SEED, a.workers)
    cal_in = deconv_set(cal_edges, CAL_SEED, a.workers)
    rl = N.RichardsonLucy(psf)
    ws = G.Workspace(16)
    say(f"generated {len(train_in)} + {len(cal_in)} APRs in {time.time() - t0:.1f} s; particles "
        f"{sum(x.n_particles for x in train_in)} + {sum(x.n_particles for x in cal_in)}")
    train = device_cases(train_in, rl, 10)
    cal = device_cases(cal_in, rl, 10)
    power = N.calibrate_power(rl, train, a.n_pre, ws)
    base_err = [N.rel_error(rl(acc, u, a.n_pre, power=power), t, ws) for acc, u, t in cal]
    say(f"start: {a.n_pre} iterations, power {power}; held-out error {np.round(base_err, 4).tolist()}")
    net = N.SurrogateNet(N.NetConfig(channels=a.channels, layers=a.layers, seed=a.seed))
    cases = [(acc, rl(acc, u, a.n_pre, power=power), t) for acc, u, t in train]
    t1 = time.time()
    losses = N.train(net, cases, a.steps, lr=a.lr, log_every=max(1, a.steps // 20),
                     progress=lambda it, loss: say(f"  step {it}: loss {loss:.4f}"))
    torch.cuda.synchronize()
    say(f"trained {a.steps} steps in {time.time() - t1:.1f} s; loss {np.round(losses, 4).tolist()}")
    sur = N.RLSurrogate(net, psf, 10, a.n_pre, power)
    mon, err = [], []
    for acc, u, t in cal:
        s, out = sur.estimate(acc, u)
        mon.append(float(np.sqrt(out[0].item())))
        err.append(N.rel_error(s, t, ws))
    sur.tau = N.calibrate_tau(mon, err, TARGET)
    say(f"held-out error {np.round(err, 4).tolist()}\nmonitor {np.round(mon, 4).tolist()}\ntau {sur.tau}")
    os.makedirs(os.path.dirname(os.path.abspath(a.out)), exist_ok=True)
    N.save_surrogate(a.out, sur, train_loss=np.asarray(losses), cal_monitor=np.asarray(mon),
                     cal_error=np.asarray(err), cal_base_error=np.asarray(base_err),
                     train_edges=np.asarray(train_edges), cal_edges=np.asarray(cal_edges),
                     steps=np.array(a.steps), lr=np.array(a.lr))
    say(f"wrote {a.out} ({time.time() - t0:.1f} s)")
    for acc, _, _ in train + cal:
        acc.close()


if __name__ == "__main__":
    main()
