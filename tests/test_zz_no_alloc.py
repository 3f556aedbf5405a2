"""The allocation-free Richardson-Lucy entry point (apr_richardson_lucy_static)
against the workspace entry point (apr_richardson_lucy) on the same inputs:
two calls in a row on the shared static scratch, the second on a smaller
APR, each equal to the workspace result; a handle beyond the scratch's size
is rejected without a launch; the entry point captured in a HIP graph
replays to the eager result."""
import sys

import numpy as np
import pytest
import torch

from aprgen.apr_input import deconv_config, deconv_psf, dense_apr, sphere_apr
from paper_2112_03592_amd import _lib as L
from paper_2112_03592_amd import apr as G

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True, file=sys.stderr)


def test_static_rl_two_calls_then_smaller():
    """Workspace results first, then two static calls back to back (the
    second on a smaller APR, so stale contents of the larger call remain in
    the scratch past its end)."""
    psf = deconv_psf()
    k = psf.shape[-1]
    big = sphere_apr(deconv_config(96, 8300))
    small = sphere_apr(deconv_config(48, 8301))
    assert small.n_particles < big.n_particles
    runs = []
    for name, inp, n_iter, power in (("96^3", big, 10, 1.0), ("48^3", small, 3, 2.2)):
        acc = G.AprAccess.from_input(inp)
        u = torch.from_numpy(np.maximum(inp.values, 0).astype(np.float32)).cuda()
        w = torch.from_numpy(G.stencil_levels(psf, "restrict", k, acc.l_min, acc.l_max)).cuda()
        wf = torch.from_numpy(G.stencil_levels(psf, "restrict", k, acc.l_min, acc.l_max, flip=True)).cuda()
        ref = G.richardson_lucy(acc, u, psf, n_iter, power=power)
        runs.append((name, acc, u, w, wf, n_iter, power, ref))
    torch.cuda.synchronize()
    outs = []
    for name, acc, u, w, wf, n_iter, power, ref in runs:
        say("static RL", name, acc.n_particles, "particles,", n_iter, "iterations")
        out = torch.full_like(u, float("nan"))
        G.richardson_lucy_static(acc, u, w, wf, n_iter, out, power=power)
        outs.append(out)
    torch.cuda.synchronize()
    for (name, acc, u, w, wf, n_iter, power, ref), out in zip(runs, outs):
        got, want = out.cpu().numpy(), ref.cpu().numpy()
        assert np.isfinite(got).all()
        # the same kernels in the same order on the same inputs: bit-identical
        assert np.array_equal(got, want), (name, float(np.max(np.abs(got - want))))
        acc.close()


def test_static_rl_rejects_a_handle_beyond_the_scratch():
    inp = dense_apr((180, 180, 180), l_min=2, seed=3)          # 5.8M particles: beyond 2^24 floats
    psf = deconv_psf()
    with G.AprAccess.from_input(inp) as acc:
        assert acc.n_tree + 3 * acc.n_particles + 1088 > L.APR_RL_STATIC_FLOATS
        u = torch.from_numpy(inp.values).cuda()
        w = torch.from_numpy(G.stencil_levels(psf, "restrict", 5, acc.l_min, acc.l_max)).cuda()
        out = torch.zeros_like(u)
        with pytest.raises(L.AprError) as e:
            G.richardson_lucy_static(acc, u, w, w, 2, out)
        assert e.value.status == L.APR_EINVAL and "static scratch" in str(e.value)
        torch.cuda.synchronize()
        assert float(out.abs().max()) == 0.0                    # nothing was launched


def test_static_rl_replayed_from_a_captured_graph():
    """The allocation-free entry point captured in a HIP graph (its launches
    are kernel nodes only): three replays, with eager calls and
    synchronisations between them, each equal bit for bit to the eager result."""
    psf = deconv_psf()
    k = psf.shape[-1]
    inp = sphere_apr(deconv_config(64, 8302))
    acc = G.AprAccess.from_input(inp)
    u = torch.from_numpy(np.maximum(inp.values, 0).astype(np.float32)).cuda()
    w = torch.from_numpy(G.stencil_levels(psf, "restrict", k, acc.l_min, acc.l_max)).cuda()
    wf = torch.from_numpy(G.stencil_levels(psf, "restrict", k, acc.l_min, acc.l_max, flip=True)).cuda()
    out = torch.empty_like(u)
    say("static RL graph capture, 64^3", acc.n_particles)
    G.richardson_lucy_static(acc, u, w, wf, 10, out=out)
    torch.cuda.synchronize()
    ref = out.clone()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        G.richardson_lucy_static(acc, u, w, wf, 10, out=out)
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        G.richardson_lucy_static(acc, u, w, wf, 10, out=out)
    torch.cuda.synchronize()
    scratch = torch.empty_like(u)
    for r in range(3):
        out.fill_(-1.0)
        torch.cuda.synchronize()
        g.replay()
        torch.cuda.synchronize()
        assert torch.equal(out, ref), f"replay {r}"
        G.richardson_lucy_static(acc, u, w, wf, 3, out=scratch)   # eager work between replays
        torch.cuda.synchronize()
    del g
    acc.close()
