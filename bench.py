#!/usr/bin/env python3
"""Throughput of APR-native convolution on one MI355X.

One step = tree fill + 3^3 APR convolution + 5^3 APR convolution of the same
particle values (the tree is shared by both filters), FP32, on the
2048 x 2048 x 1024 sphere-field APR at ~50 pixels per particle (86.6M
particles, levels 2..11), built on the device by ``apr_sphere_field``.
Inputs are resident in device memory before timing starts; the access
structure (tree structure, tile list and windows) is built once, outside the
timed region.

Prints one JSON line (see the design doc for the fields).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "Gparticles/s + pixel-equiv GB/s (3³/5³ APR conv); surrogate-vs-plain RL speedup"
HBM_PEAK_GBPS = 8000.0
# FP32 vector FMA without packed math (the library is built with packed FP32
# disabled): 256 CUs x 64 lanes x 2 FLOP x 2.4 GHz
FP32_VALU_PEAK_TFLOPS = 256 * 64 * 2 * 2.4e9 / 1e12


KERNEL_SOURCES = {"conv3": ["conv.hip", "common.hpp"], "conv5": ["conv.hip", "common.hpp"],
                  "fill": ["tree.hip", "common.hpp"], "gradmag": ["conv.hip", "common.hpp"]}


def source_hash(kernel: str = "conv5") -> str:
    """Hash of the sources that define one kernel (stale counters are dropped)."""
    h = hashlib.sha1()
    for name in KERNEL_SOURCES[kernel]:
        with open(os.path.join(ROOT, "paper_2112_03592_amd", "csrc", name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:12]


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def conv_bytes(n_p, n_t, rows, trows, bv=4):
    """Algorithmic bytes of one convolution: particle values and y read as
    centre / same-level sources, read again as level-(l-1) sources (an upper
    bound: every particle once), tree values and y read once, row ends read
    once, outputs written once."""
    return n_p * (bv + 2) + n_p * (bv + 2) + n_t * (bv + 2) + n_p * bv + 4 * (rows + trows)


def fill_bytes(n_p, n_t, rows, trows, bv=4):
    """Tree fill over the child map: the map (8 x u32 per node) and every
    particle value read once, tree values written and read back once as
    children of the next coarser level."""
    return n_p * bv + n_t * (32 + 2 * bv)


def corner_block(inp, values, edge: int):
    """The APR of the corner cube [0, edge)^3 of the image: the particles whose
    cells lie in it (edge a multiple of the coarsest cell, so none straddles),
    as an APR of its own (levels shift by l_max - log2(edge)); values gathered
    from the device tensor."""
    import numpy as np
    import torch
    from types import SimpleNamespace
    dims, l_min, l_max = inp.dims, inp.l_min, inp.l_max
    ds = l_max - (edge.bit_length() - 1)
    y_all = np.asarray(inp.y_idx)
    e_all = np.asarray(inp.xz_end).astype(np.int64)
    ys, cnts, idxs = [], [], []
    row0 = 0
    for l in range(l_min, l_max + 1):
        s = 1 << (l_max - l)
        dz, dx = -(-dims[0] // s), -(-dims[1] // s)
        lim = edge // s
        zz, xx = np.meshgrid(np.arange(lim), np.arange(lim), indexing="ij")
        rows = row0 + zz.ravel() * dx + xx.ravel()
        e = e_all[rows]
        b = np.where(rows > 0, e_all[np.maximum(rows - 1, 0)], 0)
        n = e - b
        first = np.repeat(b - np.concatenate([[0], np.cumsum(n)[:-1]]), n)
        idx = first + np.arange(int(n.sum()))
        y = y_all[idx]
        keep = y < lim
        rid = np.repeat(np.arange(rows.size), n)
        cnts.append(np.bincount(rid[keep], minlength=rows.size))
        ys.append(y[keep])
        idxs.append(idx[keep])
        row0 += dz * dx
    idx = np.concatenate(idxs)
    vals = values[torch.from_numpy(idx).to(values.device)].cpu().numpy()
    return SimpleNamespace(dims=(edge, edge, edge), l_min=l_min - ds, l_max=l_max - ds,
                           y_idx=np.concatenate(ys).astype(np.uint16),
                           xz_end=np.cumsum(np.concatenate(cnts)).astype(np.uint64), values=vals,
                           n_particles=int(idx.size))


def cpu_baseline(block, n_total: int, sample: int):
    """The FP64 oracle on this host, one thread, on a bounded sample of the
    workload: the APR of a corner cube of the image (tree structure, tree
    fill) and a seeded sample of its particles (keyed 3^3 and 5^3
    convolution); the per-particle times are extrapolated to all n_total
    particles."""
    import numpy as np
    from threadpoolctl import threadpool_limits
    from oracle import access as A
    from oracle import conv as C
    from oracle import stencil as S
    from oracle.tree import fill_tree
    with threadpool_limits(1):
        la = A.LinearAccess(block.dims, block.l_min, block.l_max, block.y_idx, block.xz_end)
        t0 = time.perf_counter()
        tr = A.tree_structure(la)
        x = np.asarray(block.values, np.float64)
        tv = fill_tree(la, tr, x)
        t_fill = time.perf_counter() - t0
        smp = np.sort(np.random.default_rng(0).choice(la.n, min(sample, la.n), replace=False))
        ws = {k: S.level_stencils(S.gaussian_stencil(k, 1.0), S.SAME, la.l_min, la.l_max) for k in (3, 5)}
        # a keyed call has fixed parts: lookup structures built on first use
        # (once per run) and a particle table built per call; the rest scales
        # with the particles it serves
        t0 = time.perf_counter()
        C.apr_conv_keyed(la, x, ws[3], smp[:1], tree=tr, tvals=tv)
        t_init = time.perf_counter() - t0
        t_conv = t_call = 0.0
        for k in (3, 5):
            t0 = time.perf_counter()
            C.apr_conv_keyed(la, x, ws[k], smp, tree=tr, tvals=tv)
            t1 = time.perf_counter()
            C.apr_conv_keyed(la, x, ws[k], smp[:1], tree=tr, tvals=tv)
            t_conv += t1 - t0
            t_call += time.perf_counter() - t1
    per_p = t_fill / la.n + max(t_conv - t_call, 0.0) / smp.size
    step = per_p * n_total
    return {"value": n_total / step / 1e9, "unit": "Gparticles/s", "cores": 1, "kind": "oracle",
            "sample": (f"FP64 oracle, 1 thread, on the APR of the {block.dims[0]}^3 corner cube of the image "
                       f"({la.n} particles): tree structure and fill ({t_fill:.2f} s) and keyed 3^3 + 5^3 "
                       f"convolution of {smp.size} seeded particles ({t_conv:.2f} s, of which {t_call:.2f} s "
                       f"per-call setup; one-time setup {t_init:.2f} s); per-particle times extrapolated to "
                       f"all {n_total} particles: estimated step {step:.1f} s")}


SURROGATE_EVAL = {
    # 8 APRs of uneven sizes from 256^3 to 768^3 (~34M particles; generated in
    # worker processes, ~20 s on 16 cores), and a smaller batch for quick runs
    "full": (256, 320, 384, 448, 512, 576, 640, 768),
    "small": (160, 192, 224, 256, 288, 320, 352, 384),
}
SURROGATE_WEIGHTS = os.path.join(ROOT, "paper_2112_03592_amd", "weights", "rl10_surrogate.npz")


MFMA_BF16_PEAK_TFLOPS = 2500.0   # dense BF16 matrix peak


def device_values(inp):
    """Particle values of a workload as a device tensor."""
    import torch
    v = inp.values
    return v if isinstance(v, torch.Tensor) else torch.from_numpy(v).cuda()


def build_workload(name: str, generator: str):
    """The named sphere-field configuration: built on the device
    (``apr_sphere_field``; noise: the Gaussian limit of the Poisson law of each
    cell sum) or by the slab-wise CPU generator (Poisson draws per cell)."""
    from aprgen.apr_input import CONFIGS, _sphere_params, load_sphere_apr
    cfg = CONFIGS[name]
    if generator == "cpu":
        return load_sphere_apr(name, progress=lambda d, n: log(f"  slab {d}/{n}") if d % 8 == 0 else None)
    import torch
    from paper_2112_03592_amd import apr as G
    cen, rad = _sphere_params(cfg)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    f = G.sphere_field(cfg.dims, cfg.l_min, cen, rad, background=cfg.background, foreground=cfg.foreground,
                       edge_sigma=cfg.edge_sigma, noise=cfg.noise, seed=cfg.seed)
    f.build_s = time.perf_counter() - t0
    return f


def layers_leg(inp, reps: int = 10):
    """The gather path on the same APR: the network layer shapes (1->16,
    16->16 on MFMA with BF16 activations, 16->16 FP32, 16->1), the 16-channel
    tree fill, and both gradients of a 16->16 layer (FP32; the weight
    gradient also with BF16 activations)."""
    import numpy as np
    import torch
    from aprgen.apr_input import gaussian_stencil
    from paper_2112_03592_amd import apr as G
    n_p = inp.n_particles
    acc = G.AprAccess.from_input(inp, gather=(3,))
    nl = acc.n_levels
    g = torch.Generator(device="cuda").manual_seed(0)

    def rnd(*shape, dtype=torch.float32):
        return torch.randn(*shape, generator=g, device="cuda").to(dtype)

    def tm(f):
        f()
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(reps):
            f()
        b.record()
        torch.cuda.synchronize()
        return a.elapsed_time(b) / reps

    w11 = rnd(nl, 16, 1, 3, 3, 3) * 0.2
    w1616 = rnd(nl, 16, 16, 3, 3, 3) * 0.05
    w161 = rnd(nl, 1, 16, 3, 3, 3) * 0.05
    bias16, bias1 = rnd(16), rnd(1)
    x1 = device_values(inp).view(-1, 1)
    t1 = G.fill_tree(acc, x1)
    h16 = rnd(n_p, 16)
    h16b = h16.to(torch.bfloat16)
    t16 = G.fill_tree(acc, h16)
    t16b = G.fill_tree(acc, h16b)
    dy = rnd(n_p, 16)
    rec = {"n_particles": n_p, "ms": {}}
    ms = rec["ms"]
    ms["fill16_bf16"] = tm(lambda: G.fill_tree(acc, h16b, t16b))
    ms["fill16_f32"] = tm(lambda: G.fill_tree(acc, h16, t16))
    ms["fwd_1to16_f32_to_bf16"] = tm(lambda: G.conv(acc, x1, t1, w11, 3, bias=bias16, relu=True,
                                                     out_dtype=torch.bfloat16))
    ms["fwd_16to16_bf16_mfma"] = tm(lambda: G.conv(acc, h16b, t16b, w1616, 3, bias=bias16, relu=True))
    ms["fwd_16to16_f32"] = tm(lambda: G.conv(acc, h16, t16, w1616, 3, bias=bias16, relu=True))
    ms["fwd_16to1_bf16_to_f32"] = tm(lambda: G.conv(acc, h16b, t16b, w161, 3, bias=bias1,
                                                     out_dtype=torch.float32))
    f8 = torch.float8_e4m3fn
    h16f8 = h16.to(f8)
    t16f8 = G.fill_tree(acc, h16f8)
    ms["fill16_fp8"] = tm(lambda: G.fill_tree(acc, h16f8, t16f8))
    ms["fwd_1to16_f32_to_fp8"] = tm(lambda: G.conv(acc, x1, t1, w11, 3, bias=bias16, relu=True, out_dtype=f8))
    ms["fwd_16to16_fp8_mfma"] = tm(lambda: G.conv(acc, h16f8, t16f8, w1616, 3, bias=bias16, relu=True))
    ms["fwd_16to1_fp8_to_f32"] = tm(lambda: G.conv(acc, h16f8, t16f8, w161, 3, bias=bias1,
                                                    out_dtype=torch.float32))
    del h16f8, t16f8
    ms["bwd_data_16to16_f32"] = tm(lambda: G.conv_bwd_data(acc, dy, w1616, 3))
    ms["bwd_weight_16to16_f32"] = tm(lambda: G.conv_bwd_weight(acc, h16, t16, dy, 3, nl, 16, 16))
    ms["bwd_weight_16to16_bf16x"] = tm(lambda: G.conv_bwd_weight(acc, h16b, t16b, dy, 3, nl, 16, 16))
    # MFMA layer against the BF16 matrix peak and the HBM roofline: gathered
    # rows (BF16, 16 channels) of particles and tree, the gather map, outputs
    t = ms["fwd_16to16_bf16_mfma"] * 1e-3
    flops = 2.0 * 27 * 16 * 16 * n_p
    bytes_alg = n_p * 32 + acc.n_tree * 32 + n_p * 27 * 4 + n_p * 32
    rec["mfma_16to16"] = {"tflops": flops / t / 1e12, "frac_mfma_bf16": flops / t / 1e12 / MFMA_BF16_PEAK_TFLOPS,
                          "GBps": bytes_alg / t / 1e9, "frac_hbm": bytes_alg / t / 1e9 / HBM_PEAK_GBPS,
                          "algorithmic_bytes": bytes_alg}
    acc.close()
    return rec


def bf16_leg(acc, inp, reps: int = 10):
    """BF16 storage of the single-channel 3^3 / 5^3 convolution (FP32
    accumulation) against FP32 storage: times and relative L2 difference."""
    import torch
    from aprgen.apr_input import gaussian_stencil
    from paper_2112_03592_amd import apr as G

    def tm(f):
        f()
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(reps):
            f()
        b.record()
        torch.cuda.synchronize()
        return a.elapsed_time(b) / reps

    xs = device_values(inp)
    xb = xs.to(torch.bfloat16)
    ts, tb = G.fill_tree(acc, xs), G.fill_tree(acc, xb)
    prec = {"fill_bf16_ms": tm(lambda: G.fill_tree(acc, xb, tb)), "fill_f32_ms": tm(lambda: G.fill_tree(acc, xs, ts))}
    for k in (3, 5):
        w = torch.from_numpy(G.stencil_levels(gaussian_stencil(k, 1.0), "same", k, inp.l_min, inp.l_max)).cuda()
        yf = G.conv(acc, xs, ts, w, k)
        yb = G.conv(acc, xb, tb, w, k, out_dtype=torch.float32)
        d = (yb.double() - yf.double()).norm() / yf.double().norm()
        prec[f"conv{k}"] = {"bf16_ms": tm(lambda: G.conv(acc, xb, tb, w, k, out_dtype=torch.float32, y=yb)),
                            "f32_ms": tm(lambda: G.conv(acc, xs, ts, w, k, y=yf)),
                            "bf16_vs_f32_rel_l2": float(d)}
        del yf, yb
    return prec


def gradmag_leg(acc, inp, x, tree, reps: int = 20):
    """Resolution-adaptive gradient magnitude: three level-scaled 3^3 Sobel
    stencils on one patch, |grad| written per particle (after a tree fill)."""
    import numpy as np
    import torch
    from aprgen.apr_input import sobel_stencils
    from paper_2112_03592_amd import apr as G
    w3 = torch.from_numpy(G.stencil_levels(sobel_stencils(), "adaptive", 3, inp.l_min, inp.l_max)).cuda()
    y = torch.empty(inp.n_particles, dtype=torch.float32, device="cuda")
    G.fill_tree(acc, x, tree)
    G.gradient_magnitude(acc, x, tree, w3, y)
    torch.cuda.synchronize()
    e = [torch.cuda.Event(enable_timing=True) for _ in range(3)]
    e[0].record()
    for _ in range(reps):
        G.fill_tree(acc, x, tree)
    e[1].record()
    for _ in range(reps):
        G.gradient_magnitude(acc, x, tree, w3, y)
    e[2].record()
    torch.cuda.synchronize()
    fill_ms, g_ms = e[0].elapsed_time(e[1]) / reps, e[1].elapsed_time(e[2]) / reps
    n_p = inp.n_particles
    return {"ms": g_ms, "fill_ms": fill_ms, "Gparticles_s": n_p / ((fill_ms + g_ms) * 1e-3) / 1e9,
            "pixel_equiv_GBps": float(np.prod(inp.dims)) * 4 / ((fill_ms + g_ms) * 1e-3) / 1e9}


def surrogate_inputs(which: str):
    """The batch's APRs, generated in worker processes (before this process
    touches the GPU)."""
    from aprgen.apr_input import deconv_set
    t0 = time.perf_counter()
    inputs = deconv_set(SURROGATE_EVAL[which], 7000, workers=8,
                        progress=lambda e, n: log(f"  generated {e}^3 deconvolution APR, {n} particles"))
    log(f"surrogate batch {SURROGATE_EVAL[which]} generated in {time.perf_counter() - t0:.1f} s")
    return inputs


def surrogate_leg(which: str, inputs, reps: int = 3, weights: str = SURROGATE_WEIGHTS):
    """Plain 10-iteration APR Richardson-Lucy against the surrogate (start
    iterations + network + monitor, plus the plain iteration when the monitor
    rejects) on a batch of deconvolution APRs; relative L2 error of the
    returned values against the plain result (FP32 on the device)."""
    import numpy as np
    import torch
    from paper_2112_03592_amd import apr as G
    from paper_2112_03592_amd import surrogate as N
    from aprgen.apr_input import deconv_psf, gaussian_stencil
    edges = SURROGATE_EVAL[which]
    # the FP64 oracle's RL10 of the 256^3 batch APR, stored by
    # tests/golden/make_rl10_deconv256.py (a file, not oracle code)
    from aprgen.apr_input import input_digest
    gold_path = os.path.join(ROOT, "tests", "golden", "rl10_deconv256.npz")
    gold = np.load(gold_path) if os.path.exists(gold_path) else None
    sur = N.load_surrogate(weights)
    sur8 = N.load_surrogate(weights, act_dtype=torch.float8_e4m3fn)
    ws = G.Workspace(16)
    rec = {"edges": list(edges), "n_particles": [], "plain_ms": [], "surrogate_ms": [], "error": [],
           "monitor": [], "fallback": [], "fp8": {"surrogate_ms": [], "error": [], "fallback": []}}
    for inp in inputs:
        acc = G.AprAccess.from_input(inp, gather=(3,))
        u = torch.from_numpy(np.maximum(inp.values, 0).astype(np.float32)).cuda()
        t = sur.plain(acc, u)
        res = sur(acc, u)                      # warm-up of both paths
        torch.cuda.synchronize()
        a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(reps):
            sur.plain(acc, u)
        b.record()
        torch.cuda.synchronize()
        plain_ms = a.elapsed_time(b) / reps
        w0 = time.perf_counter()
        for _ in range(reps):
            res = sur(acc, u)                  # includes the monitor's host synchronisation
        torch.cuda.synchronize()
        sur_ms = (time.perf_counter() - w0) * 1e3 / reps
        rec["n_particles"].append(inp.n_particles)
        rec["plain_ms"].append(plain_ms)
        rec["surrogate_ms"].append(sur_ms)
        rec["error"].append(N.rel_error(res.values, t, ws))
        rec["monitor"].append(res.monitor)
        rec["fallback"].append(bool(res.fallback))
        if not rec.get("restricted_5cubed"):
            # the 5^3 convolution with the restricted PSF (every level coarser
            # than l_max runs the 3^3 neighbourhood) against the same PSF at
            # every level, on the first APR of the batch
            tr = G.fill_tree(acc, u)
            yy = torch.empty_like(u)
            lv = {}
            for mode in ("restrict", "same"):
                wm = torch.from_numpy(G.stencil_levels(deconv_psf(), mode, 5, acc.l_min, acc.l_max)).cuda()
                G.conv(acc, u, tr, wm, 5, y=yy)
                torch.cuda.synchronize()
                e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                e0.record()
                for _ in range(20):
                    G.conv(acc, u, tr, wm, 5, y=yy)
                e1.record()
                torch.cuda.synchronize()
                lv[mode + "_ms"] = e0.elapsed_time(e1) / 20
            lv["edge"] = inp.dims[0]
            lv["finest_level_share"] = acc.particles_per_level[acc.l_max] / inp.n_particles
            rec["restricted_5cubed"] = lv
            del tr, yy
            # 100 Richardson-Lucy iterations with a 13^3 Gaussian PSF (sigma 2,
            # restricted per level) on the same 256^3 APR: the size of the
            # paper's own deconvolution run (Sec. 6.2: 42 s on its CPU, on a
            # hollow-cylinder image of compression ratio 13.3)
            psf13 = gaussian_stencil(13, 2.0)
            G.richardson_lucy(acc, u, psf13, 2)
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            G.richardson_lucy(acc, u, psf13, 100)
            e1.record()
            torch.cuda.synchronize()
            rec["rl100_13cubed"] = {"edge": inp.dims[0], "n_particles": inp.n_particles,
                                    "ms": e0.elapsed_time(e1), "paper_cpu_s": 42.0}
        if gold is not None and inp.dims[0] == int(gold["edge"]) and str(gold["digest"]) == input_digest(inp):
            g = torch.from_numpy(gold["rl10"]).cuda()
            rec["vs_fp64_oracle"] = {"edge": int(gold["edge"]), "n_particles": inp.n_particles,
                                     "surrogate": N.rel_error(res.values, g, ws),
                                     "plain_rl10": N.rel_error(t, g, ws),
                                     "source": "tests/golden/rl10_deconv256.npz (FP64 oracle RL10, stored in FP32)"}
            del g
        # the same network with FP8 (E4M3) hidden activations
        res8 = sur8(acc, u)
        torch.cuda.synchronize()
        w0 = time.perf_counter()
        for _ in range(reps):
            res8 = sur8(acc, u)
        torch.cuda.synchronize()
        rec["fp8"]["surrogate_ms"].append((time.perf_counter() - w0) * 1e3 / reps)
        rec["fp8"]["error"].append(N.rel_error(res8.values, t, ws))
        rec["fp8"]["fallback"].append(bool(res8.fallback))
        log(f"  {inp.dims[0]}^3 N_p={inp.n_particles}: plain {plain_ms:.3f} ms, surrogate {sur_ms:.3f} ms, "
            f"error {rec['error'][-1]:.4f}, monitor {res.monitor:.4f}, fallback {res.fallback}; FP8 activations "
            f"{rec['fp8']['surrogate_ms'][-1]:.3f} ms, error {rec['fp8']['error'][-1]:.4f}, "
            f"fallback {res8.fallback}")
        sur.rl.forget(acc)
        sur8.rl.forget(acc)
        acc.close()
        del t, res, u
    rec["error_reference"] = "device RL10 (FP32); vs_fp64_oracle: the FP64 oracle at the 256^3 APR"
    rec["speedup"] = float(np.sum(rec["plain_ms"]) / np.sum(rec["surrogate_ms"]))
    rec["fp8"]["speedup"] = float(np.sum(rec["plain_ms"]) / np.sum(rec["fp8"]["surrogate_ms"]))
    rec["fp8"]["max_error"] = float(np.max(rec["fp8"]["error"]))
    rec["max_error"] = float(np.max(rec["error"]))
    rec["tau"] = sur.tau
    rec["start"] = {"iterations": sur.n_pre, "power": sur.power}
    rec["batch"] = which
    return rec


def timed_steps(acc, x, tree, w, y3, y5, steps: int, warmup: int):
    """Warm-up, then `steps` steps (fill, 3^3, 5^3) with HIP events around
    each kernel on the launch stream; returns (ms per step, wall ms per step,
    fill, conv3, conv5 mean launch times)."""
    import numpy as np
    import torch
    from paper_2112_03592_amd import apr as G

    def step(ev=None):
        if ev is not None:
            ev[0].record()
        G.fill_tree(acc, x, tree)
        if ev is not None:
            ev[1].record()
        G.conv(acc, x, tree, w[3], 3, y=y3)
        if ev is not None:
            ev[2].record()
        G.conv(acc, x, tree, w[5], 5, y=y5)
        if ev is not None:
            ev[3].record()

    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    evs = [[torch.cuda.Event(enable_timing=True) for _ in range(4)] for _ in range(steps)]
    start = torch.cuda.Event(enable_timing=True)
    stop = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    w0 = time.perf_counter()
    start.record()
    for i in range(steps):
        step(evs[i])
    stop.record()
    torch.cuda.synchronize()
    wall_ms = (time.perf_counter() - w0) * 1e3 / steps
    ms = start.elapsed_time(stop) / steps
    parts = [float(np.mean([e[j].elapsed_time(e[j + 1]) for e in evs])) for j in range(3)]
    return ms, wall_ms, parts, step


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="field2k_cr50")
    ap.add_argument("--generator", default="device", choices=["device", "cpu"],
                    help="build the sphere field on the device, or with the slab-wise CPU generator")
    ap.add_argument("--cpu-sample", type=int, default=1 << 15)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--surrogate-eval", default="full", choices=["full", "small", "none"],
                    help="batch of the surrogate-vs-plain Richardson-Lucy comparison")
    ap.add_argument("--no-layers", action="store_true", help="skip the gather-path layer timings")
    ap.add_argument("--layers-workload", default="field1k_layer")
    ap.add_argument("--secondary", default="sphere512", help="second single-channel workload ('' = none)")
    ap.add_argument("--surrogate-weights", default=SURROGATE_WEIGHTS, help="trained surrogate (.npz)")
    ap.add_argument("--surrogate-only", action="store_true",
                    help="run only the surrogate comparison and print its record (profiling)")
    ap.add_argument("--layers-only", action="store_true",
                    help="run only the gather-path layer timings and print their record (profiling)")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB five times (counter calibration)")
    args = ap.parse_args()
    if args.calibrate_copy:
        import torch
        n = args.calibrate_copy * (1 << 20) // 4
        a = torch.ones(n, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        for _ in range(5):
            b.copy_(a)
        torch.cuda.synchronize()
        log(f"copied {args.calibrate_copy} MiB five times")
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU only; --gpus {args.gpus} is not supported "
              f"(multi-GPU sharding of the APR is a design in DESIGN.md, not built)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from aprgen.apr_input import CONFIGS, gaussian_stencil
    from paper_2112_03592_amd import apr as G

    # CPU work that uses worker processes runs before the GPU is touched
    sur_inputs = None
    if args.surrogate_eval != "none" and os.path.exists(args.surrogate_weights) and not args.layers_only:
        sur_inputs = surrogate_inputs(args.surrogate_eval)
    if args.surrogate_only:
        print(json.dumps(surrogate_leg(args.surrogate_eval, sur_inputs, weights=args.surrogate_weights)
                         if sur_inputs is not None
                         else {"skipped": "no trained weights or --surrogate-eval none"}), flush=True)
        return
    if not torch.cuda.is_available():
        print("bench.py needs a HIP device", file=sys.stderr)
        sys.exit(1)
    if args.layers_only:
        print(json.dumps(layers_leg(build_workload(args.layers_workload, args.generator))), flush=True)
        return

    log(f"workload {args.workload}: building the APR ({args.generator} generator)")
    t0 = time.perf_counter()
    inp = build_workload(args.workload, args.generator)
    gen_s = time.perf_counter() - t0
    cfg = CONFIGS[args.workload]
    n_p = inp.n_particles
    n_px = int(np.prod(inp.dims))
    log(f"  {n_p} particles in {gen_s:.1f} s")
    x = device_values(inp)

    cpu = None
    if not args.no_cpu_baseline:
        edge = max(1 << (inp.l_max - inp.l_min), min(inp.dims) // 4)
        block = corner_block(inp, x, edge)
        log(f"cpu baseline: oracle on the {edge}^3 corner block ({block.n_particles} particles), one thread")
        cpu = cpu_baseline(block, n_p, args.cpu_sample)
        del block

    torch.cuda.synchronize()
    t0 = time.perf_counter()
    acc = G.AprAccess.from_input(inp)
    torch.cuda.synchronize()
    build_ms = (time.perf_counter() - t0) * 1e3
    log(f"access built: N_p={n_p} N_t={acc.n_tree} tiles={acc.n_tiles} work items={acc.n_work_items} ({build_ms:.1f} ms)")

    tree = torch.empty(acc.n_tree, dtype=torch.float32, device="cuda")
    y3 = torch.empty(n_p, dtype=torch.float32, device="cuda")
    y5 = torch.empty(n_p, dtype=torch.float32, device="cuda")
    w = {k: torch.from_numpy(G.stencil_levels(gaussian_stencil(k, 1.0), "same", k, inp.l_min,
                                              inp.l_max)).cuda() for k in (3, 5)}
    ms_per_step, wall_ms, (fill_ms, c3_ms, c5_ms), step = timed_steps(acc, x, tree, w, y3, y5, args.steps,
                                                                     args.warmup)
    log(f"step {ms_per_step:.3f} ms (wall {wall_ms:.3f} ms): fill {fill_ms:.3f} conv3 {c3_ms:.3f} conv5 {c5_ms:.3f}")

    # the paper's pipeline as device time: tile pre-pass + fill + convolution
    flags, ymin = G.tile_prepass(acc)
    n_rep = 10
    pev = [[torch.cuda.Event(enable_timing=True) for _ in range(2)] for _ in range(n_rep)]
    for i in range(n_rep):
        pev[i][0].record()
        G.tile_prepass(acc, flags, ymin)
        pev[i][1].record()
    torch.cuda.synchronize()
    prepass_ms = float(np.mean([e[0].elapsed_time(e[1]) for e in pev]))
    del flags, ymin

    rows, trows, n_t = acc.n_rows, acc.n_tree_rows, acc.n_tree
    kern = {"fill": (fill_ms, fill_bytes(n_p, n_t, rows, trows), 8 * n_t),
            "conv3": (c3_ms, conv_bytes(n_p, n_t, rows, trows), 2 * 27 * n_p),
            "conv5": (c5_ms, conv_bytes(n_p, n_t, rows, trows), 2 * 125 * n_p)}
    dom = max(kern, key=lambda k: kern[k][0])
    t_ms, bytes_alg, flops = kern[dom]
    t_hbm = bytes_alg / (HBM_PEAK_GBPS * 1e9)
    t_alu = flops / (FP32_VALU_PEAK_TFLOPS * 1e12)
    traffic = None
    tpath = os.path.join(ROOT, "profiles", "traffic.json")
    if os.path.exists(tpath):
        with open(tpath) as f:
            tj = json.load(f)
        ent = tj.get("workloads", {}).get(args.workload, {}).get("kernels", {}).get(dom)
        if ent and ent.get("source_sha") == source_hash(dom):
            traffic = ent["hbm_bytes_per_launch"]
    if t_hbm >= t_alu:
        achieved = bytes_alg / (t_ms * 1e-3) / 1e9
        roof = {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBPS, "unit": "GB/s",
                "frac": achieved / HBM_PEAK_GBPS, "traffic": traffic}
    else:
        achieved = flops / (t_ms * 1e-3) / 1e12
        roof = {"bound": "alu", "achieved": achieved, "peak": FP32_VALU_PEAK_TFLOPS, "unit": "TFLOP/s",
                "frac": achieved / FP32_VALU_PEAK_TFLOPS, "traffic": traffic}
    roof.update({"kernel": dom, "launch_ms": t_ms, "algorithmic_bytes": bytes_alg,
                 "algorithmic_flops": flops, "hbm_time_at_peak_ms": t_hbm * 1e3,
                 "alu_time_at_peak_ms": t_alu * 1e3})

    def rate(ms):
        return {"ms": ms, "Gparticles_s": n_p / (ms * 1e-3) / 1e9,
                "pixel_equiv_GBps": n_px * 4 / (ms * 1e-3) / 1e9}

    # cold caches: a 1 GiB write between steps evicts L2 and the MALL
    log("cold-cache steps")
    flush = torch.empty(1 << 28, dtype=torch.float32, device="cuda")
    n_cold = min(args.steps, 20)
    cev = [[torch.cuda.Event(enable_timing=True) for _ in range(4)] for _ in range(n_cold)]
    for i in range(n_cold):
        flush.fill_(float(i))
        step(cev[i])
    torch.cuda.synchronize()
    del flush
    cold = [float(np.mean([e[j].elapsed_time(e[j + 1]) for e in cev])) for j in range(3)]
    # the device's own copy bandwidth (read + write of 1 GiB), for scale
    src = torch.empty(1 << 28, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    c0, c1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    c0.record()
    for _ in range(5):
        dst.copy_(src)
    c1.record()
    torch.cuda.synchronize()
    copy_gbps = 2 * src.numel() * 4 * 5 / (c0.elapsed_time(c1) * 1e-3) / 1e9
    del src, dst
    cold_step = sum(cold)
    alg_frac = {name: kern[name][1] / (kern[name][0] * 1e-3) / 1e9 / HBM_PEAK_GBPS for name in kern}

    value = n_p / (ms_per_step * 1e-3) / 1e9
    out = {
        "metric": METRIC, "value": value, "unit": "Gparticles/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": ms_per_step, "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f32", "data": "synthetic",
        "config": {"workload": (f"{args.workload}: {inp.dims[0]}x{inp.dims[1]}x{inp.dims[2]} sphere field, "
                                f"{cfg.n_spheres} spheres r {cfg.r_min:g}-{cfg.r_max:g}, levels "
                                f"{inp.l_min}-{inp.l_max}, built on the "
                                f"{'device' if args.generator == 'device' else 'host'}; step = tree fill + "
                                f"3^3 + 5^3 Gaussian (sigma 1) APR convolution, same stencil at every level"),
                   "n_particles": n_p, "n_tree": n_t, "pixels_per_particle": n_px / n_p,
                   "tiles": acc.n_tiles, "work_items": acc.n_work_items, "generator": args.generator},
        "pixel_equiv_GBps": n_px * 4 / (ms_per_step * 1e-3) / 1e9,
        "stages_ms": {"fill": fill_ms, "conv3": c3_ms, "conv5": c5_ms, "access_build_once": build_ms,
                      "apr_construction_once_s": gen_s, "tile_prepass": prepass_ms},
        "paper_comparable_ms": {"note": "device time: tile pre-pass + tree fill + convolution (the paper's "
                                        "GPU timings include every step)",
                                "conv3": prepass_ms + fill_ms + c3_ms, "conv5": prepass_ms + fill_ms + c5_ms,
                                "conv3_rate": rate(prepass_ms + fill_ms + c3_ms),
                                "conv5_rate": rate(prepass_ms + fill_ms + c5_ms)},
        "pipeline_3x3x3": rate(fill_ms + c3_ms),
        "pipeline_5x5x5": rate(fill_ms + c5_ms),
        "roofline": roof,
        "hbm_algorithmic_frac": alg_frac,
        "hbm_fractions_dominant": {"kernel": dom, "algorithmic": bytes_alg / (t_ms * 1e-3) / 1e9 / HBM_PEAK_GBPS,
                                   "measured_traffic": (None if traffic is None
                                                        else traffic / (t_ms * 1e-3) / 1e9 / HBM_PEAK_GBPS),
                                   "copy_kernel": copy_gbps / HBM_PEAK_GBPS, "copy_GBps": copy_gbps},
        "cold_cache": {"ms_per_step": cold_step, "stages_ms": dict(zip(("fill", "conv3", "conv5"), cold)),
                       "Gparticles_s": n_p / (cold_step * 1e-3) / 1e9,
                       "pipeline_3x3x3": rate(cold[0] + cold[1]), "pipeline_5x5x5": rate(cold[0] + cold[2])},
        "source_sha": {k: source_hash(k) for k in KERNEL_SOURCES},
    }
    log(f"cold caches: step {cold_step:.3f} ms: fill {cold[0]:.3f} conv3 {cold[1]:.3f} conv5 {cold[2]:.3f}")
    log("BF16 storage, single channel")
    out["bf16_single_channel"] = bf16_leg(acc, inp)
    log(f"  {json.dumps(out['bf16_single_channel'])}")
    out["gradient_magnitude"] = gradmag_leg(acc, inp, x, tree)
    log(f"  gradient magnitude: {json.dumps(out['gradient_magnitude'])}")
    acc.close()
    del tree, y3, y5, x
    if args.secondary:
        log(f"secondary workload {args.secondary}")
        inp2 = build_workload(args.secondary, args.generator)
        acc2 = G.AprAccess.from_input(inp2)
        x2 = device_values(inp2)
        t2 = torch.empty(acc2.n_tree, dtype=torch.float32, device="cuda")
        a3, a5 = torch.empty_like(x2), torch.empty_like(x2)
        w2 = {k: torch.from_numpy(G.stencil_levels(gaussian_stencil(k, 1.0), "same", k, inp2.l_min,
                                                   inp2.l_max)).cuda() for k in (3, 5)}
        ms2, _, parts2, _ = timed_steps(acc2, x2, t2, w2, a3, a5, args.steps, args.warmup)
        n2 = inp2.n_particles
        out["secondary"] = {"workload": args.secondary, "n_particles": n2, "ms_per_step": ms2,
                            "Gparticles_s": n2 / (ms2 * 1e-3) / 1e9,
                            "stages_ms": dict(zip(("fill", "conv3", "conv5"), parts2)),
                            "hbm_algorithmic_frac": {
                                "conv3": conv_bytes(n2, acc2.n_tree, acc2.n_rows, acc2.n_tree_rows)
                                / (parts2[1] * 1e-3) / 1e9 / HBM_PEAK_GBPS,
                                "conv5": conv_bytes(n2, acc2.n_tree, acc2.n_rows, acc2.n_tree_rows)
                                / (parts2[2] * 1e-3) / 1e9 / HBM_PEAK_GBPS}}
        log(f"  {json.dumps(out['secondary'])}")
        acc2.close()
        del inp2, x2, t2, a3, a5
    if not args.no_layers:
        log(f"layers leg on {args.layers_workload} (gather path, 16 channels; BF16 storage)")
        linp = build_workload(args.layers_workload, args.generator)
        out["layers"] = layers_leg(linp)
        out["layers"]["workload"] = args.layers_workload
        del linp
    if sur_inputs is not None:
        log(f"surrogate leg ({args.surrogate_eval} batch)")
        out["surrogate"] = surrogate_leg(args.surrogate_eval, sur_inputs, weights=args.surrogate_weights)
    elif args.surrogate_eval != "none":
        out["surrogate"] = {"skipped": "no trained weights (python -m paper_2112_03592_amd.train_surrogate)"}
    out["cpu_baseline"] = cpu
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
