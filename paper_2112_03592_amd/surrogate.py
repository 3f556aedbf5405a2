"""APR-native network that stands in for n iterations of Richardson-Lucy
deconvolution, with an error monitor and the plain iteration as fallback.

Section 7 proposes CNNs built from APR convolution layers with filters
learned per resolution level.  Here such a network corrects a cheap start:

    b = RL_m(u; power p)        m < n over-relaxed iterations (i <- i * c^p)
    h_0 = normalise(b);  h_{i+1} = ReLU(conv_i(h_i) + beta_i);  net = conv_L(h_L) + beta_L
    s = b + sd * net            (additive residual)
    s = b * exp(sd * net)       (multiplicative residual, log-domain input)

and is trained so that s matches RL_n(u) (Section 6.2) computed by the plain
iteration.  Every convolution fills the tree of its own input first.
Weights are kept as weight sets indexed by the distance to the finest level
(``apr_level_weights``) so one network serves APRs of any depth.  Training
is written out by hand: forward with stored activations, the backward
kernels layer by layer, one Adam step per APR.  All arithmetic runs in the
HIP library; this module orders the calls and owns the device buffers.
"""
from __future__ import annotations

import dataclasses
from typing import Dict, List, Optional, Sequence, Tuple

import numpy as np
import torch

from . import apr as G

ADDITIVE, MULTIPLICATIVE = "add", "mul"


# ---------------------------------------------------------------------------
# autograd wrapper of one APR convolution layer
# ---------------------------------------------------------------------------

class AprConvFunction(torch.autograd.Function):
    """y = act(conv(x, W) + b), the tree of x filled inside; backward by
    ``apr_relu_bias_grad``, ``apr_conv_bwd_data`` and ``apr_conv_bwd_weight``.
    x [N_p, c_in] FP32, w [n_wlevels, c_out, c_in, k, k, k], b [c_out]."""

    @staticmethod
    def forward(ctx, x, w, b, acc, k, relu):
        x = x.contiguous()
        tree = G.fill_tree(acc, x)
        y = G.conv(acc, x, tree, w.contiguous(), k, bias=b.contiguous(), relu=relu)
        ctx.acc, ctx.k, ctx.relu = acc, k, bool(relu)
        ctx.save_for_backward(x, tree, w, y)
        return y

    @staticmethod
    def backward(ctx, dy):
        x, tree, w, y = ctx.saved_tensors
        acc, k = ctx.acc, ctx.k
        nw, cout, cin = w.shape[0], w.shape[1], w.shape[2]
        ws = G.Workspace(max(cout, 1), device=dy.device)
        dpre, db = G.relu_bias_grad(y, dy.contiguous(), ctx.relu, ws)
        dx = G.conv_bwd_data(acc, dpre, w.contiguous(), k) if ctx.needs_input_grad[0] else None
        dw = G.conv_bwd_weight(acc, x, tree, dpre, k, nw, cin, cout) if ctx.needs_input_grad[1] else None
        return dx, dw, db, None, None, None


def apr_conv_layer(acc: G.AprAccess, x: torch.Tensor, w: torch.Tensor, b: torch.Tensor, k: int,
                   relu: bool = False) -> torch.Tensor:
    return AprConvFunction.apply(x, w, b, acc, k, relu)


# ---------------------------------------------------------------------------
# Richardson-Lucy with the per-level PSF cached per access structure
# ---------------------------------------------------------------------------

class RichardsonLucy:
    """``apr_richardson_lucy`` with the restricted PSF stencils kept per level
    range and one workspace grown to the largest APR seen."""

    def __init__(self, psf: np.ndarray, eps_rel: float = 1e-12):
        self.psf = np.asarray(psf, np.float64)
        self.k = self.psf.shape[-1]
        self.eps_rel = eps_rel
        self._stencils: Dict[Tuple[int, int], Tuple[torch.Tensor, torch.Tensor]] = {}
        self._ws: Optional[torch.Tensor] = None

    def _prep(self, acc: G.AprAccess, device):
        key = (acc.l_min, acc.l_max)
        if key not in self._stencils:
            w = torch.from_numpy(G.stencil_levels(self.psf, "restrict", self.k, acc.l_min, acc.l_max)).to(device)
            wf = torch.from_numpy(G.stencil_levels(self.psf, "restrict", self.k, acc.l_min, acc.l_max,
                                                   flip=True)).to(device)
            self._stencils[key] = (w, wf)
        nbytes = int(acc._lib.apr_richardson_lucy_workspace(acc.handle))
        if self._ws is None or self._ws.numel() < nbytes or self._ws.device != torch.device(device):
            self._ws = torch.empty(nbytes, dtype=torch.uint8, device=device)
        w, wf = self._stencils[key]
        return w, wf, self._ws

    def forget(self, acc: Optional[G.AprAccess] = None) -> None:
        """Release the workspace (it is re-allocated on the next call)."""
        self._ws = None

    def __call__(self, acc: G.AprAccess, u: torch.Tensor, n_iter: int, init: Optional[torch.Tensor] = None,
                 out: Optional[torch.Tensor] = None, power: float = 1.0) -> torch.Tensor:
        w, wf, ws = self._prep(acc, u.device)
        if out is None:
            out = torch.empty_like(u)
        G.L.check(acc._lib.apr_richardson_lucy(acc.handle, self.k, w.shape[0], G._ptr(w), G._ptr(wf), G._ptr(u),
                                               G._ptr(init), G._ptr(out), int(n_iter), float(self.eps_rel),
                                               float(power), G._ptr(ws), G._stream()))
        return out


# ---------------------------------------------------------------------------
# the network
# ---------------------------------------------------------------------------

@dataclasses.dataclass
class NetConfig:
    channels: int = 16
    layers: int = 4
    k: int = 3
    n_sets: int = 4
    mode: str = MULTIPLICATIVE
    seed: int = 0
    last_scale: float = 0.01   # the last layer starts near zero: s starts near u

    def chans(self) -> List[int]:
        return [1] + [self.channels] * (self.layers - 1) + [1]


class SurrogateNet:
    """Weights W_i [n_sets, c_out, c_in, k, k, k] and biases b_i [c_out] on the device."""

    def __init__(self, cfg: NetConfig = NetConfig(), device="cuda"):
        self.cfg = cfg
        self.device = torch.device(device)
        rng = np.random.default_rng(cfg.seed)
        ch = cfg.chans()
        self.W: List[torch.Tensor] = []
        self.b: List[torch.Tensor] = []
        for i in range(cfg.layers):
            ci, co = ch[i], ch[i + 1]
            w = rng.normal(size=(cfg.n_sets, co, ci, cfg.k, cfg.k, cfg.k)) * np.sqrt(2.0 / (ci * cfg.k ** 3))
            if i == cfg.layers - 1:
                w *= cfg.last_scale
            self.W.append(torch.from_numpy(w.astype(np.float32)).to(self.device))
            self.b.append(torch.zeros(co, dtype=torch.float32, device=self.device))
        self._m = [torch.zeros_like(t) for t in self.W + self.b]
        self._v = [torch.zeros_like(t) for t in self.W + self.b]
        self.step = 0
        self.ws = G.Workspace(max(cfg.channels, 1), device=self.device)
        self._levels: Dict[Tuple[int, int], Tuple[int, List[torch.Tensor]]] = {}
        self._version = 0

    # -- parameters ---------------------------------------------------------
    @property
    def log(self) -> bool:
        return self.cfg.mode == MULTIPLICATIVE

    def params(self) -> List[torch.Tensor]:
        return self.W + self.b

    def level_params(self, acc: G.AprAccess) -> List[torch.Tensor]:
        """Per-level weights of every layer for this APR's level range."""
        key = (acc.l_min, acc.l_max)
        hit = self._levels.get(key)
        if hit is None or hit[0] != self._version:
            hit = (self._version, [G.level_weights(w, acc.l_min, acc.l_max) for w in self.W])
            self._levels[key] = hit
        return hit[1]

    def state_dict(self) -> Dict[str, np.ndarray]:
        d = {f"W{i}": w.cpu().numpy() for i, w in enumerate(self.W)}
        d.update({f"b{i}": b.cpu().numpy() for i, b in enumerate(self.b)})
        d["config"] = np.array(repr(dataclasses.asdict(self.cfg)))
        return d

    def save(self, path: str) -> None:
        np.savez(path, **self.state_dict())

    @classmethod
    def load(cls, path: str, device="cuda") -> "SurrogateNet":
        import ast
        with np.load(path, allow_pickle=False) as f:
            cfg = NetConfig(**ast.literal_eval(str(f["config"])))
            net = cls(cfg, device=device)
            for i in range(cfg.layers):
                net.W[i].copy_(torch.from_numpy(f[f"W{i}"]))
                net.b[i].copy_(torch.from_numpy(f[f"b{i}"]))
        net._version += 1
        return net

    # -- forward / backward -------------------------------------------------
    def forward(self, acc: G.AprAccess, u: torch.Tensor, train: bool = False,
                act_dtype: torch.dtype = torch.float32):
        """s for particle values u [N_p] (FP32).  With ``train`` the layer
        inputs, their trees and the layer outputs are kept for ``backward``
        (FP32 only); otherwise hidden activations are stored as act_dtype."""
        cfg = self.cfg
        if train and act_dtype != torch.float32:
            raise ValueError("training runs in FP32")
        Wl = self.level_params(acc)
        stats = G.moments(u, self.log, self.ws)
        h = G.pointwise(4 if self.log else 0, u, None, stats).view(-1, 1)
        ins, trees, outs = [], [], []
        for i in range(cfg.layers):
            last = i == cfg.layers - 1
            tree = G.fill_tree(acc, h)
            y = G.conv(acc, h, tree, Wl[i], cfg.k, bias=self.b[i], relu=not last,
                       out_dtype=torch.float32 if last else act_dtype)
            if train:
                ins.append(h)
                trees.append(tree)
                outs.append(y)
            h = y
        net = h.view(-1)
        s = G.pointwise(6 if self.log else 2, net, u, stats)
        cache = (stats, ins, trees, outs, s) if train else None
        return s, cache

    def backward(self, acc: G.AprAccess, cache, ds: torch.Tensor) -> List[torch.Tensor]:
        """Gradients of the weight sets and biases given dL/ds."""
        cfg = self.cfg
        stats, ins, trees, outs, s = cache
        Wl = self.level_params(acc)
        g = G.pointwise(7 if self.log else 3, ds, s, stats).view(-1, 1)
        gW: List[Optional[torch.Tensor]] = [None] * cfg.layers
        gb: List[Optional[torch.Tensor]] = [None] * cfg.layers
        ch = cfg.chans()
        nl = acc.l_max - acc.l_min + 1
        for i in range(cfg.layers - 1, -1, -1):
            relu = i < cfg.layers - 1
            g, gb[i] = G.relu_bias_grad(outs[i], g, relu, self.ws)
            dWl = G.conv_bwd_weight(acc, ins[i], trees[i], g, cfg.k, nl, ch[i], ch[i + 1])
            gW[i] = G.fold_level_weights(dWl, cfg.n_sets, acc.l_min, acc.l_max)
            if i > 0:
                g = G.conv_bwd_data(acc, g, Wl[i], cfg.k)
        return gW + gb

    def loss_and_grad(self, acc: G.AprAccess, u: torch.Tensor, t: torch.Tensor):
        """(device FP64 [loss, |t|^2], gradients) with loss = |s - t|^2 / |t|^2."""
        s, cache = self.forward(acc, u, train=True)
        out, ds = G.rel_l2(s, t, self.ws, grad=True)
        return out, self.backward(acc, cache, ds)

    def adam_step(self, grads: Sequence[torch.Tensor], lr: float, beta1: float = 0.9, beta2: float = 0.999,
                  eps: float = 1e-8) -> None:
        self.step += 1
        for p, g, m, v in zip(self.params(), grads, self._m, self._v):
            G.adam(p, g, m, v, self.step, lr, beta1, beta2, eps)
        self._version += 1

    def train_step(self, acc: G.AprAccess, u: torch.Tensor, t: torch.Tensor, lr: float) -> torch.Tensor:
        out, grads = self.loss_and_grad(acc, u, t)
        self.adam_step(grads, lr)
        return out


# ---------------------------------------------------------------------------
# inference with the error monitor and the fallback
# ---------------------------------------------------------------------------

@dataclasses.dataclass
class SurrogateResult:
    values: torch.Tensor
    monitor: float            # |RL_1(s) - s| / |s|, RL step observed from u and started at s
    fallback: bool            # True when the plain iteration produced ``values``


class RLSurrogate:
    """Estimate of ``n_iter`` Richardson-Lucy iterations: ``n_pre``
    over-relaxed iterations with exponent ``power``, then the network.  The
    estimate is accepted when the monitor m = |RL_1(s) - s| / |s| is at most
    ``tau``; otherwise the plain iteration runs (tau = 0 always falls back)."""

    def __init__(self, net: SurrogateNet, psf: np.ndarray, n_iter: int = 10, n_pre: int = 4,
                 power: float = 2.0, tau: float = float("inf"), act_dtype: torch.dtype = torch.bfloat16):
        self.net = net
        self.rl = RichardsonLucy(psf)
        self.n_iter = n_iter
        self.n_pre = n_pre
        self.power = power
        self.tau = tau
        self.act_dtype = act_dtype
        self._out = torch.empty(2, dtype=torch.float64, device=net.device)

    def base(self, acc: G.AprAccess, u: torch.Tensor) -> torch.Tensor:
        return self.rl(acc, u, self.n_pre, power=self.power)

    def estimate(self, acc: G.AprAccess, u: torch.Tensor) -> Tuple[torch.Tensor, torch.Tensor]:
        """(s, device FP64 [m^2, |s|^2]) without a host synchronisation."""
        s, _ = self.net.forward(acc, self.base(acc, u), act_dtype=self.act_dtype)
        r1 = self.rl(acc, u, 1, init=s)
        out, _ = G.rel_l2(r1, s, self.net.ws, out=self._out)
        return s, out

    def plain(self, acc: G.AprAccess, u: torch.Tensor) -> torch.Tensor:
        return self.rl(acc, u, self.n_iter)

    def __call__(self, acc: G.AprAccess, u: torch.Tensor) -> SurrogateResult:
        s, out = self.estimate(acc, u)
        m = float(np.sqrt(max(float(out[0].item()), 0.0)))   # the one host synchronisation
        if m <= self.tau:
            return SurrogateResult(s, m, False)
        return SurrogateResult(self.plain(acc, u), m, True)


def rel_error(a: torch.Tensor, b: torch.Tensor, ws: G.Workspace) -> float:
    """|a - b| / |b| from the FP64 device reduction."""
    out, _ = G.rel_l2(a, b, ws)
    return float(np.sqrt(max(float(out[0].item()), 0.0)))


def calibrate_power(rl: RichardsonLucy, cases, n_pre: int, ws: G.Workspace,
                    grid: Sequence[float] = tuple(np.round(np.arange(1.0, 3.01, 0.1), 2))) -> float:
    """Exponent p on ``grid`` minimising the mean relative error of
    RL_{n_pre}(u; p) against the target over cases (acc, u, t)."""
    best, best_p = None, 1.0
    for p in grid:
        e = float(np.mean([rel_error(rl(acc, u, n_pre, power=float(p)), t, ws) for acc, u, t in cases]))
        if best is None or e < best:
            best, best_p = e, float(p)
    return best_p


def train(net: SurrogateNet, cases, steps: int, lr: float = 1e-3, lr_min: float = 1e-5,
          log_every: int = 0, progress=None) -> List[float]:
    """Adam over the training cases (acc, base, target) in turn, cosine
    learning-rate decay from lr to lr_min.  Returns the per-step losses
    |s - t| / |t| (read back every ``log_every`` steps; empty when 0);
    ``progress(step, loss)`` is called at each read-back."""
    losses: List[float] = []
    for it in range(steps):
        acc, b, t = cases[it % len(cases)]
        rate = lr_min + 0.5 * (lr - lr_min) * (1.0 + np.cos(np.pi * it / max(1, steps)))
        out = net.train_step(acc, b, t, rate)
        if log_every and (it % log_every == 0 or it == steps - 1):
            losses.append(float(np.sqrt(max(float(out[0].item()), 0.0))))
            if progress:
                progress(it, losses[-1])
    return losses


def calibrate_tau(monitors: Sequence[float], errors: Sequence[float], target: float) -> float:
    """Largest threshold tau such that every calibration case with monitor
    <= tau has error <= target; 0 (always fall back) when the case with the
    smallest monitor already misses the target."""
    m = np.asarray(monitors, np.float64)
    e = np.asarray(errors, np.float64)
    tau = 0.0
    for v in np.unique(m):                     # ascending distinct monitor values
        if np.any(e[m <= v] > target):
            break
        tau = float(v)
    return tau


def save_surrogate(path: str, sur: RLSurrogate, **extra) -> None:
    """Weights, network configuration, start iteration (n_pre, power), tau and
    any extra arrays (training record) in one .npz file."""
    d = sur.net.state_dict()
    d.update({"n_iter": np.array(sur.n_iter), "n_pre": np.array(sur.n_pre), "power": np.array(sur.power),
              "tau": np.array(sur.tau), "psf": np.asarray(sur.rl.psf)})
    d.update({k: np.asarray(v) for k, v in extra.items()})
    np.savez(path, **d)


def load_surrogate(path: str, device="cuda", act_dtype: torch.dtype = torch.bfloat16) -> RLSurrogate:
    net = SurrogateNet.load(path, device=device)
    with np.load(path, allow_pickle=False) as f:
        return RLSurrogate(net, f["psf"], int(f["n_iter"]), int(f["n_pre"]), float(f["power"]), float(f["tau"]),
                           act_dtype=act_dtype)
