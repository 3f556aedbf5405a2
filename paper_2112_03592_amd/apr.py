"""Python binding of the aprconv library: argument marshalling only.

Device buffers are torch tensors on the current HIP device; every call is
issued on ``torch.cuda.current_stream()``.  All arithmetic runs in the HIP
kernels of ``libaprconv.so``.
"""
from __future__ import annotations

import ctypes
from typing import Optional

import numpy as np
import torch

from . import _lib as L

_DT = {torch.float32: L.APR_F32, torch.bfloat16: L.APR_BF16, torch.float8_e4m3fn: L.APR_FP8}
_MODES = {"same": L.APR_STENCIL_SAME, "restrict": L.APR_STENCIL_RESTRICT,
          "adaptive": L.APR_STENCIL_ADAPTIVE}
_EPI = {None: L.APR_EPI_NONE, "ratio": L.APR_EPI_RATIO, "mul": L.APR_EPI_MUL, "mulpow": L.APR_EPI_MULPOW,
        "gradmag": L.APR_EPI_GRADMAG}


def _stream() -> int:
    return torch.cuda.current_stream().cuda_stream


def _ptr(t: Optional[torch.Tensor]) -> Optional[int]:
    if t is None:
        return None
    if not t.is_cuda or not t.is_contiguous():
        raise ValueError("expected a contiguous device tensor")
    return t.data_ptr()


class AprAccess:
    """Device access structure of one APR (``apr_access_build``)."""

    def __init__(self, dims, l_min: int, l_max: int, y_idx: np.ndarray, xz_end: np.ndarray,
                 validate: bool = True, gather=()):
        lib = L.load()
        self._lib = lib
        y = np.ascontiguousarray(y_idx, dtype=np.uint16)
        e = np.ascontiguousarray(xz_end, dtype=np.uint64)
        d = L.AccessDesc()
        d.dims[:] = [int(v) for v in dims]
        d.l_min, d.l_max = int(l_min), int(l_max)
        d.y_idx = y.ctypes.data if y.size else None
        d.n_particles = y.size
        d.xz_end = e.ctypes.data if e.size else None
        d.n_rows = e.size
        d.flags = (L.APR_VALIDATE_PARTITION | L.APR_VALIDATE_BALANCE) if validate else 0
        if 3 in gather:
            d.flags |= L.APR_BUILD_GATHER3
        if 5 in gather:
            d.flags |= L.APR_BUILD_GATHER5
        self.gather = tuple(gather)
        h = ctypes.c_void_p()
        L.check(lib.apr_access_build(ctypes.byref(d), _stream(), ctypes.byref(h)))
        self._h = h
        info = L.AccessInfo()
        L.check(lib.apr_access_get_info(h, ctypes.byref(info)))
        self.n_particles = int(info.n_particles)
        self.n_tree = int(info.n_tree)
        self.n_rows = int(info.n_rows)
        self.n_tree_rows = int(info.n_tree_rows)
        self.l_min, self.l_max = int(info.l_min), int(info.l_max)
        self.tree_l_min, self.tree_l_max = int(info.tree_l_min), int(info.tree_l_max)
        self.n_tiles = int(info.n_tiles)
        self.n_work_items = int(info.n_work_items)
        self.device_bytes = int(info.device_bytes)
        self.dims = tuple(int(v) for v in dims)
        self.level_dims = {l: tuple(info.dims[l]) for l in range(self.l_max + 1)}
        self.particles_per_level = {l: int(info.particles_per_level[l]) for l in range(self.l_min, self.l_max + 1)}
        self.tree_per_level = {l: int(info.tree_per_level[l])
                               for l in range(self.tree_l_min, self.tree_l_max + 1)}

    @classmethod
    def from_input(cls, inp, validate: bool = True, gather=()) -> "AprAccess":
        return cls(inp.dims, inp.l_min, inp.l_max, inp.y_idx, inp.xz_end, validate=validate, gather=gather)

    @property
    def handle(self) -> ctypes.c_void_p:
        if self._h is None:
            raise RuntimeError("AprAccess is closed")
        return self._h

    @property
    def n_levels(self) -> int:
        return self.l_max - self.l_min + 1

    def export_tree(self):
        ty = np.zeros(self.n_tree, np.uint16)
        te = np.zeros(self.n_tree_rows, np.uint64)
        L.check(self._lib.apr_access_export_tree(self.handle, ty.ctypes.data if ty.size else None,
                                                 te.ctypes.data if te.size else None))
        return ty, te

    def export_apr(self):
        """The particle LinearAccess held by the handle (``apr_access_export``)."""
        y = np.zeros(self.n_particles, np.uint16)
        e = np.zeros(self.n_rows, np.uint64)
        L.check(self._lib.apr_access_export(self.handle, L.APR_EXPORT_APR, y.ctypes.data if y.size else None,
                                            e.ctypes.data if e.size else None))
        return y, e

    def export_tiles(self):
        """Tile list [n_tiles, 4] (level, tile z, tile x, first y), finest
        level first, and the XCD range starts [9] of the launch list of work
        items."""
        t = np.zeros((self.n_tiles, 4), np.int32)
        off = np.zeros(9, np.int64)
        L.check(self._lib.apr_access_export(self.handle, L.APR_EXPORT_TILES, t.ctypes.data if t.size else None,
                                            off.ctypes.data))
        return t, off

    def close(self):
        if getattr(self, "_h", None) is not None:
            self._lib.apr_access_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()


def fill_tree(acc: AprAccess, x: torch.Tensor, tree: Optional[torch.Tensor] = None) -> torch.Tensor:
    """Tree values for particle values x [N_p] or [N_p, C] (``apr_fill_tree``)."""
    C = 1 if x.dim() == 1 else x.shape[1]
    if x.shape[0] != acc.n_particles:
        raise ValueError("x has the wrong number of particles")
    if tree is None:
        shape = (acc.n_tree,) if x.dim() == 1 else (acc.n_tree, C)
        tree = torch.empty(shape, dtype=x.dtype, device=x.device)
    L.check(acc._lib.apr_fill_tree(acc.handle, _ptr(x), _ptr(tree) if tree.numel() else None, C,
                                   _DT[x.dtype], _stream()))
    return tree


def tile_prepass(acc: AprAccess, flags: Optional[torch.Tensor] = None, ymin: Optional[torch.Tensor] = None):
    """The Section 5.2 pre-pass on its own (``apr_tile_prepass``): per
    candidate tile, occupied flag and smallest particle y."""
    lib = L.load()
    n = int(lib.apr_tile_prepass_size(acc.handle))
    if flags is None:
        flags = torch.empty(max(n, 1), dtype=torch.int32, device="cuda")
    if ymin is None:
        ymin = torch.empty(max(n, 1), dtype=torch.int32, device="cuda")
    L.check(lib.apr_tile_prepass(acc.handle, _ptr(flags), _ptr(ymin), _stream()))
    return flags[:n], ymin[:n]


def stencil_levels(w, mode: str, k: int, l_min: int, l_max: int, flip: bool = False) -> np.ndarray:
    """Per-level stencils [l_max-l_min+1, *lead, k, k, k] (FP32) computed by
    ``apr_stencil_levels`` from w [*lead, k, k, k]."""
    w = np.ascontiguousarray(w, dtype=np.float64)
    lead = w.shape[:-3]
    nf = int(np.prod(lead)) if lead else 1
    out = np.zeros((l_max - l_min + 1, nf, k * k * k), np.float32)
    L.check(L.load().apr_stencil_levels(_MODES[mode], k, nf, w.ctypes.data, l_min, l_max, int(flip),
                                        out.ctypes.data))
    return out.reshape((l_max - l_min + 1,) + lead + (k, k, k))


def _desc(k, c_in, c_out, nw, x_dtype, y_dtype, epilogue=None, eps=0.0, epi_arg=None, bias=None,
          relu=False, residual=None, power=1.0) -> L.ConvDesc:
    d = L.ConvDesc()
    d.k, d.c_in, d.c_out, d.n_wlevels = k, c_in, c_out, nw
    d.x_dtype, d.y_dtype = _DT[x_dtype], _DT[y_dtype]
    d.epilogue = _EPI[epilogue]
    d.eps = float(eps)
    d.epi_arg = _ptr(epi_arg) if epi_arg is not None else None
    d.bias = _ptr(bias) if bias is not None else None
    d.relu = int(bool(relu))
    d.residual = _ptr(residual) if residual is not None else None
    d.power = float(power)
    return d


def _wshape(acc: AprAccess, w: torch.Tensor, k: int):
    """(n_wlevels, c_out, c_in) of FP32 weights [nw, k,k,k] or [nw, c_out, c_in, k,k,k]."""
    if w.dtype != torch.float32:
        raise ValueError("weights are FP32")
    if w.dim() == 4:
        nw, cout, cin = w.shape[0], 1, 1
    elif w.dim() == 6:
        nw, cout, cin = w.shape[0], w.shape[1], w.shape[2]
    else:
        raise ValueError("w must be [nw, k, k, k] or [nw, c_out, c_in, k, k, k]")
    if nw not in (1, acc.n_levels) or w.shape[-1] != k or w.numel() != nw * cout * cin * k ** 3:
        raise ValueError("w must hold 1 or n_levels stencils of side k")
    return nw, cout, cin


def conv(acc: AprAccess, x: torch.Tensor, tree: torch.Tensor, w: torch.Tensor, k: int,
         y: Optional[torch.Tensor] = None, out_dtype: Optional[torch.dtype] = None,
         epilogue: Optional[str] = None, epi_arg: Optional[torch.Tensor] = None,
         eps: float = 0.0, bias: Optional[torch.Tensor] = None, relu: bool = False,
         residual: Optional[torch.Tensor] = None, power: float = 1.0) -> torch.Tensor:
    """APR convolution (``apr_conv``).  x [N_p] or [N_p, c_in]; w FP32
    [nw, k,k,k] or [nw, c_out, c_in, k,k,k] with nw 1 or the number of levels."""
    nw, cout, cin = _wshape(acc, w, k)
    if x.shape[0] != acc.n_particles or (x.dim() == 2 and x.shape[1] != cin) or (x.dim() == 1 and cin != 1):
        raise ValueError("x has the wrong shape")
    if y is None:
        shape = (acc.n_particles,) if (w.dim() == 4 and x.dim() == 1) else (acc.n_particles, cout)
        y = torch.empty(shape, dtype=out_dtype or x.dtype, device=x.device)
    d = _desc(k, cin, cout, nw, x.dtype, y.dtype, epilogue, eps, epi_arg, bias, relu, residual, power)
    L.check(acc._lib.apr_conv(acc.handle, ctypes.byref(d), _ptr(x),
                              _ptr(tree) if tree is not None and tree.numel() else None,
                              _ptr(w), _ptr(y), _stream()))
    return y


def gradient_magnitude(acc: AprAccess, x: torch.Tensor, tree: torch.Tensor, w3: torch.Tensor,
                       y: Optional[torch.Tensor] = None) -> torch.Tensor:
    """|grad| of particle values x [N_p] (FP32 or BF16) from three 3^3 stencils
    per level, w3 FP32 [nw, 3, 3, 3, 3] (``apr_conv`` with APR_EPI_GRADMAG);
    per-level stencils come from ``stencil_levels(..., "adaptive", ...)``."""
    if w3.dtype != torch.float32 or w3.dim() != 5 or tuple(w3.shape[1:]) != (3, 3, 3, 3):
        raise ValueError("w3 must be FP32 [nw, 3, 3, 3, 3]")
    nw = w3.shape[0]
    if nw not in (1, acc.n_levels):
        raise ValueError("w3 must hold 1 or n_levels stencil triples")
    if x.dim() != 1 or x.shape[0] != acc.n_particles:
        raise ValueError("x has the wrong shape")
    if y is None:
        y = torch.empty(acc.n_particles, dtype=torch.float32, device=x.device)
    d = _desc(3, 1, 1, nw, x.dtype, y.dtype, "gradmag")
    L.check(acc._lib.apr_conv(acc.handle, ctypes.byref(d), _ptr(x),
                              _ptr(tree) if tree is not None and tree.numel() else None,
                              _ptr(w3.contiguous()), _ptr(y), _stream()))
    return y


def conv_bwd_data(acc: AprAccess, dy: torch.Tensor, w: torch.Tensor, k: int,
                  dx: Optional[torch.Tensor] = None) -> torch.Tensor:
    """Gradient of ``conv`` with respect to x (``apr_conv_bwd_data``); dy FP32."""
    nw, cout, cin = _wshape(acc, w, k)
    dy2 = dy.reshape(acc.n_particles, cout).contiguous()
    if dx is None:
        dx = torch.empty((acc.n_particles, cin), dtype=torch.float32, device=dy.device)
    dt = torch.empty((max(acc.n_tree, 1), cin), dtype=torch.float32, device=dy.device)
    d = _desc(k, cin, cout, nw, torch.float32, torch.float32)
    L.check(acc._lib.apr_conv_bwd_data(acc.handle, ctypes.byref(d), _ptr(dy2), _ptr(w), _ptr(dx), _ptr(dt),
                                       _stream()))
    return dx


def conv_bwd_weight(acc: AprAccess, x: torch.Tensor, tree: torch.Tensor, dy: torch.Tensor, k: int,
                    nw: int, c_in: int, c_out: int) -> torch.Tensor:
    """Gradient of ``conv`` with respect to the weights (``apr_conv_bwd_weight``):
    FP32 [nw, c_out, c_in, k, k, k]."""
    d = _desc(k, c_in, c_out, nw, x.dtype, torch.float32)
    nbytes = int(acc._lib.apr_conv_bwd_weight_ws(acc.handle, ctypes.byref(d)))
    ws = torch.empty(max(nbytes, 8), dtype=torch.uint8, device=x.device)
    dw = torch.empty((nw, c_out, c_in, k, k, k), dtype=torch.float32, device=x.device)
    dy2 = dy.reshape(acc.n_particles, c_out).contiguous()
    L.check(acc._lib.apr_conv_bwd_weight(acc.handle, ctypes.byref(d), _ptr(x),
                                         _ptr(tree) if tree is not None and tree.numel() else None,
                                         _ptr(dy2), _ptr(dw), _ptr(ws), nbytes, _stream()))
    return dw


def neighbor_map(acc: AprAccess, k: int, particles: torch.Tensor) -> torch.Tensor:
    """Source/index code of every tap of the listed particles (``apr_neighbor_map``)."""
    p = particles.to(torch.int64).contiguous()
    out = torch.full((p.numel(), k ** 3), -2, dtype=torch.int64, device=p.device)
    L.check(acc._lib.apr_neighbor_map(acc.handle, k, _ptr(p), p.numel(), _ptr(out), _stream()))
    return out


def richardson_lucy(acc: AprAccess, u: torch.Tensor, psf, n_iter: int, eps_rel: float = 1e-12,
                    out: Optional[torch.Tensor] = None, init: Optional[torch.Tensor] = None,
                    power: float = 1.0) -> torch.Tensor:
    """APR Richardson-Lucy deconvolution of particle values u (FP32) with the
    PSF restricted to every level (``apr_richardson_lucy``), starting from
    ``init`` (u when None), the update raised to ``power``."""
    psf = np.asarray(psf, np.float64)
    k = psf.shape[-1]
    w = torch.from_numpy(stencil_levels(psf, "restrict", k, acc.l_min, acc.l_max)).to(u.device)
    wf = torch.from_numpy(stencil_levels(psf, "restrict", k, acc.l_min, acc.l_max, flip=True)).to(u.device)
    nbytes = int(acc._lib.apr_richardson_lucy_workspace(acc.handle))
    ws = torch.empty(nbytes, dtype=torch.uint8, device=u.device)
    if out is None:
        out = torch.empty_like(u)
    L.check(acc._lib.apr_richardson_lucy(acc.handle, k, w.shape[0], _ptr(w), _ptr(wf), _ptr(u), _ptr(init), _ptr(out),
                                         int(n_iter), float(eps_rel), float(power), _ptr(ws), _stream()))
    return out


def richardson_lucy_static(acc: AprAccess, u: torch.Tensor, w: torch.Tensor, w_flip: torch.Tensor, n_iter: int,
                           out: torch.Tensor, eps_rel: float = 1e-12, init: Optional[torch.Tensor] = None,
                           power: float = 1.0) -> torch.Tensor:
    """``apr_richardson_lucy_static``: the same iterations on the library's
    static per-device scratch (no device allocation in the call).  w, w_flip:
    FP32 per-level PSF and flipped PSF [nw, k, k, k] already on the device
    (``stencil_levels`` with "restrict"); out: a caller-allocated FP32 [N_p]."""
    k = int(w.shape[-1])
    L.check(acc._lib.apr_richardson_lucy_static(acc.handle, k, int(w.shape[0]), _ptr(w), _ptr(w_flip), _ptr(u),
                                                _ptr(init), _ptr(out), int(n_iter), float(eps_rel), float(power),
                                                _stream()))
    return out


# ---------------------------------------------------------------------------
# Surrogate network support (apr_moments ... apr_level_weights)
# ---------------------------------------------------------------------------

class Workspace:
    """Device scratch of apr_nn_workspace bytes for up to ``channels`` channels."""

    def __init__(self, channels: int = 16, device="cuda"):
        n = int(L.load().apr_nn_workspace(channels))
        self.channels = channels
        self.buf = torch.empty(n, dtype=torch.uint8, device=device)

    @property
    def ptr(self) -> int:
        return self.buf.data_ptr()


def _f32(t: torch.Tensor) -> torch.Tensor:
    if t.dtype != torch.float32:
        raise ValueError("expected FP32")
    return t


def moments(u: torch.Tensor, log: bool, ws: Workspace, stats: Optional[torch.Tensor] = None) -> torch.Tensor:
    """Device FP64 [mean, sd] of u or log(max(u, 1)) (``apr_moments``)."""
    if stats is None:
        stats = torch.empty(2, dtype=torch.float64, device=u.device)
    L.check(L.load().apr_moments(int(log), _ptr(_f32(u)), u.numel(), _ptr(stats), ws.ptr, _stream()))
    return stats


def pointwise(op: int, a: torch.Tensor, b: Optional[torch.Tensor], stats: torch.Tensor,
              out: Optional[torch.Tensor] = None) -> torch.Tensor:
    """Elementwise map ``op`` of ``apr_pointwise``."""
    if out is None:
        out = torch.empty_like(a)
    if b is not None and b.numel() != a.numel():
        raise ValueError("a and b differ in size")
    L.check(L.load().apr_pointwise(int(op), _ptr(_f32(a)), _ptr(b), a.numel(), _ptr(stats), _ptr(out),
                                   _stream()))
    return out


def relu_bias_grad(y: Optional[torch.Tensor], dy: torch.Tensor, relu: bool, ws: Workspace,
                   want_db: bool = True, dy_pre: Optional[torch.Tensor] = None):
    """(dy * [y > 0] or dy, column sums) (``apr_relu_bias_grad``)."""
    dy2 = dy if dy.dim() == 2 else dy.reshape(-1, 1)
    c = dy2.shape[1]
    if c > ws.channels:
        raise ValueError("workspace too small for this many channels")
    if dy_pre is None:
        dy_pre = torch.empty_like(dy2)
    db = torch.empty(c, dtype=torch.float32, device=dy.device) if want_db else None
    L.check(L.load().apr_relu_bias_grad(_ptr(y) if relu else None, _ptr(_f32(dy2)), dy2.shape[0], c, int(relu),
                                        _ptr(dy_pre), _ptr(db), ws.ptr, _stream()))
    return dy_pre, db


def rel_l2(a: torch.Tensor, b: torch.Tensor, ws: Workspace, grad: bool = False, grad_scale: float = 1.0,
           out: Optional[torch.Tensor] = None):
    """(device FP64 [|a-b|^2/|b|^2, |b|^2], gradient or None) (``apr_rel_l2``)."""
    if out is None:
        out = torch.empty(2, dtype=torch.float64, device=a.device)
    g = torch.empty_like(a) if grad else None
    L.check(L.load().apr_rel_l2(_ptr(_f32(a)), _ptr(_f32(b)), a.numel(), _ptr(out), _ptr(g), float(grad_scale),
                                ws.ptr, _stream()))
    return out, g


def adam(p: torch.Tensor, g: torch.Tensor, m: torch.Tensor, v: torch.Tensor, step: int, lr: float,
         beta1: float = 0.9, beta2: float = 0.999, eps: float = 1e-8) -> None:
    """In-place Adam step on p (``apr_adam``)."""
    L.check(L.load().apr_adam(_ptr(p), _ptr(g), _ptr(m), _ptr(v), p.numel(), float(lr), float(beta1),
                              float(beta2), float(eps), int(step), _stream()))


def level_weights(P: torch.Tensor, l_min: int, l_max: int) -> torch.Tensor:
    """Per-level weights [l_max-l_min+1, ...] from weight sets P [n_sets, ...]."""
    out = torch.empty((l_max - l_min + 1,) + tuple(P.shape[1:]), dtype=torch.float32, device=P.device)
    L.check(L.load().apr_level_weights(0, _ptr(_f32(P)), _ptr(out), P[0].numel(), P.shape[0], l_min, l_max,
                                       _stream()))
    return out


def fold_level_weights(G: torch.Tensor, n_sets: int, l_min: int, l_max: int) -> torch.Tensor:
    """Gradient of ``level_weights``: per-set sums of the per-level rows of G."""
    out = torch.empty((n_sets,) + tuple(G.shape[1:]), dtype=torch.float32, device=G.device)
    L.check(L.load().apr_level_weights(1, _ptr(_f32(G)), _ptr(out), G[0].numel(), n_sets, l_min, l_max,
                                       _stream()))
    return out


class _DeviceArray:
    """A device array handed out by the library, seen by torch through the
    CUDA array interface (no copy)."""

    def __init__(self, ptr: int, n: int, typestr: str):
        self.__cuda_array_interface__ = {"shape": (n,), "typestr": typestr, "data": (ptr, False), "version": 3}


class DeviceField:
    """An APR built on the device by ``apr_sphere_field``: the LinearAccess
    copied to the host (numpy; ``AprAccess.from_input`` takes it) and the
    particle values as a device tensor."""

    def __init__(self, dims, l_min, l_max, y_idx, xz_end, values):
        self.dims, self.l_min, self.l_max = tuple(dims), int(l_min), int(l_max)
        self.y_idx, self.xz_end, self.values = y_idx, xz_end, values
        self.n_particles = int(values.numel())


def sphere_field(dims, l_min: int, centres, radii, background: float = 100.0, foreground: float = 1000.0,
                 edge_sigma: float = 1.0, noise: bool = True, seed: int = 0) -> DeviceField:
    """APR of a synthetic sphere field built on the device (``apr_sphere_field``)."""
    lib = L.load()
    c = np.ascontiguousarray(centres, dtype=np.float64).reshape(-1, 3)
    r = np.ascontiguousarray(radii, dtype=np.float64).reshape(-1)
    if c.shape[0] != r.shape[0]:
        raise ValueError("one radius per centre")
    d = L.SphereFieldDesc()
    d.dims[:] = [int(v) for v in dims]
    d.l_min = int(l_min)
    d.n_spheres = r.size
    d.centres = c.ctypes.data if r.size else None
    d.radii = r.ctypes.data if r.size else None
    d.background, d.foreground, d.edge_sigma = float(background), float(foreground), float(edge_sigma)
    d.noise = 1 if noise else 0
    d.seed = int(seed)
    h = ctypes.c_void_p()
    L.check(lib.apr_sphere_field(ctypes.byref(d), _stream(), ctypes.byref(h)))
    try:
        info = L.FieldInfo()
        L.check(lib.apr_field_get_info(h, ctypes.byref(info)))
        n, rows = int(info.n_particles), int(info.n_rows)
        y = torch.as_tensor(_DeviceArray(info.y_idx, n, "<i2"), device="cuda").cpu().numpy().view(np.uint16)
        e = torch.as_tensor(_DeviceArray(info.xz_end, rows, "<i8"), device="cuda").cpu().numpy().view(np.uint64)
        v = torch.as_tensor(_DeviceArray(info.values, n, "<f4"), device="cuda").clone()
        torch.cuda.current_stream().synchronize()
    finally:
        L.check(lib.apr_field_destroy(h))
    return DeviceField(tuple(int(a) for a in info.dims), info.l_min, info.l_max, y, e, v)
