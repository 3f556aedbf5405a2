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

_DT = {torch.float32: L.APR_F32, torch.bfloat16: L.APR_BF16}
_MODES = {"same": L.APR_STENCIL_SAME, "restrict": L.APR_STENCIL_RESTRICT,
          "adaptive": L.APR_STENCIL_ADAPTIVE}
_EPI = {None: L.APR_EPI_NONE, "ratio": L.APR_EPI_RATIO, "mul": L.APR_EPI_MUL}


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
                 validate: bool = True):
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
        self.device_bytes = int(info.device_bytes)
        self.dims = tuple(int(v) for v in dims)
        self.level_dims = {l: tuple(info.dims[l]) for l in range(self.l_max + 1)}
        self.particles_per_level = {l: int(info.particles_per_level[l]) for l in range(self.l_min, self.l_max + 1)}
        self.tree_per_level = {l: int(info.tree_per_level[l])
                               for l in range(self.tree_l_min, self.tree_l_max + 1)}

    @classmethod
    def from_input(cls, inp, validate: bool = True) -> "AprAccess":
        return cls(inp.dims, inp.l_min, inp.l_max, inp.y_idx, inp.xz_end, validate=validate)

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


def conv(acc: AprAccess, x: torch.Tensor, tree: torch.Tensor, w: torch.Tensor, k: int,
         y: Optional[torch.Tensor] = None, out_dtype: Optional[torch.dtype] = None,
         epilogue: Optional[str] = None, epi_arg: Optional[torch.Tensor] = None,
         eps: float = 0.0) -> torch.Tensor:
    """Single-channel APR convolution (``apr_conv``).  w: FP32 device tensor
    [n_wlevels, k, k, k] with n_wlevels 1 or the number of levels."""
    if w.dtype != torch.float32:
        raise ValueError("weights are FP32")
    nw = w.shape[0]
    if nw not in (1, acc.n_levels) or w.numel() != nw * k ** 3:
        raise ValueError("w must be [1 or n_levels, k, k, k]")
    if x.shape[0] != acc.n_particles:
        raise ValueError("x has the wrong number of particles")
    if y is None:
        y = torch.empty(acc.n_particles, dtype=out_dtype or x.dtype, device=x.device)
    d = L.ConvDesc()
    d.k, d.c_in, d.c_out, d.n_wlevels = k, 1, 1, nw
    d.x_dtype, d.y_dtype = _DT[x.dtype], _DT[y.dtype]
    d.epilogue = _EPI[epilogue]
    d.eps = float(eps)
    d.epi_arg = _ptr(epi_arg) if epi_arg is not None else None
    L.check(acc._lib.apr_conv(acc.handle, ctypes.byref(d), _ptr(x),
                              _ptr(tree) if tree is not None and tree.numel() else None,
                              _ptr(w), _ptr(y), _stream()))
    return y


def neighbor_map(acc: AprAccess, k: int, particles: torch.Tensor) -> torch.Tensor:
    """Source/index code of every tap of the listed particles (``apr_neighbor_map``)."""
    p = particles.to(torch.int64).contiguous()
    out = torch.full((p.numel(), k ** 3), -2, dtype=torch.int64, device=p.device)
    L.check(acc._lib.apr_neighbor_map(acc.handle, k, _ptr(p), p.numel(), _ptr(out), _stream()))
    return out
