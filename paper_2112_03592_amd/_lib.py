"""ctypes declarations of the aprconv C ABI (include/aprconv.h).

Loading fails loudly: there is no fallback implementation of any entry point.
"""
from __future__ import annotations

import ctypes
import os
from ctypes import POINTER, c_char_p, c_double, c_float, c_int32, c_int64, c_uint16, c_uint32, c_uint64, c_void_p

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libaprconv.so")

APR_OK, APR_EINVAL, APR_EUNBALANCED, APR_EPARTITION, APR_EUNSUPPORTED, APR_ENOMEM, APR_EDEVICE = range(7)
STATUS_NAMES = {0: "APR_OK", 1: "APR_EINVAL", 2: "APR_EUNBALANCED", 3: "APR_EPARTITION",
                4: "APR_EUNSUPPORTED", 5: "APR_ENOMEM", 6: "APR_EDEVICE"}
APR_F32, APR_BF16, APR_FP8 = 0, 1, 2
APR_VALIDATE_PARTITION, APR_VALIDATE_BALANCE, APR_BUILD_GATHER3, APR_BUILD_GATHER5 = 1, 2, 4, 8
APR_MAX_LEVELS = 17
APR_STENCIL_SAME, APR_STENCIL_RESTRICT, APR_STENCIL_ADAPTIVE = 0, 1, 2
APR_EPI_NONE, APR_EPI_RATIO, APR_EPI_MUL, APR_EPI_MULPOW, APR_EPI_GRADMAG = 0, 1, 2, 3, 4
APR_RL_STATIC_FLOATS = 1 << 24

APR_EXPORT_APR, APR_EXPORT_TREE, APR_EXPORT_TILES = 0, 1, 2

EXPORTED = ["apr_access_build", "apr_access_get_info", "apr_access_export_tree", "apr_access_export",
            "apr_access_destroy",
            "apr_fill_tree", "apr_stencil_levels", "apr_conv", "apr_neighbor_map",
            "apr_richardson_lucy_workspace", "apr_richardson_lucy", "apr_richardson_lucy_static",
            "apr_conv_bwd_data",
            "apr_conv_bwd_weight_ws", "apr_conv_bwd_weight", "apr_nn_workspace", "apr_moments",
            "apr_pointwise", "apr_relu_bias_grad", "apr_rel_l2", "apr_adam", "apr_level_weights",
            "apr_sphere_field", "apr_field_get_info", "apr_field_destroy",
            "apr_tile_prepass_size", "apr_tile_prepass",
            "apr_last_error"]
_SIZE_RETURNING = ("apr_richardson_lucy_workspace", "apr_conv_bwd_weight_ws", "apr_nn_workspace",
                   "apr_tile_prepass_size")


class AccessDesc(ctypes.Structure):
    _fields_ = [("dims", c_int32 * 3), ("l_min", c_int32), ("l_max", c_int32),
                ("y_idx", c_void_p), ("n_particles", c_int64), ("xz_end", c_void_p),
                ("n_rows", c_int64), ("flags", c_uint32)]


class AccessInfo(ctypes.Structure):
    _fields_ = [("n_particles", c_int64), ("n_tree", c_int64), ("n_rows", c_int64),
                ("n_tree_rows", c_int64), ("l_min", c_int32), ("l_max", c_int32),
                ("tree_l_min", c_int32), ("tree_l_max", c_int32),
                ("dims", (c_int32 * 3) * APR_MAX_LEVELS),
                ("particles_per_level", c_int64 * APR_MAX_LEVELS),
                ("tree_per_level", c_int64 * APR_MAX_LEVELS),
                ("n_tiles", c_int64), ("device_bytes", c_int64), ("n_work_items", c_int64)]


class ConvDesc(ctypes.Structure):
    _fields_ = [("k", c_int32), ("c_in", c_int32), ("c_out", c_int32), ("n_wlevels", c_int32),
                ("x_dtype", c_int32), ("y_dtype", c_int32), ("epilogue", c_int32), ("eps", c_float),
                ("epi_arg", c_void_p), ("bias", c_void_p), ("relu", c_int32), ("residual", c_void_p),
                ("power", c_float)]


class SphereFieldDesc(ctypes.Structure):
    _fields_ = [("dims", c_int32 * 3), ("l_min", c_int32), ("n_spheres", c_int64),
                ("centres", c_void_p), ("radii", c_void_p), ("background", c_double),
                ("foreground", c_double), ("edge_sigma", c_double), ("noise", c_int32), ("seed", c_uint64)]


class FieldInfo(ctypes.Structure):
    _fields_ = [("dims", c_int32 * 3), ("l_min", c_int32), ("l_max", c_int32),
                ("n_particles", c_int64), ("n_rows", c_int64), ("y_idx", c_void_p), ("xz_end", c_void_p),
                ("values", c_void_p)]


class AprError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


_lib = None


def load(path: str = LIB_PATH) -> ctypes.CDLL:
    """Load libaprconv.so and declare its signatures (raises if missing)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"{path} is not built; run `python -m paper_2112_03592_amd.build` "
                          f"(the HIP library is required, there is no fallback)")
    lib = ctypes.CDLL(path)
    lib.apr_access_build.argtypes = [POINTER(AccessDesc), c_void_p, POINTER(c_void_p)]
    lib.apr_access_get_info.argtypes = [c_void_p, POINTER(AccessInfo)]
    lib.apr_access_export_tree.argtypes = [c_void_p, c_void_p, c_void_p]
    lib.apr_access_export.argtypes = [c_void_p, c_int32, c_void_p, c_void_p]
    lib.apr_access_destroy.argtypes = [c_void_p]
    lib.apr_fill_tree.argtypes = [c_void_p, c_void_p, c_void_p, c_int32, c_int32, c_void_p]
    lib.apr_stencil_levels.argtypes = [c_int32, c_int32, c_int32, c_void_p, c_int32, c_int32, c_int32,
                                       c_void_p]
    lib.apr_conv.argtypes = [c_void_p, POINTER(ConvDesc), c_void_p, c_void_p, c_void_p, c_void_p, c_void_p]
    lib.apr_neighbor_map.argtypes = [c_void_p, c_int32, c_void_p, c_int64, c_void_p, c_void_p]
    lib.apr_richardson_lucy_workspace.argtypes = [c_void_p]
    lib.apr_richardson_lucy_workspace.restype = ctypes.c_size_t
    lib.apr_richardson_lucy.argtypes = [c_void_p, c_int32, c_int32, c_void_p, c_void_p, c_void_p, c_void_p,
                                        c_void_p, c_int32, c_float, c_float, c_void_p, c_void_p]
    lib.apr_richardson_lucy_static.argtypes = [c_void_p, c_int32, c_int32, c_void_p, c_void_p, c_void_p, c_void_p,
                                               c_void_p, c_int32, c_float, c_float, c_void_p]
    lib.apr_conv_bwd_data.argtypes = [c_void_p, POINTER(ConvDesc), c_void_p, c_void_p, c_void_p, c_void_p,
                                      c_void_p]
    lib.apr_conv_bwd_weight_ws.argtypes = [c_void_p, POINTER(ConvDesc)]
    lib.apr_conv_bwd_weight_ws.restype = ctypes.c_size_t
    lib.apr_conv_bwd_weight.argtypes = [c_void_p, POINTER(ConvDesc), c_void_p, c_void_p, c_void_p, c_void_p,
                                        c_void_p, ctypes.c_size_t, c_void_p]
    lib.apr_nn_workspace.argtypes = [c_int32]
    lib.apr_nn_workspace.restype = ctypes.c_size_t
    lib.apr_moments.argtypes = [c_int32, c_void_p, c_int64, c_void_p, c_void_p, c_void_p]
    lib.apr_pointwise.argtypes = [c_int32, c_void_p, c_void_p, c_int64, c_void_p, c_void_p, c_void_p]
    lib.apr_relu_bias_grad.argtypes = [c_void_p, c_void_p, c_int64, c_int32, c_int32, c_void_p, c_void_p,
                                       c_void_p, c_void_p]
    lib.apr_rel_l2.argtypes = [c_void_p, c_void_p, c_int64, c_void_p, c_void_p, c_float, c_void_p, c_void_p]
    lib.apr_adam.argtypes = [c_void_p, c_void_p, c_void_p, c_void_p, c_int64, c_float, c_float, c_float,
                             c_float, c_int32, c_void_p]
    lib.apr_level_weights.argtypes = [c_int32, c_void_p, c_void_p, c_int64, c_int32, c_int32, c_int32,
                                      c_void_p]
    lib.apr_sphere_field.argtypes = [POINTER(SphereFieldDesc), c_void_p, POINTER(c_void_p)]
    lib.apr_field_get_info.argtypes = [c_void_p, POINTER(FieldInfo)]
    lib.apr_field_destroy.argtypes = [c_void_p]
    lib.apr_tile_prepass_size.argtypes = [c_void_p]
    lib.apr_tile_prepass_size.restype = c_int64
    lib.apr_tile_prepass.argtypes = [c_void_p, c_void_p, c_void_p, c_void_p]
    lib.apr_last_error.argtypes = []
    lib.apr_last_error.restype = c_char_p
    for name in EXPORTED:
        if name != "apr_last_error" and name not in _SIZE_RETURNING:
            getattr(lib, name).restype = c_int32
    _lib = lib
    return lib


def check(status: int) -> None:
    if status != APR_OK:
        msg = load().apr_last_error().decode(errors="replace")
        raise AprError(status, msg)
