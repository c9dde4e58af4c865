"""ctypes declarations mirroring include/gesr.h (argument marshalling only).

Loading fails loudly if libgesr.so has not been built: there is no fallback
implementation of any step.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libgesr.so")

GESR_OK = 0
GESR_ERR_INVALID = 1
GESR_ERR_CAPACITY = 2
GESR_ERR_HIP = 3
GESR_ERR_UNSUPPORTED = 4
GESR_BIN_SYNC = 1
GESR_BIN_WORK_ORDER = 2
BIN_STATIC_SCRATCH_BYTES = 64 << 20
MAX_VIEWS = 32
REC_FLOATS = 16
PARTIAL_FLOATS = 10
GRAD2D_FLOATS = 12  # du dv dL00 dL10 dL11 dop dbeta dr dg db dz + zero pad

EXPORTS = (
    "gesr_ctx_create", "gesr_ctx_destroy", "gesr_last_error", "gesr_status_string", "gesr_default_settings",
    "gesr_query_sizes", "gesr_project", "gesr_bin", "gesr_bin_static", "gesr_render_fwd", "gesr_render_bwd", "gesr_render_bwd_tiles",
    "gesr_render_fwd_ext", "gesr_render_bwd_ext", "gesr_render_bwd_tiles_ext", "gesr_surface_points",
    "gesr_project_bwd", "gesr_l1_grad", "gesr_autotune", "gesr_autotune_candidate", "gesr_default_adam_settings",
    "gesr_adam_step", "gesr_prune_workspace_size", "gesr_prune", "gesr_shape_reset", "gesr_knn_workspace_size",
    "gesr_knn", "gesr_gsr_workspace_size", "gesr_gsr", "gesr_default_loss_settings", "gesr_loss_workspace_size",
    "gesr_loss_eq8", "gesr_align_workspace_size", "gesr_surface_align",
)
KNN_MAX = 16

c_float_p = ctypes.POINTER(ctypes.c_float)
c_u32_p = ctypes.POINTER(ctypes.c_uint32)


class Camera(ctypes.Structure):
    _fields_ = [("width", ctypes.c_int32), ("height", ctypes.c_int32), ("fx", ctypes.c_float),
                ("fy", ctypes.c_float), ("cx", ctypes.c_float), ("cy", ctypes.c_float),
                ("viewmat", ctypes.c_float * 12), ("campos", ctypes.c_float * 3)]


class Settings(ctypes.Structure):
    _fields_ = [("sh_degree", ctypes.c_int32), ("kappa", ctypes.c_float), ("rho", ctypes.c_float),
                ("alpha_min", ctypes.c_float), ("alpha_max", ctypes.c_float), ("t_min", ctypes.c_float),
                ("blur", ctypes.c_float), ("znear", ctypes.c_float), ("clip_fac", ctypes.c_float),
                ("bg", ctypes.c_float * 3), ("tile_w", ctypes.c_int32), ("tile_h", ctypes.c_int32),
                ("batch", ctypes.c_int32), ("radix_bits", ctypes.c_int32), ("variant", ctypes.c_int32),
                ("reserved", ctypes.c_int32 * 3)]


class Splats(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("mean", ctypes.c_void_p), ("scale", ctypes.c_void_p),
                ("quat", ctypes.c_void_p), ("opacity", ctypes.c_void_p), ("beta", ctypes.c_void_p),
                ("sh", ctypes.c_void_p)]


class Proj(ctypes.Structure):
    _fields_ = [("rec", ctypes.c_void_p), ("tiles_touched", ctypes.c_void_p), ("rect", ctypes.c_void_p),
                ("depth_key", ctypes.c_void_p)]


class Bins(ctypes.Structure):
    _fields_ = [("m_cap", ctypes.c_uint64), ("tile_sorted", ctypes.c_void_p), ("val_sorted", ctypes.c_void_p),
                ("ranges", ctypes.c_void_p), ("worklist", ctypes.c_void_p), ("inst_base", ctypes.c_void_p),
                ("counters", ctypes.c_void_p), ("scratch", ctypes.c_void_p), ("scratch_bytes", ctypes.c_size_t),
                ("tile_work", ctypes.c_void_p)]


class Grads(ctypes.Structure):
    _fields_ = [("mean", ctypes.c_void_p), ("scale", ctypes.c_void_p), ("quat", ctypes.c_void_p),
                ("opacity", ctypes.c_void_p), ("beta", ctypes.c_void_p), ("sh", ctypes.c_void_p)]


class Sizes(ctypes.Structure):
    _fields_ = [("total_tiles", ctypes.c_uint64), ("total_pixels", ctypes.c_uint64),
                ("bin_scratch_bytes", ctypes.c_size_t), ("bwd_workspace_bytes", ctypes.c_size_t),
                ("max_sort_blocks", ctypes.c_uint64)]


class FwdCounts(ctypes.Structure):
    _fields_ = [("n_listed", ctypes.c_void_p), ("n_hit", ctypes.c_void_p)]


class FwdChannels(ctypes.Structure):
    _fields_ = [("depth", ctypes.c_void_p), ("alpha", ctypes.c_void_p)]


class BwdChannels(ctypes.Structure):
    _fields_ = [("dL_ddepth", ctypes.c_void_p), ("dL_dalpha", ctypes.c_void_p)]


SURFACE_MAX_SAMPLES = 32
SURFACE_BYTES_PER_SPLAT = 64


class SurfaceSettings(ctypes.Structure):
    _fields_ = [("n_samples", ctypes.c_int32), ("level", ctypes.c_float), ("span", ctypes.c_float),
                ("min_alpha", ctypes.c_float)]


class Params(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int32), ("sh_coeffs", ctypes.c_int32), ("mean", ctypes.c_void_p),
                ("log_scale", ctypes.c_void_p), ("quat", ctypes.c_void_p), ("opacity_logit", ctypes.c_void_p),
                ("beta", ctypes.c_void_p), ("sh", ctypes.c_void_p)]


class AdamSettings(ctypes.Structure):
    _fields_ = [("lr_mean", ctypes.c_float), ("lr_scale", ctypes.c_float), ("lr_quat", ctypes.c_float),
                ("lr_opacity", ctypes.c_float), ("lr_beta", ctypes.c_float), ("lr_sh_dc", ctypes.c_float),
                ("lr_sh_rest", ctypes.c_float), ("beta1", ctypes.c_float), ("beta2", ctypes.c_float),
                ("eps", ctypes.c_float), ("entropy_weight", ctypes.c_float), ("step", ctypes.c_int32),
                ("reserved", ctypes.c_int32 * 4)]


class PruneSettings(ctypes.Structure):
    _fields_ = [("min_opacity", ctypes.c_float), ("min_beta", ctypes.c_float)]


class GsrSettings(ctypes.Structure):
    _fields_ = [("w_sdf", ctypes.c_float), ("w_nor", ctypes.c_float)]


_lib = None


def load():
    """Loads libgesr.so; raises if it is missing (no fallback path exists)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"HIP library not built: {LIB_PATH} is missing (run __graft_entry__.build() "
                           "or python paper_2411_09156_amd/build.py)")
    lib = ctypes.CDLL(LIB_PATH)
    P = ctypes.POINTER
    vp = ctypes.c_void_p
    st = ctypes.c_int
    lib.gesr_ctx_create.argtypes = [ctypes.c_int, P(vp)]
    lib.gesr_ctx_create.restype = st
    lib.gesr_ctx_destroy.argtypes = [vp]
    lib.gesr_ctx_destroy.restype = None
    lib.gesr_last_error.argtypes = [vp]
    lib.gesr_last_error.restype = ctypes.c_char_p
    lib.gesr_status_string.argtypes = [st]
    lib.gesr_status_string.restype = ctypes.c_char_p
    lib.gesr_default_settings.argtypes = [P(Settings)]
    lib.gesr_default_settings.restype = None
    lib.gesr_query_sizes.argtypes = [vp, P(Camera), ctypes.c_int, ctypes.c_int, P(Settings), ctypes.c_uint64,
                                     P(Sizes)]
    lib.gesr_query_sizes.restype = st
    lib.gesr_project.argtypes = [vp, P(Splats), P(Camera), ctypes.c_int, P(Settings), P(Proj), vp]
    lib.gesr_project.restype = st
    lib.gesr_bin.argtypes = [vp, P(Proj), P(Camera), ctypes.c_int, ctypes.c_int, P(Settings), P(Bins),
                             ctypes.c_int, P(ctypes.c_uint64), vp]
    lib.gesr_bin.restype = st
    lib.gesr_bin_static.argtypes = lib.gesr_bin.argtypes
    lib.gesr_bin_static.restype = st
    lib.gesr_render_fwd.argtypes = [vp, P(Proj), P(Bins), P(Camera), ctypes.c_int, ctypes.c_int, P(Settings),
                                    vp, vp, vp, P(FwdCounts), vp]
    lib.gesr_render_fwd.restype = st
    lib.gesr_render_fwd_ext.argtypes = [vp, P(Proj), P(Bins), P(Camera), ctypes.c_int, ctypes.c_int, P(Settings),
                                        vp, vp, vp, P(FwdCounts), P(FwdChannels), vp]
    lib.gesr_render_fwd_ext.restype = st
    lib.gesr_render_bwd.argtypes = [vp, P(Splats), P(Proj), P(Bins), P(Camera), ctypes.c_int, P(Settings),
                                    vp, vp, vp, vp, vp, P(Grads), vp]
    lib.gesr_render_bwd.restype = st
    lib.gesr_render_bwd_ext.argtypes = [vp, P(Splats), P(Proj), P(Bins), P(Camera), ctypes.c_int, P(Settings),
                                        vp, vp, vp, P(BwdChannels), vp, vp, P(Grads), vp]
    lib.gesr_render_bwd_ext.restype = st
    lib.gesr_render_bwd_tiles.argtypes = [vp, P(Proj), P(Bins), P(Camera), ctypes.c_int, ctypes.c_int, P(Settings),
                                          vp, vp, vp, vp, vp]
    lib.gesr_render_bwd_tiles.restype = st
    lib.gesr_render_bwd_tiles_ext.argtypes = [vp, P(Proj), P(Bins), P(Camera), ctypes.c_int, ctypes.c_int,
                                              P(Settings), vp, vp, vp, P(BwdChannels), vp, vp]
    lib.gesr_render_bwd_tiles_ext.restype = st
    lib.gesr_project_bwd.argtypes = [vp, P(Splats), P(Proj), P(Bins), P(Camera), ctypes.c_int, P(Settings), vp, vp,
                                     P(Grads), vp]
    lib.gesr_project_bwd.restype = st
    lib.gesr_surface_points.argtypes = [vp, P(Splats), P(Proj), P(Bins), P(Camera), ctypes.c_int, P(Settings),
                                        P(SurfaceSettings), vp, vp, vp, ctypes.c_uint32, vp, vp, vp, vp, vp, vp]
    lib.gesr_surface_points.restype = st
    lib.gesr_l1_grad.argtypes = [vp, vp, vp, ctypes.c_uint64, ctypes.c_float, vp, vp]
    lib.gesr_l1_grad.restype = st
    lib.gesr_default_loss_settings.argtypes = [P(LossSettings)]
    lib.gesr_default_loss_settings.restype = None
    lib.gesr_loss_workspace_size.argtypes = [P(Camera), ctypes.c_int]
    lib.gesr_loss_workspace_size.restype = ctypes.c_size_t
    lib.gesr_loss_eq8.argtypes = [vp, P(Camera), ctypes.c_int, P(LossSettings), vp, vp, vp, vp, vp, ctypes.c_size_t,
                                  vp]
    lib.gesr_loss_eq8.restype = st
    lib.gesr_align_workspace_size.argtypes = [ctypes.c_int]
    lib.gesr_align_workspace_size.restype = ctypes.c_size_t
    lib.gesr_surface_align.argtypes = [vp, P(Splats), vp, ctypes.c_float, ctypes.c_float, P(Grads), vp, vp,
                                       ctypes.c_size_t, vp]
    lib.gesr_surface_align.restype = st
    lib.gesr_autotune.argtypes = [vp, P(Splats), P(Camera), ctypes.c_int, P(Settings), ctypes.c_int, c_float_p,
                                  ctypes.c_int, P(ctypes.c_int), vp]
    lib.gesr_autotune.restype = st
    lib.gesr_autotune_candidate.argtypes = [ctypes.c_int, P(Settings)]
    lib.gesr_autotune_candidate.restype = ctypes.c_int
    lib.gesr_default_adam_settings.argtypes = [P(AdamSettings)]
    lib.gesr_default_adam_settings.restype = None
    lib.gesr_adam_step.argtypes = [vp, P(Params), P(Params), P(Params), P(Grads), P(AdamSettings), vp, vp, vp]
    lib.gesr_adam_step.restype = st
    lib.gesr_prune_workspace_size.argtypes = [ctypes.c_int]
    lib.gesr_prune_workspace_size.restype = ctypes.c_size_t
    lib.gesr_prune.argtypes = [vp, P(Params), P(Params), P(Params), P(PruneSettings), P(Params), P(Params),
                               P(Params), vp, vp, vp, vp, ctypes.c_size_t, vp]
    lib.gesr_prune.restype = st
    lib.gesr_shape_reset.argtypes = [vp, P(Params), P(Params), P(Params), ctypes.c_float, vp]
    lib.gesr_shape_reset.restype = st
    lib.gesr_knn_workspace_size.argtypes = [ctypes.c_int, ctypes.c_int]
    lib.gesr_knn_workspace_size.restype = ctypes.c_size_t
    lib.gesr_knn.argtypes = [vp, P(Splats), ctypes.c_int, vp, vp, vp, vp, vp, vp, ctypes.c_size_t, vp]
    lib.gesr_knn.restype = st
    lib.gesr_gsr_workspace_size.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int]
    lib.gesr_gsr_workspace_size.restype = ctypes.c_size_t
    lib.gesr_gsr.argtypes = [vp, P(Splats), P(Settings), ctypes.c_int, vp, vp, vp, vp, vp, vp, P(GsrSettings), vp,
                             vp, P(Grads), vp, ctypes.c_size_t, vp]
    lib.gesr_gsr.restype = st
    _lib = lib
    return lib


class LossSettings(ctypes.Structure):
    _fields_ = [("lambda_dssim", ctypes.c_float), ("c1", ctypes.c_float), ("c2", ctypes.c_float),
                ("sigma", ctypes.c_float)]


class GesrError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"gesr status {status}: {message}")
        self.status = status
