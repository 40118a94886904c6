"""ctypes binding of librf.so (include/radfoam.h): argument marshalling only.

Every step of the walk runs in the HIP library. This module converts torch
CUDA tensors to device pointers, passes torch's current HIP stream, and turns
non-zero status codes into exceptions. There is no CPU fallback: if the
library is missing, importing the package fails.
"""

from __future__ import annotations

import ctypes
import os
from typing import Optional

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "librf.so")

RF_OK = 0
RF_ERR_INVALID_ARG = 1
RF_F32 = 0
RF_BF16 = 1
RF_DENSITY_PLAIN = 0
RF_DENSITY_SOFTPLUS = 1
RF_RAY_BAD_START = -1
RF_RAY_MAX_STEPS = -2
STATUS_NAMES = {0: "RF_OK", 1: "RF_ERR_INVALID_ARG", 2: "RF_ERR_HIP", 3: "RF_ERR_OOM",
                4: "RF_ERR_UNSUPPORTED", 5: "RF_ERR_BUSY"}
RF_ERR_BUSY = 5


class RfError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


class Scene(ctypes.Structure):
    _fields_ = [("sites", ctypes.c_void_p), ("nbr_off", ctypes.c_void_p), ("nbr_idx", ctypes.c_void_p),
                ("density", ctypes.c_void_p), ("sh", ctypes.c_void_p), ("n_sites", ctypes.c_int64),
                ("n_edges", ctypes.c_int64), ("sh_degree", ctypes.c_int32), ("density_activation", ctypes.c_int32)]


class AdamArgs(ctypes.Structure):
    _fields_ = [("lr", ctypes.c_float * 4), ("t", ctypes.c_int32 * 4), ("beta1", ctypes.c_float),
                ("beta2", ctypes.c_float), ("eps", ctypes.c_float), ("softplus_density", ctypes.c_int32)]


class AdamState(ctypes.Structure):
    _fields_ = [(k, ctypes.c_void_p) for k in ("m_sites", "v_sites", "m_density", "v_density", "m_sh", "v_sh")]


class PackedSceneDesc(ctypes.Structure):
    _fields_ = [("base", ctypes.c_void_p), ("bytes", ctypes.c_size_t), ("n_sites", ctypes.c_int64),
                ("n_edges", ctypes.c_int64), ("sh_degree", ctypes.c_int32), ("attr_dtype", ctypes.c_int32),
                ("off_planes", ctypes.c_size_t), ("off_adj", ctypes.c_size_t), ("off_row", ctypes.c_size_t),
                ("off_rec", ctypes.c_size_t), ("off_err", ctypes.c_size_t), ("rec_bytes", ctypes.c_int32),
                ("reserved", ctypes.c_int32)]


class Rays(ctypes.Structure):
    _fields_ = [("origin", ctypes.c_void_p), ("dir", ctypes.c_void_p), ("t_max", ctypes.c_void_p),
                ("start_cell", ctypes.c_void_p), ("n_rays", ctypes.c_int64)]


class Params(ctypes.Structure):
    _fields_ = [("eps", ctypes.c_float), ("max_steps", ctypes.c_int32)]


class CameraDesc(ctypes.Structure):
    _fields_ = [("pose", ctypes.c_float * 12), ("fov_deg", ctypes.c_float), ("width", ctypes.c_int32),
                ("height", ctypes.c_int32), ("model", ctypes.c_int32)]


class BoundDesc(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("p", ctypes.c_float * 6)]


class SurfaceDesc(ctypes.Structure):
    _fields_ = [("kind", ctypes.c_int32), ("max_bounces", ctypes.c_int32), ("centre", ctypes.c_float * 3),
                ("radius", ctypes.c_float), ("ior", ctypes.c_float), ("bound", BoundDesc)]


class WalkLog(ctypes.Structure):
    _fields_ = [("code", ctypes.c_void_p), ("t_exit", ctypes.c_void_p), ("tail", ctypes.c_void_p),
                ("capacity", ctypes.c_int32)]


class Quantiles(ctypes.Structure):
    _fields_ = [("draws", ctypes.c_void_p), ("t", ctypes.c_void_p), ("segment", ctypes.c_void_p),
                ("sigma", ctypes.c_void_p)]


class ServerStats(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_int64), ("completed", ctypes.c_int64), ("rejected_busy", ctypes.c_int64),
                ("rays_done", ctypes.c_int64), ("pool_used_bytes", ctypes.c_int64), ("pool_bytes", ctypes.c_int64),
                ("launches", ctypes.c_int64), ("inflight", ctypes.c_int64)]


_lib: Optional[ctypes.CDLL] = None


def lib() -> ctypes.CDLL:
    """The loaded librf.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                              f"or python paper_2502_01157_amd/build.py")
        # torch first: librf.so and torch both need libamdhip64.so.7, and the
        # first one loaded serves both, so torch must get its own build of it
        import torch  # noqa: F401

        L = ctypes.CDLL(LIB_PATH)
        P = ctypes.c_void_p
        st = ctypes.c_int
        L.rf_last_error.restype = ctypes.c_char_p
        L.rf_version.restype = ctypes.c_char_p
        L.rf_packed_bytes.argtypes = [ctypes.c_int64, ctypes.c_int64, ctypes.c_int32, ctypes.c_int32,
                                      ctypes.POINTER(ctypes.c_size_t)]
        L.rf_pack_scene.argtypes = [ctypes.POINTER(Scene), ctypes.c_int32, P, ctypes.c_size_t, ctypes.c_int,
                                    ctypes.POINTER(PackedSceneDesc), P]
        L.rf_packed_errors.argtypes = [ctypes.POINTER(PackedSceneDesc), P, P]
        L.rf_raygen.argtypes = [ctypes.POINTER(CameraDesc), ctypes.POINTER(BoundDesc), ctypes.c_int32, P, P, P, P,
                                P, P]
        L.rf_render_forward.argtypes = [ctypes.POINTER(PackedSceneDesc), ctypes.POINTER(Rays),
                                        ctypes.POINTER(Params), P, P, P, P]
        L.rf_render_trace.argtypes = [ctypes.POINTER(PackedSceneDesc), ctypes.POINTER(Rays),
                                      ctypes.POINTER(Params), ctypes.c_int32, P, P, P, P, P, P]
        L.rf_render_backward.argtypes = [ctypes.POINTER(PackedSceneDesc), ctypes.POINTER(Rays),
                                         ctypes.POINTER(Params), P, P, P, P, P, P, P, P, ctypes.c_int32, P, P]
        L.rf_render_forward_logged.argtypes = [ctypes.POINTER(PackedSceneDesc), ctypes.POINTER(Rays),
                                               ctypes.POINTER(Params), P, P, P, ctypes.POINTER(WalkLog), P]
        L.rf_render_backward_logged.argtypes = [ctypes.POINTER(PackedSceneDesc), ctypes.POINTER(Rays),
                                                ctypes.POINTER(Params), P, P, P, P, ctypes.POINTER(WalkLog), P, P,
                                                P, ctypes.c_int32, P]
        L.rf_quantile_forward.argtypes = [ctypes.POINTER(PackedSceneDesc), ctypes.POINTER(Rays),
                                          ctypes.POINTER(Params), P, ctypes.POINTER(WalkLog),
                                          ctypes.POINTER(Quantiles), P, P]
        L.rf_render_backward_quantile.argtypes = [ctypes.POINTER(PackedSceneDesc), ctypes.POINTER(Rays),
                                                  ctypes.POINTER(Params), P, P, P, P, ctypes.POINTER(WalkLog),
                                                  ctypes.POINTER(Quantiles), P, P, P, P, ctypes.c_int32, P]
        L.rf_locate.argtypes = [ctypes.POINTER(PackedSceneDesc), P, ctypes.c_int64, P, ctypes.c_int32, P, P]
        L.rf_train_schedule.argtypes = [ctypes.c_int32, ctypes.c_int32, ctypes.POINTER(AdamArgs)]
        L.rf_adam_step.argtypes = [ctypes.c_int64, ctypes.c_int32, ctypes.POINTER(AdamArgs), P, P, P, P, P, P,
                                   ctypes.POINTER(AdamState), P]
        L.rf_densify_scores.argtypes = [P, P, P, ctypes.c_int64, P, P, P]
        L.rf_sample_workspace.argtypes = [ctypes.c_int64, ctypes.POINTER(ctypes.c_size_t)]
        L.rf_sample_cells.argtypes = [P, ctypes.c_int64, P, ctypes.c_int64, P, P, ctypes.c_size_t, P]
        L.rf_sample_cells_noalloc.argtypes = [P, ctypes.c_int64, P, ctypes.c_int64, P, P]
        L.rf_insert_sites.argtypes = [P, P, P, ctypes.c_int64, P, P, ctypes.c_int64, ctypes.c_float, P, P]
        L.rf_gather_rows.argtypes = [P, ctypes.c_int64, ctypes.c_int32, P, ctypes.c_int64, P, P]
        L.rf_keep_workspace.argtypes = [ctypes.c_int64, ctypes.POINTER(ctypes.c_size_t)]
        L.rf_keep_index.argtypes = [P, ctypes.c_int64, P, P, P, ctypes.c_size_t, P]
        L.rf_prune_mask.argtypes = [P, P, P, ctypes.c_int64, ctypes.c_float, P, P]
        L.rf_render_forward_surface.argtypes = [ctypes.POINTER(PackedSceneDesc), ctypes.POINTER(Rays),
                                                ctypes.POINTER(Params), ctypes.POINTER(SurfaceDesc), P, P, P,
                                                ctypes.POINTER(WalkLog), P]
        L.rf_render_backward_surface.argtypes = [ctypes.POINTER(PackedSceneDesc), ctypes.POINTER(Rays),
                                                 ctypes.POINTER(Params), ctypes.POINTER(SurfaceDesc), P, P, P, P,
                                                 ctypes.POINTER(WalkLog), P, P, P, P]
        L.rf_packed_planes.argtypes = [ctypes.POINTER(PackedSceneDesc), P, P]
        L.rf_packed_attributes.argtypes = [ctypes.POINTER(PackedSceneDesc), P, P, P]
        for name in ("rf_packed_bytes", "rf_pack_scene", "rf_packed_errors", "rf_raygen", "rf_render_forward",
                     "rf_render_trace", "rf_render_backward", "rf_render_forward_logged",
                     "rf_render_backward_logged", "rf_quantile_forward", "rf_render_backward_quantile",
                     "rf_locate", "rf_render_forward_surface", "rf_render_backward_surface",
                     "rf_train_schedule", "rf_adam_step", "rf_densify_scores", "rf_sample_workspace",
                     "rf_sample_cells", "rf_sample_cells_noalloc", "rf_prune_mask", "rf_insert_sites",
                     "rf_gather_rows", "rf_keep_workspace", "rf_keep_index",
                     "rf_packed_planes", "rf_packed_attributes"):
            getattr(L, name).restype = st
        L.rf_server_create.argtypes = [ctypes.POINTER(PackedSceneDesc), ctypes.POINTER(Params),
                                       ctypes.POINTER(BoundDesc), ctypes.c_size_t, ctypes.c_int32,
                                       ctypes.POINTER(ctypes.c_void_p)]
        L.rf_server_submit.argtypes = [P, ctypes.POINTER(CameraDesc), ctypes.c_int32, ctypes.POINTER(ctypes.c_uint64)]
        L.rf_server_poll.argtypes = [P, ctypes.POINTER(ctypes.c_uint64), ctypes.c_int32,
                                     ctypes.POINTER(ctypes.c_int32)]
        L.rf_server_result.argtypes = [P, ctypes.c_uint64, P, ctypes.c_size_t]
        L.rf_server_stats_get.argtypes = [P, ctypes.POINTER(ServerStats)]
        L.rf_server_destroy.argtypes = [P]
        L.rf_server_create_mode.argtypes = [ctypes.POINTER(PackedSceneDesc), ctypes.POINTER(Params),
                                            ctypes.POINTER(BoundDesc), ctypes.c_size_t, ctypes.c_int32,
                                            ctypes.c_int32, ctypes.POINTER(ctypes.c_void_p)]
        for name in ("rf_server_create", "rf_server_create_mode", "rf_server_submit", "rf_server_poll",
                     "rf_server_result",
                     "rf_server_stats_get", "rf_server_destroy"):
            getattr(L, name).restype = st
        _lib = L
    return _lib


def check(status: int) -> None:
    if status != RF_OK:
        raise RfError(status, lib().rf_last_error().decode(errors="replace"))
