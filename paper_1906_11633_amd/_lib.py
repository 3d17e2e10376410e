"""ctypes declarations of the C ABI in include/orrb.h (argument marshalling only).

Loads the in-tree ``liborrb.so``.  There is no fallback: if the library is missing or
fails to load, every entry point raises.
"""
from __future__ import annotations

import ctypes as C
import os
import threading

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liborrb.so")

P = C.c_void_p

ORRB_OK = 0
STATUS_NAMES = {0: "ORRB_OK", 1: "ORRB_ERR_INVALID_ARGUMENT", 2: "ORRB_ERR_OUT_OF_MEMORY",
                3: "ORRB_ERR_WORKSPACE_TOO_SMALL", 4: "ORRB_ERR_DEVICE", 5: "ORRB_ERR_UNSUPPORTED"}
MAX_LIGHTS_PER_SCENE = 8
MAX_SPOT_LIGHTS_PER_SCENE = 4
NOALLOC_SCRATCH_BYTES = 64 << 20  # ORRB_NOALLOC_SCRATCH_BYTES
# words of the per-call stats destination (orrb_outputs.stats)
STATS_WORDS = 8
STAT_NAMES = ("wait_timeouts", "bin_overflow_frames", "survivor_resetup_frames", "near_vertices", "guard_vertices",
              "tiled_extra_flushes", "invalid_state")


class OrrbError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {message}")
        self.status = status


class LayoutDesc(C.Structure):
    _fields_ = [("n_scenes", C.c_int32), ("scene_object_begin", P), ("object_mesh", P),
                ("scene_light_begin", P), ("light_type", P), ("n_frames", C.c_int32),
                ("frame_scene", P), ("width", P), ("height", P), ("shadow_res", C.c_int32)]


class Tuning(C.Structure):
    _fields_ = [("tile_w", C.c_int32), ("tile_h", C.c_int32), ("bin_cap", C.c_int32), ("persistent", C.c_int32),
                ("path", C.c_int32)]

    def as_tuple(self):
        return (self.tile_w, self.tile_h, self.bin_cap, self.persistent, self.path)


class LayoutInfo(C.Structure):
    _fields_ = [("n_scenes", C.c_int64), ("n_objects", C.c_int64), ("n_lights", C.c_int64),
                ("n_frames", C.c_int64), ("total_pixels", C.c_int64), ("vertex_instances", C.c_int64),
                ("triangle_instances", C.c_int64), ("tile_items", C.c_int64), ("frame_path_frames", C.c_int64),
                ("workspace_bytes", C.c_size_t),
                ("workspace_bytes_any", C.c_size_t), ("grad_workspace_bytes", C.c_size_t),
                ("table_bytes", C.c_size_t), ("tuning", Tuning), ("render_kernels", C.c_int64)]


class Scenes(C.Structure):
    _fields_ = [("object_pose", P), ("object_seg", P), ("object_visible", P)]


class Cameras(C.Structure):
    _fields_ = [("view", P), ("intr", P), ("near_plane", P)]


class Params(C.Structure):
    _fields_ = [("albedo", P), ("roughness", P), ("specular", P), ("light_vec", P),
                ("light_intensity", P), ("exposure", P), ("post", P), ("grain", P), ("grain_w", C.c_int32),
                ("grain_h", C.c_int32), ("light_dir", P), ("light_cone", P), ("shadow_view", P), ("shadow_intr", P),
                ("texture", P), ("tex_xform", P), ("emission", P), ("normal_texture", P)]


class Outputs(C.Structure):
    _fields_ = [("rgb", P), ("depth", P), ("normal", P), ("seg", P), ("tri_id", P), ("vis", P), ("stats", P),
                ("alpha", P), ("rgb8", P), ("track", P)]


class Track(C.Structure):
    """orrb_track: one tracker record per (frame, object of the frame's scene)."""
    _fields_ = [("count", C.c_int32), ("i_min", C.c_int32), ("j_min", C.c_int32), ("i_max", C.c_int32),
                ("j_max", C.c_int32), ("x", C.c_float), ("y", C.c_float), ("w", C.c_float), ("sum_i", C.c_uint64),
                ("sum_j", C.c_uint64)]


TRACK_BYTES = 48
POST_WORDS = 12  # ORRB_POST_WORDS


class Grads(C.Structure):
    _fields_ = [("albedo", P), ("roughness", P), ("specular", P), ("light_vec", P), ("light_intensity", P),
                ("exposure", P)]


class KernelTimes(C.Structure):
    _fields_ = [("vertex_ms", C.c_double), ("raster_ms", C.c_double), ("frame_ms", C.c_double),
                ("vertex_launches", C.c_int64), ("raster_launches", C.c_int64), ("frame_launches", C.c_int64)]


# name -> (restype, argtypes)
SIGNATURES = {
    "orrb_create": (C.c_int, [C.c_int, C.POINTER(P)]),
    "orrb_destroy": (None, [P]),
    "orrb_last_error": (C.c_char_p, []),
    "orrb_add_mesh": (C.c_int, [P, P, P, C.c_int32, P, C.c_int32, C.POINTER(C.c_int32)]),
    "orrb_set_mesh_uv": (C.c_int, [P, C.c_int32, P]),
    "orrb_validate_batch": (C.c_int, [P, P, C.POINTER(Scenes), C.POINTER(Cameras), C.POINTER(Params), P, P]),
    "orrb_add_texture": (C.c_int, [P, P, C.c_int32, C.c_int32, C.POINTER(C.c_int32)]),
    "orrb_layout_create": (C.c_int, [P, C.POINTER(LayoutDesc), C.POINTER(P)]),
    "orrb_layout_destroy": (None, [P]),
    "orrb_layout_info_get": (C.c_int, [P, C.POINTER(LayoutInfo)]),
    "orrb_layout_set_tuning": (C.c_int, [P, C.POINTER(Tuning)]),
    "orrb_render_batch": (C.c_int, [P, P, C.POINTER(Scenes), C.POINTER(Cameras), C.POINTER(Params),
                                    C.POINTER(Outputs), P, C.c_size_t, P]),
    "orrb_render_batch_noalloc": (C.c_int, [P, P, C.POINTER(Scenes), C.POINTER(Cameras), C.POINTER(Params),
                                            C.POINTER(Outputs), P]),
    "orrb_autotune": (C.c_int, [P, P, C.POINTER(Scenes), C.POINTER(Cameras), C.POINTER(Params), C.POINTER(Outputs),
                                P, C.c_size_t, P, C.c_char_p, C.POINTER(Tuning), C.POINTER(C.c_double)]),
    "orrb_graph_create": (C.c_int, [P, P, C.POINTER(Scenes), C.POINTER(Cameras), C.POINTER(Params),
                                    C.POINTER(Outputs), P, C.c_size_t, P, C.POINTER(P)]),
    "orrb_graph_launch": (C.c_int, [P, P]),
    "orrb_graph_destroy": (None, [P]),
    "orrb_shade_backward": (C.c_int, [P, P, C.POINTER(Scenes), C.POINTER(Cameras), C.POINTER(Params), P, P,
                                      C.POINTER(Grads), P, C.c_size_t, P]),
    "orrb_profile_enable": (C.c_int, [P, C.c_int]),
    "orrb_profile_read": (C.c_int, [P, C.POINTER(KernelTimes)]),
    "orrb_wait_timeouts": (C.c_int, [P, C.POINTER(C.c_uint64)]),
}

_lock = threading.Lock()
_lib = None


def load():
    """Load liborrb.so (raises if it has not been built)."""
    global _lib
    with _lock:
        if _lib is None:
            if not os.path.exists(LIB_PATH):
                raise RuntimeError(f"{LIB_PATH} is missing: build the HIP library first "
                                   "(python -c 'import __graft_entry__ as g; g.build()')")
            lib = C.CDLL(LIB_PATH)
            for name, (res, args) in SIGNATURES.items():
                fn = getattr(lib, name)
                fn.restype = res
                fn.argtypes = args
            _lib = lib
    return _lib


def check(status: int):
    if status != ORRB_OK:
        msg = load().orrb_last_error()
        raise OrrbError(status, msg.decode() if msg else "")
