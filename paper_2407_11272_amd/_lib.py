"""ctypes declarations of the C ABI in ``include/wn.h`` (no torch types cross it).

The shared library is built in-tree by ``paper_2407_11272_amd.build``.  There is no
fallback: if ``libwn.so`` is missing or fails to load, every entry point raises.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libwn.so")

WN_OK = 0
WN_ERR_INVALID_ARG = -1
WN_ERR_HIP = -2
WN_ERR_WORKSPACE = -3
WN_ERR_BAD_INDEX = -4
WN_ERR_UNSUPPORTED = -5

WN_OCC_NONE = 0
WN_OCC_THRESHOLD = 1
WN_OCC_SIGMOID = 2

WN_OP_VOXELIZE = 0
WN_OP_BACKWARD = 1
WN_OP_BATCHED = 2
WN_OP_LOSS = 3
WN_OP_FLIP = 4
WN_OP_MORPH = 5
WN_OP_CUBIFY = 6
WN_OP_SMOOTH = 7
WN_OP_SAMPLE = 8
WN_OP_NN = 9
WN_OP_NAIVE = 10

WN_INTEGRAL_GWN = 0
WN_INTEGRAL_NAIVE = 1

WN_BATCH_NO_GRAPH = 1

WN_NOALLOC_SCRATCH_BYTES = 96 << 20

WN_BWD_BEGIN = 1
WN_BWD_END = 2
WN_BWD_VERTEX_SUMS = 4
WN_BWD_TILE = 256

#: every symbol include/wn.h declares
EXPORTED = (
    "wn_workspace_size",
    "wn_voxelize",
    "wn_build_strips",
    "wn_voxelize_strips",
    "wn_occupancy",
    "wn_occupancy_backward",
    "wn_sigmoid_mse",
    "wn_backward",
    "wn_backward_range",
    "wn_backward_splits",
    "wn_build_face_pairs",
    "wn_voxelize_naive",
    "wn_backward_naive",
    "wn_voxelize_batched",
    "wn_workspace_size_batched",
    "wn_release_workspace",
    "wn_autotune",
    "wn_flip_duplicate",
    "wn_adam",
    "wn_morph_step",
    "wn_workspace_size_cubify",
    "wn_cubify",
    "wn_workspace_size_marching",
    "wn_marching_cubes",
    "wn_laplacian_smooth",
    "wn_sample_surface",
    "wn_nn_distance",
    "wn_chamfer_hausdorff",
    "wn_voxelize_strips_noalloc",
    "wn_get_device_error",
    "wn_status_string",
    "wn_version",
)


class WnGrid(ctypes.Structure):
    _fields_ = [("lo", ctypes.c_float * 3), ("hi", ctypes.c_float * 3), ("n", ctypes.c_int32 * 3)]


class WnMeshDesc(ctypes.Structure):
    _fields_ = [
        ("V", ctypes.c_void_p),
        ("nV", ctypes.c_int64),
        ("F", ctypes.c_void_p),
        ("nF", ctypes.c_int64),
        ("grid", WnGrid),
        ("W", ctypes.c_void_p),
        ("occ", ctypes.c_void_p),
        ("occ_mode", ctypes.c_int32),
        ("tau", ctypes.c_float),
        ("k", ctypes.c_float),
        ("point_begin", ctypes.c_int64),
        ("point_count", ctypes.c_int64),
        ("strips", ctypes.c_void_p),
        ("n_strip_records", ctypes.c_int64),
    ]


class WnError(RuntimeError):
    def __init__(self, fn: str, status: int, msg: str):
        super().__init__(f"{fn}: {msg} (status {status})")
        self.status = status


_lib = None


def load():
    """Load ``libwn.so`` (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_2407_11272_amd.build` "
                          "(there is no CPU fallback)")
    lib = ctypes.CDLL(LIB_PATH)
    vp, i64, i32, f32, sz = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_float, ctypes.c_size_t
    gp = ctypes.POINTER(WnGrid)
    lib.wn_workspace_size.restype = sz
    lib.wn_workspace_size.argtypes = [i32, i64, i64, i64]
    lib.wn_voxelize.restype = i32
    lib.wn_voxelize.argtypes = [vp, i64, vp, i64, gp, vp, i64, vp, i32, f32, f32, vp, vp, sz, vp]
    lib.wn_build_strips.restype = i32
    lib.wn_build_strips.argtypes = [vp, i64, i64, vp, i64, ctypes.POINTER(ctypes.c_int64)]
    lib.wn_voxelize_strips.restype = i32
    lib.wn_voxelize_strips.argtypes = [vp, i64, vp, i64, vp, i64, gp, vp, i64, vp, i32, f32, f32, vp, vp, sz, vp]
    lib.wn_occupancy.restype = i32
    lib.wn_occupancy.argtypes = [vp, i64, i32, f32, f32, vp, vp]
    lib.wn_occupancy_backward.restype = i32
    lib.wn_occupancy_backward.argtypes = [vp, vp, i64, f32, f32, vp, vp]
    lib.wn_release_workspace.restype = i32
    lib.wn_release_workspace.argtypes = [vp]
    lib.wn_sigmoid_mse.restype = i32
    lib.wn_sigmoid_mse.argtypes = [vp, vp, i64, f32, f32, vp, vp, vp, sz, vp]
    lib.wn_backward.restype = i32
    lib.wn_backward.argtypes = [vp, i64, vp, i64, gp, vp, i64, vp, vp, vp, vp, sz, vp]
    lib.wn_backward_range.restype = i32
    lib.wn_backward_range.argtypes = [vp, i64, vp, i64, vp, i64, gp, vp, i64, vp, i64, i64, i32, vp, vp, vp, sz,
                                      vp]
    lib.wn_build_face_pairs.restype = i32
    lib.wn_build_face_pairs.argtypes = [vp, i64, i64, vp, i64, ctypes.POINTER(ctypes.c_int64)]
    lib.wn_backward_splits.restype = i64
    lib.wn_backward_splits.argtypes = [i64, i64]
    lib.wn_voxelize_naive.restype = i32
    lib.wn_voxelize_naive.argtypes = [vp, i64, vp, i64, gp, vp, i64, vp, i32, f32, f32, vp, vp, sz, vp]
    lib.wn_backward_naive.restype = i32
    lib.wn_backward_naive.argtypes = [vp, i64, vp, i64, gp, vp, i64, vp, vp, vp, vp, sz, vp]
    lib.wn_voxelize_batched.restype = i32
    lib.wn_voxelize_batched.argtypes = [ctypes.POINTER(WnMeshDesc), i32, i32, vp, sz, vp]
    lib.wn_workspace_size_batched.restype = sz
    lib.wn_workspace_size_batched.argtypes = [ctypes.POINTER(WnMeshDesc), i32]
    lib.wn_autotune.restype = i32
    lib.wn_autotune.argtypes = [i32, ctypes.POINTER(WnMeshDesc), i32, vp, sz, vp, ctypes.c_char_p, sz]
    lib.wn_flip_duplicate.restype = i32
    lib.wn_flip_duplicate.argtypes = [vp, i64, vp, i64, f32, vp, vp, vp, sz, vp]
    lib.wn_adam.restype = i32
    lib.wn_adam.argtypes = [vp, vp, vp, vp, i64, i64, f32, f32, f32, f32, vp]
    lib.wn_morph_step.restype = i32
    lib.wn_morph_step.argtypes = [vp, i64, vp, i64, gp, vp, i32, f32, f32, f32, f32, f32, f32, i64, i32, vp, vp,
                                  vp, vp, sz, vp]
    lib.wn_workspace_size_cubify.restype = sz
    lib.wn_workspace_size_cubify.argtypes = [gp]
    lib.wn_cubify.restype = i32
    lib.wn_cubify.argtypes = [vp, gp, vp, i64, vp, i64, vp, vp, sz, vp]
    lib.wn_workspace_size_marching.restype = sz
    lib.wn_workspace_size_marching.argtypes = [gp]
    lib.wn_marching_cubes.restype = i32
    lib.wn_marching_cubes.argtypes = [vp, gp, f32, vp, i64, vp, i64, vp, vp, sz, vp]
    lib.wn_laplacian_smooth.restype = i32
    lib.wn_laplacian_smooth.argtypes = [vp, i64, vp, i64, f32, i32, i32, vp, vp, sz, vp]
    lib.wn_sample_surface.restype = i32
    lib.wn_sample_surface.argtypes = [vp, i64, vp, i64, vp, i64, vp, vp, vp, sz, vp]
    lib.wn_nn_distance.restype = i32
    lib.wn_nn_distance.argtypes = [vp, i64, vp, i64, vp, vp, sz, vp]
    lib.wn_chamfer_hausdorff.restype = i32
    lib.wn_chamfer_hausdorff.argtypes = [vp, i64, vp, i64, vp, vp, sz, vp]
    lib.wn_voxelize_strips_noalloc.restype = i32
    lib.wn_voxelize_strips_noalloc.argtypes = [vp, i64, vp, i64, vp, i64, gp, vp, i64, vp, i32, f32, f32, vp, vp]
    lib.wn_get_device_error.restype = i32
    lib.wn_get_device_error.argtypes = [vp, vp]
    lib.wn_status_string.restype = ctypes.c_char_p
    lib.wn_status_string.argtypes = [i32]
    lib.wn_version.restype = ctypes.c_char_p
    lib.wn_version.argtypes = []
    _lib = lib
    return lib


def status_string(status: int) -> str:
    return load().wn_status_string(int(status)).decode()


def check(fn: str, status: int) -> None:
    if status != WN_OK:
        raise WnError(fn, status, status_string(status))
