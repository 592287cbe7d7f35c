"""ctypes declarations of the C ABI in include/diffrt.h (libdiffrt.so).

Loading fails loudly when the library is missing: there is no fallback
implementation of any step.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libdiffrt.so")

DR_SUCCESS = 0
DR_TERM_INTERIOR = 1
DR_TERM_PRIMARY = 2
DR_TERM_SECONDARY = 4
DR_TERM_ALL = 7

# every entry point declared in include/diffrt.h
EXPORTS = ["drSceneCreate", "drSceneUpdateVertices", "drSceneUpdateAlbedo", "drSceneGetInfo", "drRender",
           "drRenderBackward", "drAdamStep", "drSetProfiling", "drGetProfile", "drGetLastDeviceError", "drSceneDestroy",
           "drGetErrorString", "drEdgeFeatures", "drMlpForward", "drMlpSoftmaxXent", "drMlpBackward",
           "drSceneRefit", "drBatchCreate", "drBatchRefit", "drBatchAdvanceSeed", "drBatchForward", "drBatchBackward",
           "drBatchSetLaunch", "drBatchDestroy", "drAdamStepCounted", "drMlpSoftmaxXentNoAlloc",
           "drBatchCheckHierarchy"]

MLP_PARAMS = 6337
EDGE_FEATURES = 32


class SceneDesc(C.Structure):
    _fields_ = [("num_vertices", C.c_int32), ("num_triangles", C.c_int32),
                ("vertices", C.c_void_p), ("indices", C.c_void_p), ("normals", C.c_void_p),
                ("albedo", C.c_void_p), ("emission", C.c_void_p),
                ("emission_two_sided", C.c_int32), ("background", C.c_float)]


class Camera(C.Structure):
    _fields_ = [("position", C.c_float * 3), ("look_at", C.c_float * 3), ("up", C.c_float * 3),
                ("fov_y_deg", C.c_float), ("near_clip", C.c_float),
                ("width", C.c_int32), ("height", C.c_int32), ("window", C.c_int32 * 4)]


class RenderOptions(C.Structure):
    _fields_ = [("spp", C.c_int32), ("max_depth", C.c_int32), ("seed", C.c_uint64),
                ("view_id", C.c_uint32), ("terms", C.c_uint32), ("unit_mask", C.c_void_p),
                ("edge_pdf", C.c_void_p), ("edge_mix", C.c_float), ("edge_mix_terms", C.c_uint32),
                ("edge_stats", C.c_void_p), ("aov", C.c_int32), ("edge_t_mode", C.c_int32),
                ("edge_candidates", C.c_int32), ("edge_nee", C.c_float), ("edge_nee_width", C.c_float)]


class Profile(C.Structure):
    _fields_ = [("forward_ms", C.c_double), ("primary_ms", C.c_double), ("backward_ms", C.c_double),
                ("forward_launches", C.c_int64), ("primary_launches", C.c_int64),
                ("backward_launches", C.c_int64), ("counts", (C.c_int64 * 5) * 3),
                ("bvh_depth", C.c_int32), ("edge_tree_depth", C.c_int32)]

COUNT_NAMES = ["bvh_nodes", "bvh_tris", "tree_nodes", "atomics", "rays"]
KERNELS = ["forward", "primary", "backward"]


class DiffrtError(RuntimeError):
    pass


_lib = None


def load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it with `python -m paper_1904_12228_amd.build` "
                          "(or __graft_entry__.build()); there is no CPU fallback")
    lib = C.CDLL(LIB_PATH)
    vp, i32 = C.c_void_p, C.c_int32
    sig = {
        "drSceneCreate": [C.POINTER(vp), C.POINTER(SceneDesc), vp],
        "drSceneUpdateVertices": [vp, vp, vp],
        "drSceneUpdateAlbedo": [vp, vp, vp],
        "drSceneGetInfo": [vp, C.POINTER(i32), C.POINTER(i32), C.POINTER(i32)],
        "drRender": [vp, C.POINTER(Camera), C.POINTER(RenderOptions), vp, vp],
        "drRenderBackward": [vp, C.POINTER(Camera), C.POINTER(RenderOptions), vp, vp, vp, vp, vp],
        "drAdamStep": [vp, vp, vp, vp, C.c_int64, C.c_float, C.c_float, C.c_float, C.c_float, C.c_int64, vp],
        "drSetProfiling": [vp, i32, i32],
        "drGetProfile": [vp, C.POINTER(Profile), i32],
        "drGetLastDeviceError": [vp],
        "drSceneDestroy": [vp],
        "drGetErrorString": [C.c_int],
        "drEdgeFeatures": [vp, C.POINTER(Camera), vp, vp],
        "drMlpForward": [vp, vp, i32, vp, vp],
        "drMlpSoftmaxXent": [vp, vp, vp, i32, vp, vp, vp, vp, vp],
        "drMlpBackward": [vp, vp, i32, vp, vp, vp],
        "drSceneRefit": [vp, vp, vp],
        "drBatchCreate": [C.POINTER(vp), vp, i32, C.POINTER(Camera), C.POINTER(RenderOptions), C.POINTER(vp),
                          C.POINTER(vp), vp],
        "drBatchRefit": [vp, vp],
        "drBatchCheckHierarchy": [vp, C.POINTER(i32), vp],
        "drBatchAdvanceSeed": [vp, vp],
        "drBatchForward": [vp, vp],
        "drBatchBackward": [vp, vp, vp, vp, vp],
        "drBatchSetLaunch": [vp, i32, i32],
        "drBatchDestroy": [vp],
        "drAdamStepCounted": [vp, vp, vp, vp, C.c_int64, C.c_float, C.c_float, C.c_float, C.c_float, vp, vp],
        "drMlpSoftmaxXentNoAlloc": [vp, vp, vp, i32, vp, vp, vp, vp],
    }
    assert set(sig) == set(EXPORTS), sorted(set(EXPORTS) ^ set(sig))
    for name, args in sig.items():
        f = getattr(lib, name)
        f.argtypes = args
        f.restype = C.c_char_p if name == "drGetErrorString" else C.c_int
    _lib = lib
    return lib


def check(status: int, what: str):
    if status != DR_SUCCESS:
        msg = load().drGetErrorString(status).decode()
        raise DiffrtError(f"{what} failed: {msg} ({status})")
