"""ctypes declarations of the C ABI in include/glamer.h (argument marshalling only)."""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libglamer.so")

GLM_OK = 0
GLM_EINVAL = -1
GLM_ENOMEM = -2
GLM_EHIP = -3
GLM_ESTATE = -4
GLM_EDATA = -5

GLM_ALPHA_ONLY = 1
GLM_FP32_ALPHA = 2
GLM_RAYS_ORDERED = 4
GLM_NFW_HALOS = 8
GLM_RAYS_STAGED = 16
GLM_INTERP_DEFLECTIONS = 1

# every symbol include/glamer.h declares
EXPORTED = [
    "glm_tree_create", "glm_tree_destroy", "glm_build_tree", "glm_tree_get_info", "glm_tree_export",
    "glm_shoot_workspace_bytes", "glm_shoot", "glm_shoot_direct", "glm_shoot_adjoint",
    "glm_last_error", "glm_version", "glm_shoot_batched_workspace_bytes", "glm_shoot_batched",
    "glm_refine_workspace_bytes", "glm_refine_round", "glm_tree_knn", "glm_interp_state_bytes",
    "glm_interp_round_workspace_bytes", "glm_interp_init", "glm_refine_interp_round",
    "glm_shoot_indexed_workspace_bytes", "glm_shoot_indexed", "glm_shoot_potential", "glm_shoot_direct_nfw",
    "glm_knn_workspace_bytes", "glm_knn", "glm_interp_estimate", "glm_tree_workspace_bytes",
    "glm_tree_required_bytes", "glm_adjoint_workspace_bytes", "glm_shoot_noalloc", "glm_stage_rays",
]

GLM_NOALLOC_MAX_RAYS = 1048576
GLM_COUNTS = 8  # int32 counts per ray (glm_shoot)


class GlmParams(ctypes.Structure):
    _fields_ = [("theta", ctypes.c_double), ("q", ctypes.c_double), ("leaf_size", ctypes.c_int32),
                ("order", ctypes.c_int32), ("flags", ctypes.c_uint32)]


class GlmTreeInfo(ctypes.Structure):
    _fields_ = [("n", ctypes.c_int64), ("ncells", ctypes.c_int64), ("nleaves", ctypes.c_int64),
                ("nlisted", ctypes.c_int64), ("max_level", ctypes.c_int32), ("order", ctypes.c_int32),
                ("check_flags", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("root_x0", ctypes.c_double), ("root_y0", ctypes.c_double), ("root_side", ctypes.c_double),
                ("device_bytes", ctypes.c_size_t)]


class GlmLensRays(ctypes.Structure):
    _fields_ = [("tree", ctypes.c_void_p), ("rx", ctypes.c_void_p), ("ry", ctypes.c_void_p),
                ("nrays", ctypes.c_int64), ("a1", ctypes.c_void_p), ("a2", ctypes.c_void_p),
                ("kappa", ctypes.c_void_p), ("g1", ctypes.c_void_p), ("g2", ctypes.c_void_p)]


class GlamerError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"glamer status {status}: {msg}")
        self.status = status


_lib = None


def load(path: str = LIB_PATH):
    """Load libglamer.so.  Raises if it has not been built: there is no fallback."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"{path} is missing: build it with paper_1312_1128_amd.build_ext.build()")
    import torch  # noqa: F401  -- the HIP runtime torch loaded is the one this library binds to

    lib = ctypes.CDLL(path)
    vp, i64, u32, i32 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_uint32, ctypes.c_int
    st = ctypes.c_int
    P = ctypes.POINTER
    lib.glm_tree_create.argtypes = [P(vp)]
    lib.glm_tree_create.restype = st
    lib.glm_tree_destroy.argtypes = [vp]
    lib.glm_tree_destroy.restype = None
    lib.glm_build_tree.argtypes = [vp, vp, vp, vp, vp, i64, P(GlmParams), vp, ctypes.c_size_t, vp]
    lib.glm_build_tree.restype = st
    lib.glm_tree_workspace_bytes.argtypes = [i64, P(GlmParams), P(ctypes.c_size_t)]
    lib.glm_tree_workspace_bytes.restype = st
    lib.glm_tree_required_bytes.argtypes = [vp, P(ctypes.c_size_t)]
    lib.glm_tree_required_bytes.restype = st
    lib.glm_adjoint_workspace_bytes.argtypes = [vp, i64, P(ctypes.c_size_t)]
    lib.glm_adjoint_workspace_bytes.restype = st
    lib.glm_tree_get_info.argtypes = [vp, P(GlmTreeInfo)]
    lib.glm_tree_get_info.restype = st
    lib.glm_tree_export.argtypes = [vp] + [vp] * 17
    lib.glm_tree_export.restype = st
    lib.glm_shoot_workspace_bytes.argtypes = [i64, P(ctypes.c_size_t)]
    lib.glm_shoot_workspace_bytes.restype = st
    lib.glm_shoot.argtypes = [vp, vp, vp, i64, vp, vp, vp, vp, vp, vp, u32, vp, ctypes.c_size_t, vp]
    lib.glm_stage_rays.argtypes = [vp, vp, i64, vp, ctypes.c_size_t, vp]
    lib.glm_stage_rays.restype = st
    lib.glm_shoot.restype = st
    lib.glm_shoot_noalloc.argtypes = [vp, vp, vp, i64, vp, vp, vp, vp, vp, vp, u32, vp]
    lib.glm_shoot_noalloc.restype = st
    lib.glm_shoot_direct.argtypes = [vp, vp, vp, vp, i64, ctypes.c_double, vp, vp, i64, i32, P(vp), vp]
    lib.glm_shoot_direct.restype = st
    lib.glm_shoot_direct_nfw.argtypes = [vp, vp, vp, vp, i64, ctypes.c_double, vp, vp, i64, i32, P(vp), vp]
    lib.glm_shoot_direct_nfw.restype = st
    lib.glm_shoot_adjoint.argtypes = [vp, vp, vp, i64, vp, vp, vp, vp, vp, vp, vp, vp, vp, u32, vp, ctypes.c_size_t, vp]
    lib.glm_shoot_adjoint.restype = st
    lib.glm_shoot_batched_workspace_bytes.argtypes = [P(ctypes.c_int64), i32, P(ctypes.c_size_t)]
    lib.glm_shoot_batched_workspace_bytes.restype = st
    lib.glm_shoot_batched.argtypes = [P(GlmLensRays), i32, u32, vp, ctypes.c_size_t, vp]
    lib.glm_shoot_batched.restype = st
    lib.glm_refine_workspace_bytes.argtypes = [i64, P(ctypes.c_size_t)]
    lib.glm_refine_workspace_bytes.restype = st
    lib.glm_refine_round.argtypes = [vp, vp, vp, vp, vp, vp, i64, i64, vp, vp, ctypes.c_size_t, vp]
    lib.glm_refine_round.restype = st
    sz = ctypes.c_size_t
    lib.glm_interp_state_bytes.argtypes = [i64, P(sz)]
    lib.glm_interp_state_bytes.restype = st
    lib.glm_interp_round_workspace_bytes.argtypes = [i64, i64, P(sz)]
    lib.glm_interp_round_workspace_bytes.restype = st
    lib.glm_interp_init.argtypes = [vp, vp, i64, ctypes.c_double, ctypes.c_double, ctypes.c_double, i64, vp, sz, vp]
    lib.glm_interp_init.restype = st
    lib.glm_refine_interp_round.argtypes = [vp, vp, vp, vp, vp, vp, vp, vp, i64, i64, i64, ctypes.c_float, u32, vp,
                                            vp, vp, i64, vp, sz, vp, sz, vp]
    lib.glm_refine_interp_round.restype = st
    lib.glm_interp_estimate.argtypes = [vp, vp, vp, vp, vp, vp, vp, vp, vp, i64, i64, i64, vp, sz, vp]
    lib.glm_interp_estimate.restype = st
    lib.glm_shoot_indexed_workspace_bytes.argtypes = [i64, P(sz)]
    lib.glm_shoot_indexed_workspace_bytes.restype = st
    lib.glm_shoot_indexed.argtypes = [vp, vp, vp, vp, i64, vp, vp, vp, vp, vp, u32, vp, sz, vp]
    lib.glm_shoot_indexed.restype = st
    lib.glm_shoot_potential.argtypes = [vp, vp, vp, i64, vp, vp, vp, vp, u32, vp, sz, vp]
    lib.glm_shoot_potential.restype = st
    lib.glm_tree_knn.argtypes = [vp, ctypes.c_int32, vp, vp]
    lib.glm_tree_knn.restype = st
    lib.glm_knn_workspace_bytes.argtypes = [i64, i32, P(ctypes.c_size_t)]
    lib.glm_knn_workspace_bytes.restype = st
    lib.glm_knn.argtypes = [vp, vp, vp, vp, i64, i32, vp, vp, ctypes.c_size_t, vp]
    lib.glm_knn.restype = st
    lib.glm_last_error.argtypes = []
    lib.glm_last_error.restype = ctypes.c_char_p
    lib.glm_version.argtypes = []
    lib.glm_version.restype = ctypes.c_char_p
    _lib = lib
    return lib


def check(rc: int):
    if rc != GLM_OK:
        raise GlamerError(rc, load().glm_last_error().decode())
