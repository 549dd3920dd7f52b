"""ctypes binding of libaf.so (include/af.h).  Argument marshalling only:
every step of the method runs in the library's HIP kernels.  There is no
fallback: if the library is missing, loading raises."""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libaf.so")

AF_OK, AF_ERR_ARG, AF_ERR_CFL, AF_ERR_LAYOUT, AF_ERR_BALANCE, AF_ERR_DEVICE, AF_ERR_STATE = 0, -1, -2, -3, -4, -5, -6
STATUS_NAMES = {0: "AF_OK", -1: "AF_ERR_ARG", -2: "AF_ERR_CFL", -3: "AF_ERR_LAYOUT", -4: "AF_ERR_BALANCE",
                -5: "AF_ERR_DEVICE", -6: "AF_ERR_STATE"}

# Every symbol include/af.h declares.
EXPORTS = [
    "af_last_error", "af_ctx_create", "af_ctx_destroy", "af_ctx_set_tile", "af_ctx_get_tile",
    "af_ctx_set_fused_pairs", "af_ctx_get_fused_pairs",
    "af_hier_create", "af_hier_destroy", "af_hier_num_leaves", "af_hier_get_leaves",
    "af_hier_level_range", "af_hier_finest_level", "af_hier_side_relations", "af_hier_side_mask",
    "af_hier_leaf_xy",
    "af_patch_step", "af_ghost_fill", "af_flux_correct", "af_regrid_tag", "af_hier_regrid",
    "af_regrid_apply", "af_reduce_sum", "af_reduce_sum_noalloc", "af_amr_coarse_step", "af_amr_coarse_steps",
    "af_level_advance",
    "af_ctx_advance_shapes", "af_ctx_advance_shapes_upwind", "af_ctx_set_advance_shape", "af_autotune",
    "af_ctx_get_advance_shape",
    "af_cnn_last_error", "af_cnn_create", "af_cnn_destroy", "af_cnn_num_params", "af_cnn_set_params",
    "af_cnn_get_params", "af_cnn_set_normalization", "af_cnn_forward", "af_cnn_loss_grad",
    "af_cnn_adam_step", "af_cnn_features", "af_cnn_tag",
]

# Measurement helpers the library also exports (csrc/af_probe.h); not part
# of the method's interface.
PROBES = ["af_fma_probe", "af_amr_coarse_step_timed"]


class af_problem(ctypes.Structure):
    _fields_ = [("eq", ctypes.c_int32), ("prec", ctypes.c_int32), ("m", ctypes.c_int32),
                ("n0x", ctypes.c_int32), ("n0y", ctypes.c_int32), ("lmax", ctypes.c_int32),
                ("x0", ctypes.c_double), ("y0", ctypes.c_double), ("lx", ctypes.c_double),
                ("ly", ctypes.c_double), ("a", ctypes.c_double), ("b", ctypes.c_double),
                ("c", ctypes.c_double), ("omega", ctypes.c_double), ("xc", ctypes.c_double),
                ("yc", ctypes.c_double), ("qmax", ctypes.c_double)]


class af_state(ctypes.Structure):
    _fields_ = [("dof", ctypes.c_void_p * 4), ("npatch", ctypes.c_int32), ("pitch", ctypes.c_int32)]


class AFError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


_lib = None


def load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is not built; run `python -m paper_2205_07572_amd.build`")
    # libaf.so and torch both need libamdhip64.so.7; the first one loaded
    # serves the process, so torch (whose runtime owns the device memory and
    # streams we are handed) is loaded first.
    import torch  # noqa: F401
    L = ctypes.CDLL(LIB_PATH)
    P = ctypes.c_void_p
    i32 = ctypes.c_int32
    D = ctypes.c_double
    S = ctypes.POINTER(af_state)
    L.af_last_error.restype = ctypes.c_char_p
    L.af_ctx_create.argtypes = [ctypes.POINTER(af_problem), ctypes.POINTER(P)]
    L.af_ctx_destroy.argtypes = [P]
    L.af_ctx_set_tile.argtypes = [P, i32]
    L.af_ctx_get_tile.argtypes = [P]
    L.af_ctx_get_tile.restype = i32
    L.af_ctx_set_fused_pairs.argtypes = [P, i32]
    L.af_ctx_get_fused_pairs.argtypes = [P]
    L.af_ctx_get_fused_pairs.restype = i32
    L.af_hier_create.argtypes = [P, i32, P, P, P, ctypes.POINTER(P)]
    L.af_hier_destroy.argtypes = [P]
    L.af_hier_num_leaves.argtypes = [P]
    L.af_hier_num_leaves.restype = i32
    L.af_hier_get_leaves.argtypes = [P, P, P, P]
    L.af_hier_level_range.argtypes = [P, i32, ctypes.POINTER(i32), ctypes.POINTER(i32)]
    L.af_hier_finest_level.argtypes = [P]
    L.af_hier_finest_level.restype = i32
    L.af_hier_side_relations.argtypes = [P, P]
    L.af_hier_side_mask.argtypes = [P]
    L.af_hier_side_mask.restype = P
    L.af_patch_step.argtypes = [P, S, S, i32, i32, i32, D, D, i32, P, P, P, P]
    L.af_hier_leaf_xy.argtypes = [P]
    L.af_hier_leaf_xy.restype = P
    L.af_ghost_fill.argtypes = [P, P, S, ctypes.c_uint32, i32, i32, P]
    L.af_flux_correct.argtypes = [P, P, S, ctypes.c_uint32, i32, P, P]
    L.af_regrid_tag.argtypes = [P, P, S, ctypes.c_uint32, i32, i32, D, D, P, P, P]
    L.af_hier_regrid.argtypes = [P, P, P, ctypes.POINTER(P)]
    L.af_regrid_apply.argtypes = [P, P, S, ctypes.c_uint32, P, S, P]
    L.af_reduce_sum.argtypes = [P, P, S, ctypes.c_uint32, P, P]
    L.af_reduce_sum_noalloc.argtypes = [P, P, S, ctypes.c_uint32, P, P]
    L.af_amr_coarse_step.argtypes = [P, P, S, ctypes.POINTER(ctypes.c_uint32), D, D, P, i32, P]
    L.af_amr_coarse_steps.argtypes = [P, P, S, ctypes.POINTER(ctypes.c_uint32), D, D, i32, P, i32, P]
    L.af_level_advance.argtypes = [P, P, S, ctypes.POINTER(ctypes.c_uint32), i32, D, i32, P]
    L.af_ctx_advance_shapes.argtypes = [P, P, P, i32]
    L.af_ctx_advance_shapes.restype = i32
    L.af_ctx_advance_shapes_upwind.argtypes = [P, P, P, i32]
    L.af_ctx_advance_shapes_upwind.restype = i32
    L.af_ctx_set_advance_shape.argtypes = [P, i32, i32]
    L.af_autotune.argtypes = [P, P, S, i32, D, i32, P, P, P]
    L.af_ctx_get_advance_shape.argtypes = [P, ctypes.POINTER(i32), ctypes.POINTER(i32)]
    L.af_fma_probe.argtypes = [i32, P, i32, i32, P]
    L.af_amr_coarse_step_timed.argtypes = [P, P, S, ctypes.POINTER(ctypes.c_uint32), D, D, P, P, P, i32,
                                           ctypes.POINTER(i32), P]
    L.af_cnn_last_error.restype = ctypes.c_char_p
    L.af_cnn_create.argtypes = [i32, ctypes.POINTER(P)]
    L.af_cnn_destroy.argtypes = [P]
    L.af_cnn_num_params.argtypes = [P]
    L.af_cnn_num_params.restype = i32
    L.af_cnn_set_params.argtypes = [P, P]
    L.af_cnn_get_params.argtypes = [P, P]
    L.af_cnn_set_normalization.argtypes = [P, P, P]
    L.af_cnn_forward.argtypes = [P, P, i32, P, P, P]
    L.af_cnn_loss_grad.argtypes = [P, P, P, i32, P, P, P, P]
    L.af_cnn_adam_step.argtypes = [P, P, ctypes.c_float, i32, P]
    L.af_cnn_features.argtypes = [P, P, P, S, ctypes.c_uint32, P, P]
    L.af_cnn_tag.argtypes = [P, P, P, S, ctypes.c_uint32, P, P, P, P]
    for name in EXPORTS + PROBES:
        if name not in ("af_last_error", "af_hier_num_leaves", "af_ctx_get_tile", "af_ctx_get_fused_pairs",
                        "af_hier_finest_level",
                        "af_hier_side_mask", "af_hier_leaf_xy", "af_ctx_advance_shapes", "af_ctx_advance_shapes_upwind", "af_cnn_last_error",
                        "af_cnn_num_params"):
            getattr(L, name).restype = ctypes.c_int
    _lib = L
    return L


def check(status):
    if status != AF_OK:
        msg = load().af_last_error()
        raise AFError(status, msg.decode() if msg else "")


def check_cnn(status):
    if status != AF_OK:
        msg = load().af_cnn_last_error()
        raise AFError(status, msg.decode() if msg else "")
