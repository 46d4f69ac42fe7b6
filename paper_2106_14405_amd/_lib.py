"""ctypes declarations of the C ABI in include/rbsim.h (librbsim.so).

Argument marshalling only; every step of the physics runs in the HIP
library.  Importing this module raises if the library has not been built.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "librbsim.so")

SIM_ABI_VERSION = 6
SIM_OK, SIM_EINVAL, SIM_EDEVICE, SIM_EWORKSPACE, SIM_EABI, SIM_ECAPACITY = 0, -1, -2, -3, -4, -5
SPHERE, BOX, CAPSULE = 0, 1, 2
DYNAMIC, STATIC, KINEMATIC = 0, 1, 2
COLD, PREV, LEARNED = 0, 1, 2
PGS, JACOBI = 0, 1
FLAG_NONFINITE, FLAG_CAPACITY, FLAG_NOT_CONVERGED, FLAG_FELLBACK, FLAG_BAD_RESET = 1, 2, 4, 8, 16

_P = C.POINTER
_f = C.c_float


class BatchDesc(C.Structure):
    _fields_ = [
        ("abi_version", C.c_int), ("num_scenes", C.c_int),
        ("h_body_offset", _P(C.c_int32)), ("h_shape", _P(C.c_uint8)), ("h_motion", _P(C.c_uint8)),
        ("h_param", _P(_f)), ("h_mass", _P(_f)), ("h_friction", _P(_f)), ("h_restitution", _P(_f)),
        ("h_pose", _P(_f)), ("h_vel", _P(_f)),
        ("arm", C.c_int), ("h_arm_base", _P(_f)), ("h_arm_theta", _P(_f)),
        ("link_len", _f * 7), ("arm_radius", _f),
        ("gravity", _f * 3), ("margin", _f), ("baumgarte", _f), ("slop", _f), ("rest_thresh", _f),
        ("ground_friction", _f), ("ground_restitution", _f),
        ("max_pairs", C.c_int), ("max_contacts", C.c_int),
        ("solver", C.c_int), ("warm_start", C.c_int), ("tolerance", _f), ("threads", C.c_int),
        ("stream", C.c_void_p), ("hbm_min_bodies", C.c_int),
        ("h_joint", _P(C.c_uint8)), ("h_joint_axis", _P(_f)), ("h_joint_anchor", _P(_f)),
        ("h_joint_limits", _P(_f)), ("h_joint_parent", _P(C.c_int32)),
        ("n_hulls", C.c_int), ("h_hull_index", _P(C.c_int32)), ("h_hull_vert", _P(_f)),
        ("h_hull_face", _P(C.c_int32)),
    ]


class StateView(C.Structure):
    _fields_ = [("n_bodies", C.c_long), ("pose", C.c_void_p), ("vel", C.c_void_p), ("rest", C.c_void_p),
                ("theta", C.c_void_p), ("arm_state", C.c_void_p), ("joint_state", C.c_void_p),
                ("cache_cap", C.c_int), ("cache_count", C.c_void_p), ("cache_key", C.c_void_p),
                ("cache_lam", C.c_void_p)]


class ContactView(C.Structure):
    _fields_ = [("max_contacts", C.c_int), ("max_pairs", C.c_int), ("count", C.c_void_p), ("key", C.c_void_p),
                ("normal", C.c_void_p), ("point", C.c_void_p), ("phi", C.c_void_p), ("lambda_", C.c_void_p),
                ("colour", C.c_void_p), ("features", C.c_void_p), ("n_pairs", C.c_void_p),
                ("pair_key", C.c_void_p)]


class StatsView(C.Structure):
    _fields_ = [("pairs", C.c_void_p), ("contacts", C.c_void_p), ("colours", C.c_void_p), ("sweeps", C.c_void_p),
                ("flags", C.c_void_p), ("residual", C.c_void_p), ("arm_force", C.c_void_p)]


class ResetPool(C.Structure):
    _fields_ = [("size", C.c_int), ("pose", C.c_void_p), ("vel", C.c_void_p), ("theta", C.c_void_p),
                ("index", C.c_void_p), ("joint_state", C.c_void_p)]


class MlpWeights(C.Structure):
    _fields_ = [("w1", C.c_void_p), ("w2", C.c_void_p), ("w3", C.c_void_p), ("b1", C.c_void_p),
                ("b2", C.c_void_p), ("b3", C.c_void_p), ("mean", C.c_void_p), ("std", C.c_void_p)]


MLP_NPARAM, MLP_NWEIGHT, MLP_NBIAS = 5443, 5312, 131

EXPORTED = ["sim_workspace_bytes", "sim_create", "sim_step", "sim_contacts", "sim_state", "sim_stats",
            "sim_set_export", "sim_set_solver", "sim_set_mlp", "sim_reset", "sim_set_trace", "sim_set_stream",
            "sim_destroy", "sim_last_error", "sim_mlp_forward", "sim_mlp_workspace_bytes", "sim_mlp_stats",
            "sim_mlp_grad", "sim_mlp_adam", "sim_mlp_export", "sim_mlp_gather", "sim_set_persistent",
            "sim_autotune_scratch_bytes", "sim_autotune", "sim_state_bytes", "sim_save_state",
            "sim_load_state", "sim_mlp_grad_noalloc", "sim_mlp_grad_noalloc_max_rows", "sim_query_arm", "sim_set_sleep", "sim_set_persistent_table",
            "sim_set_motors"]

_lib = None


def load():
    """Load librbsim.so (built in-tree).  Raises when it is missing."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build the HIP library first "
                          "(python -c 'import __graft_entry__ as g; g.build()')")
    L = C.CDLL(LIB_PATH)
    L.sim_workspace_bytes.argtypes = [_P(BatchDesc)]
    L.sim_workspace_bytes.restype = C.c_size_t
    L.sim_create.argtypes = [_P(BatchDesc), C.c_void_p, C.c_size_t, _P(C.c_void_p)]
    L.sim_step.argtypes = [C.c_void_p, C.c_void_p, _f, C.c_int]
    L.sim_contacts.argtypes = [C.c_void_p, _P(ContactView)]
    L.sim_state.argtypes = [C.c_void_p, _P(StateView)]
    L.sim_stats.argtypes = [C.c_void_p, _P(StatsView)]
    L.sim_set_export.argtypes = [C.c_void_p, C.c_int]
    L.sim_set_solver.argtypes = [C.c_void_p, C.c_int, C.c_int, _f]
    L.sim_set_mlp.argtypes = [C.c_void_p] + [C.c_void_p] * 8
    L.sim_reset.argtypes = [C.c_void_p, C.c_void_p, _P(ResetPool)]
    L.sim_set_stream.argtypes = [C.c_void_p, C.c_void_p]
    L.sim_set_trace.argtypes = [C.c_void_p, C.c_void_p]
    L.sim_destroy.argtypes = [C.c_void_p]
    L.sim_destroy.restype = None
    L.sim_last_error.argtypes = []
    L.sim_last_error.restype = C.c_char_p
    _v = C.c_void_p
    L.sim_mlp_forward.argtypes = [_P(MlpWeights), _v, C.c_long, _v, _v]
    L.sim_mlp_workspace_bytes.argtypes = [C.c_long]
    L.sim_mlp_workspace_bytes.restype = C.c_size_t
    L.sim_mlp_stats.argtypes = [_v, C.c_long, _v, _v, _v, C.c_size_t, _v]
    L.sim_mlp_grad.argtypes = [_v, _v, _v, _v, _v, _v, C.c_long, _v, _v, _v, C.c_size_t, _v]
    L.sim_mlp_grad_noalloc.argtypes = [_v, _v, _v, _v, _v, _v, C.c_long, _v, _v, _v]
    L.sim_mlp_grad_noalloc_max_rows.argtypes = []
    L.sim_mlp_grad_noalloc_max_rows.restype = C.c_long
    L.sim_mlp_adam.argtypes = [_v, _v, _v, _v, C.c_int, _f, _f, _v, _v]
    L.sim_mlp_export.argtypes = [_v, _v, _v, _v]
    L.sim_mlp_gather.argtypes = [_v, _v, _v, C.c_long, _f, _v]
    L.sim_set_persistent.argtypes = [_v, C.c_int, C.c_int]
    L.sim_query_arm.argtypes = [_v, _v, C.c_int, _f, _v, _v]
    L.sim_set_sleep.argtypes = [_v, _f, C.c_int]
    L.sim_set_motors.argtypes = [_v, _f, _f]
    L.sim_autotune_scratch_bytes.argtypes = [_v]
    L.sim_autotune_scratch_bytes.restype = C.c_size_t
    L.sim_autotune.argtypes = [_v, _v, C.c_size_t, C.c_int, _f, C.c_int, _P(C.c_uint32)]
    L.sim_set_persistent_table.argtypes = [_v, C.c_uint32]
    L.sim_state_bytes.argtypes = [_v]
    L.sim_state_bytes.restype = C.c_size_t
    L.sim_save_state.argtypes = [_v, _v]
    L.sim_load_state.argtypes = [_v, _v]
    for name in ("sim_create", "sim_step", "sim_contacts", "sim_state", "sim_stats", "sim_set_export",
                 "sim_set_solver", "sim_set_mlp", "sim_reset", "sim_set_trace", "sim_set_stream",
                 "sim_mlp_forward", "sim_mlp_stats", "sim_mlp_grad", "sim_mlp_grad_noalloc", "sim_mlp_adam", "sim_mlp_export",
                 "sim_mlp_gather", "sim_set_persistent", "sim_query_arm", "sim_set_sleep", "sim_set_persistent_table", "sim_autotune", "sim_save_state", "sim_load_state",
                 "sim_set_motors"):
        getattr(L, name).restype = C.c_int
    _lib = L
    return L


class SimError(RuntimeError):
    pass


def check(rc: int, what: str):
    if rc != SIM_OK:
        msg = load().sim_last_error().decode(errors="replace")
        raise SimError(f"{what} failed ({rc}): {msg}")
