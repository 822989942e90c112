"""ctypes declarations of libtreecode.so (include/treecode.h).

Loading fails loudly when the library has not been built: there is no
fallback path.  Build it with ``python -m paper_2412_01733_amd.build``.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libtreecode.so")

TC_OK, TC_ERR_INVALID, TC_ERR_NOMEM, TC_ERR_DEVICE, TC_ERR_STATE, TC_ERR_OVERFLOW, TC_ERR_INPUT = range(7)
STATUS_NAMES = {0: "TC_OK", 1: "TC_ERR_INVALID", 2: "TC_ERR_NOMEM", 3: "TC_ERR_DEVICE", 4: "TC_ERR_STATE",
                5: "TC_ERR_OVERFLOW", 6: "TC_ERR_INPUT"}
TC_F32, TC_F64 = 0, 1
TC_WALK_F32C, TC_WALK_F64 = 0, 1
TC_COUNT, TC_STORE_LISTS = 1, 2

# Every exported symbol of the C ABI, as declared in include/treecode.h.
EXPORTS = ("tc_set_allocator", "tc_build", "tc_moments", "tc_forces", "tc_forces_backward",
           "tc_forces_noalloc", "tc_leapfrog_step", "tc_tree_stats", "tc_tree_set_walk_status",
           "tc_tree_set_timing", "tc_tree_export",
           "tc_interaction_counts", "tc_tree_target_order", "tc_tree_free", "tc_last_error", "tc_version")


class TcStats(ctypes.Structure):
    _fields_ = [
        ("n", ctypes.c_int64),
        ("n_nodes", ctypes.c_int64),
        ("n_leaves", ctypes.c_int64),
        ("n_multi_leaves", ctypes.c_int64),
        ("lo", ctypes.c_double * 3),
        ("L", ctypes.c_double),
        ("log2L", ctypes.c_int32),
        ("max_level", ctypes.c_int32),
        ("state", ctypes.c_uint32),
        ("last_mode", ctypes.c_uint32),
        ("interactions", ctypes.c_uint64),
        ("node_visits", ctypes.c_uint64),
        ("lane_visits", ctypes.c_uint64),
        ("momentum", ctypes.c_double * 3),
        ("sum_m_abs_a", ctypes.c_double),
        ("kinetic", ctypes.c_double),
        ("potential", ctypes.c_double),
        ("lin_momentum", ctypes.c_double * 3),
        ("ang_momentum", ctypes.c_double * 3),
        ("stage_ms", ctypes.c_float * 8),
        ("lists_stored", ctypes.c_uint32),
        ("max_stack", ctypes.c_uint32),
        ("group_pops", ctypes.c_uint64),
        ("visits_no_accept", ctypes.c_uint64),
        ("visits_all_accept", ctypes.c_uint64),
        ("visits_box_open", ctypes.c_uint64),
        ("visits_box_accept", ctypes.c_uint64),
        ("walk_steps", ctypes.c_uint64),
        ("walk_single_steps", ctypes.c_uint64),
        ("visits_overlap", ctypes.c_uint64),
        ("visits_overlap_all_accept", ctypes.c_uint64),
        ("list_bytes", ctypes.c_uint64),
    ]


ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p, ctypes.c_void_p)
FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p)


class TreecodeError(RuntimeError):
    def __init__(self, status, message):
        super().__init__("%s: %s" % (STATUS_NAMES.get(status, status), message))
        self.status = status


_lib = None


def load():
    """Load libtreecode.so (raises if it has not been built)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError("libtreecode.so is not built (%s); run `python -m paper_2412_01733_amd.build`" % LIB_PATH)
    L = ctypes.CDLL(LIB_PATH)
    P, I64, D, U32, I = ctypes.c_void_p, ctypes.c_int64, ctypes.c_double, ctypes.c_uint32, ctypes.c_int
    st = ctypes.c_int
    L.tc_set_allocator.argtypes = [ALLOC_FN, FREE_FN, P]
    L.tc_set_allocator.restype = st
    L.tc_build.argtypes = [P, P, I64, I, P, ctypes.POINTER(P)]
    L.tc_build.restype = st
    L.tc_moments.argtypes = [P, P]
    L.tc_moments.restype = st
    L.tc_forces.argtypes = [P, D, D, D, I, U32, P, P, P]
    L.tc_forces.restype = st
    L.tc_forces_backward.argtypes = [P, P, P, P, P, P]
    L.tc_forces_backward.restype = st
    L.tc_forces_noalloc.argtypes = [P, P, I64, I, D, D, D, I, P, P, P]
    L.tc_forces_noalloc.restype = st
    L.tc_leapfrog_step.argtypes = [ctypes.POINTER(P), P, P, P, P, P, I64, I, D, D, D, D, I, P]
    L.tc_leapfrog_step.restype = st
    L.tc_tree_stats.argtypes = [P, ctypes.POINTER(TcStats), P]
    L.tc_tree_stats.restype = st
    L.tc_tree_set_walk_status.argtypes = [P, ctypes.c_uint32, P]
    L.tc_tree_set_walk_status.restype = st
    L.tc_tree_set_timing.argtypes = [P, I]
    L.tc_tree_set_timing.restype = st
    L.tc_tree_export.argtypes = [P, P, P, P, P, P, P, P, P]
    L.tc_tree_export.restype = st
    L.tc_interaction_counts.argtypes = [P, P, P]
    L.tc_interaction_counts.restype = st
    L.tc_tree_target_order.argtypes = [P, P, P]
    L.tc_tree_target_order.restype = st
    L.tc_tree_free.argtypes = [P]
    L.tc_tree_free.restype = None
    L.tc_last_error.argtypes = []
    L.tc_last_error.restype = ctypes.c_char_p
    L.tc_version.argtypes = []
    L.tc_version.restype = ctypes.c_char_p
    _lib = L
    return L


def check(status):
    if status != TC_OK:
        raise TreecodeError(status, load().tc_last_error().decode())
