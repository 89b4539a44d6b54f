"""ctypes view of the C-ABI in include/lbmswim.h (argument marshalling only)."""
from __future__ import annotations

import ctypes as C
import os

_LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "_lib", "liblbmswim.so")

LBM_OK, LBM_E_ARG, LBM_E_HIP, LBM_E_OVERLAP, LBM_E_UNSTABLE, LBM_E_STATE, LBM_E_CAPACITY, LBM_E_SYNC = \
    0, -1, -2, -3, -4, -5, -6, -7
ERROR_NAMES = {-1: "LBM_E_ARG", -2: "LBM_E_HIP", -3: "LBM_E_OVERLAP", -4: "LBM_E_UNSTABLE",
               -5: "LBM_E_STATE", -6: "LBM_E_CAPACITY", -7: "LBM_E_SYNC"}
STORAGE = {"f64": 0, "f32": 1, "f16s": 2, "bf16s": 3}
TUNE = {"block": 0, "xcd_order": 1, "graph_steps": 2, "full_remap": 3, "nontemporal": 4, "coop_remap": 5,
        "streaming": 6}
TRAJ_DOUBLES = 16

SYMBOLS = [
    "lbm_init", "lbm_init_batch", "lbm_set_bodies", "lbm_set_bodies_box", "lbm_set_step_limit",
    "lbm_step", "lbm_prepare", "lbm_body_forces", "lbm_body_forces_box", "lbm_get_bodies", "lbm_get_bodies_box",
    "lbm_get_links", "lbm_export_populations", "lbm_export_cells", "lbm_import_populations",
    "lbm_flow_average_begin", "lbm_flow_average_get", "lbm_step_count",
    "lbm_status", "lbm_adjoint", "lbm_tune", "lbm_set_timing", "lbm_get_timing", "lbm_vacuum_run", "lbm_vacuum_run_noalloc",
    "lbm_copy_kernel", "lbm_stream_copy", "lbm_struct_sizes", "lbm_last_error", "lbm_destroy",
]


class LbmParams(C.Structure):
    _fields_ = [("nx", C.c_int32), ("ny", C.c_int32), ("nz", C.c_int32),
                ("periodic_mask", C.c_uint32), ("tau", C.c_double),
                ("storage", C.c_int32), ("shift_log2", C.c_int32),
                ("pop", C.c_void_p * 2), ("flags", C.c_void_p),
                ("traj", C.c_void_p), ("traj_cap", C.c_int64), ("stream", C.c_void_p),
                ("stride", C.c_int64), ("force_average", C.c_int32), ("reserved", C.c_int32),
                ("body_force", C.c_double * 3)]


class LbmBody(C.Structure):
    _fields_ = [("shape", C.c_int32), ("kinematic", C.c_int32),
                ("radius", C.c_double), ("half_len", C.c_double),
                ("mass", C.c_double), ("inertia", C.c_double * 3),
                ("anchor", C.c_double * 3), ("disp", C.c_double * 3),
                ("quat", C.c_double * 4), ("vel", C.c_double * 3), ("omega", C.c_double * 3)]


class LbmSpring(C.Structure):
    _fields_ = [("i", C.c_int32), ("j", C.c_int32), ("k", C.c_double),
                ("gamma", C.c_double), ("rest_len", C.c_double)]


class LbmDrive(C.Structure):
    _fields_ = [("left", C.c_int32), ("middle", C.c_int32), ("right", C.c_int32),
                ("gate_lagged", C.c_int32), ("amplitude", C.c_double), ("period", C.c_double),
                ("phase_lag", C.c_double), ("off_left", C.c_int64), ("off_right", C.c_int64)]


class LbmError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"{ERROR_NAMES.get(code, code)}: {msg}")
        self.code = code


_lib = None


def load():
    """Load the in-tree library; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        raise ImportError(f"{_LIB_PATH} is missing; build it with python -m paper_1108_0786_amd.build")
    lib = C.CDLL(_LIB_PATH)
    P = C.POINTER
    ctx_p = C.c_void_p
    sig = {
        "lbm_init": ([P(LbmParams), P(ctx_p)], C.c_int),
        "lbm_init_batch": ([P(LbmParams), C.c_int32, P(ctx_p)], C.c_int),
        "lbm_set_bodies": ([ctx_p, P(LbmBody), C.c_int32, P(LbmSpring), C.c_int32, P(LbmDrive), C.c_int32], C.c_int),
        "lbm_set_bodies_box": ([ctx_p, C.c_int32, P(LbmBody), C.c_int32, P(LbmSpring), C.c_int32,
                                P(LbmDrive), C.c_int32], C.c_int),
        "lbm_set_step_limit": ([ctx_p, C.c_int32, C.c_int64], C.c_int),
        "lbm_step": ([ctx_p, C.c_int64], C.c_int),
        "lbm_prepare": ([ctx_p, C.c_int64], C.c_int),
        "lbm_body_forces": ([ctx_p, C.c_void_p, C.c_void_p, C.c_int32], C.c_int),
        "lbm_body_forces_box": ([ctx_p, C.c_int32, C.c_void_p, C.c_void_p, C.c_int32], C.c_int),
        "lbm_get_bodies": ([ctx_p, P(LbmBody), C.c_int32], C.c_int),
        "lbm_get_bodies_box": ([ctx_p, C.c_int32, P(LbmBody), C.c_int32], C.c_int),
        "lbm_get_links": ([ctx_p, C.c_int32, C.c_void_p, C.c_void_p, C.c_void_p, C.c_int64, P(C.c_int64)], C.c_int),
        "lbm_export_populations": ([ctx_p, C.c_int32, C.c_void_p], C.c_int),
        "lbm_import_populations": ([ctx_p, C.c_int32, C.c_void_p], C.c_int),
        "lbm_export_cells": ([ctx_p, C.c_int32, C.c_void_p, C.c_int64, C.c_void_p], C.c_int),
        "lbm_flow_average_begin": ([ctx_p, C.c_int32, C.c_int32], C.c_int),
        "lbm_flow_average_get": ([ctx_p, C.c_int32, C.c_void_p, C.c_void_p], C.c_int),
        "lbm_step_count": ([ctx_p, C.c_int32, P(C.c_int64)], C.c_int),
        "lbm_status": ([ctx_p], C.c_int),
        "lbm_adjoint": ([ctx_p, C.c_int64, C.c_int32, P(C.c_double), P(C.c_double), P(C.c_double)], C.c_int),
        "lbm_tune": ([ctx_p, C.c_int32, C.c_int64], C.c_int),
        "lbm_set_timing": ([ctx_p, C.c_int32], C.c_int),
        "lbm_get_timing": ([ctx_p, P(C.c_double), P(C.c_int64)], C.c_int),
        "lbm_vacuum_run": ([P(LbmBody), C.c_int32, P(LbmSpring), C.c_int32, P(LbmDrive), C.c_int32, C.c_int32,
                            C.c_int64, C.c_void_p, C.c_int64, P(LbmBody), C.c_void_p], C.c_int),
        "lbm_vacuum_run_noalloc": ([P(LbmBody), C.c_int32, P(LbmSpring), C.c_int32, P(LbmDrive), C.c_int32,
                                    C.c_int32, C.c_int64, C.c_void_p, C.c_int64, P(LbmBody), C.c_void_p], C.c_int),
        "lbm_copy_kernel": ([C.c_void_p, C.c_void_p, C.c_int64, C.c_int32, C.c_int32, C.c_void_p], C.c_int),
        "lbm_stream_copy": ([C.c_void_p, C.c_void_p, C.c_int64, C.c_int64, C.c_int32, C.c_int32, C.c_void_p],
                            C.c_int),
        "lbm_struct_sizes": ([P(C.c_int64)], C.c_int),
        "lbm_last_error": ([ctx_p], C.c_char_p),
        "lbm_destroy": ([ctx_p], None),
    }
    for name, (args, res) in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = res
    sizes = (C.c_int64 * 4)()
    lib.lbm_struct_sizes(sizes)
    want = [C.sizeof(LbmParams), C.sizeof(LbmBody), C.sizeof(LbmSpring), C.sizeof(LbmDrive)]
    if list(sizes) != want:
        raise ImportError(f"struct layout mismatch: library {list(sizes)} vs binding {want}")
    _lib = lib
    return lib


def check(lib, ctx, rc):
    if rc != LBM_OK:
        msg = lib.lbm_last_error(ctx) if ctx else b""
        raise LbmError(rc, (msg or b"").decode())
    return rc
