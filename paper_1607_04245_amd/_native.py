"""ctypes loader of libfemq.so (the HIP library behind include/fem.h).

The library is loaded on first use. If it has not been built this raises: the
package has no other compute path. torch is imported first so that the HIP
runtime torch ships is the one the library binds to (both name the same
soname), which lets the library run on torch's streams and memory.
"""
from __future__ import annotations

import ctypes
import os
import pathlib
import re

# FEMQ_LIB names another build of the same library (the host-sanitized build
# that the sanitizer test loads); unset, the in-tree library is used.
LIB_PATH = pathlib.Path(os.environ.get("FEMQ_LIB") or pathlib.Path(__file__).resolve().parent / "libfemq.so")
HEADER = pathlib.Path(__file__).resolve().parents[1] / "include" / "fem.h"

FEM_OK = 0
FEM_ERR_INVALID_ARG = -1
FEM_ERR_UNSUPPORTED = -2
FEM_ERR_DEGENERATE = -3
FEM_ERR_HIP = -4
FEM_ERR_NO_TUNING = -5

STATUS_NAMES = {0: "FEM_OK", -1: "FEM_ERR_INVALID_ARG", -2: "FEM_ERR_UNSUPPORTED",
                -3: "FEM_ERR_DEGENERATE", -4: "FEM_ERR_HIP", -5: "FEM_ERR_NO_TUNING"}

F32, F64 = 0, 1
STRATEGY_LANE, STRATEGY_TRANSPOSE, STRATEGY_MFMA, STRATEGY_SHUFFLE, STRATEGY_DEDUP, STRATEGY_COMPONENT = 0, 1, 2, 3, 4, 5
OP_RESIDUAL, OP_RESIDUAL_MESH, OP_GEOMETRY, OP_BACKWARD, OP_RESIDUAL_GATHER = 0, 1, 2, 3, 4
OP_RESIDUAL_P2, OP_BACKWARD_P2 = 5, 6
OP_JACOBIAN, OP_JACOBIAN_P2 = 7, 8
OP_RESIDUAL_P3, OP_BACKWARD_P3, OP_JACOBIAN_P3 = 9, 10, 11
COEF_QUAD, COEF_P1, COEF_P0 = 0, 1, 2
BATCH_NOALLOC_MAX_MESHES = 1024


class FemError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {message}")
        self.status = status


class fem_tuning(ctypes.Structure):
    _fields_ = [("strategy", ctypes.c_int), ("vec", ctypes.c_int),
                ("waves_per_block", ctypes.c_int), ("blocks_per_cu", ctypes.c_int)]


class fem_mesh_desc(ctypes.Structure):
    _fields_ = [("dim", ctypes.c_int), ("physics", ctypes.c_int), ("rule", ctypes.c_int),
                ("coef_space", ctypes.c_int), ("n_elem", ctypes.c_int64),
                ("inv_j", ctypes.c_void_p), ("det_j", ctypes.c_void_p), ("u", ctypes.c_void_p),
                ("coef", ctypes.c_void_p), ("elem_vec", ctypes.c_void_p)]


_c = ctypes
_vp = ctypes.c_void_p
_i = ctypes.c_int
_i64 = ctypes.c_int64

SIGNATURES = {
    "fem_geometry": (_i, [_i, _i64, _i64, _vp, _vp, _i, _vp, _vp, _vp, _vp]),
    "fem_integrate_residual": (_i, [_i, _i, _i, _i, _i, _i64, _vp, _vp, _vp, _vp, _vp, _vp]),
    "fem_integrate_residual_mesh": (_i, [_i, _i, _i, _i, _i, _i64, _i64, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp,
                                         _vp]),
    "fem_integrate_residual_gather": (_i, [_i, _i, _i, _i, _i, _i64, _i64, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp,
                                           _vp]),
    "fem_integrate_residual_p2": (_i, [_i, _i, _i, _i, _i, _i64, _vp, _vp, _vp, _vp, _vp, _vp]),
    "fem_integrate_residual_p3": (_i, [_i, _i, _i, _i, _i, _i64, _vp, _vp, _vp, _vp, _vp, _vp]),
    "fem_integrate_residual_p3_backward": (_i, [_i, _i, _i, _i, _i, _i64, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp]),
    "fem_integrate_residual_p2_backward": (_i, [_i, _i, _i, _i, _i, _i64, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp]),
    "fem_integrate_jacobian": (_i, [_i, _i, _i, _i, _i, _i, _i64, _vp, _vp, _vp, _vp, _vp]),
    "fem_mesh_plan_create": (_i, [_i, _i64, _i64, _vp, _vp, ctypes.POINTER(ctypes.c_void_p)]),
    "fem_mesh_plan_info": (_i, [_vp, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int64),
                                ctypes.POINTER(ctypes.c_int64), ctypes.POINTER(ctypes.c_int),
                                ctypes.POINTER(ctypes.c_int64)]),
    "fem_mesh_plan_destroy": (None, [_vp]),
    "fem_geometry_planned": (_i, [_vp, _vp, _i, _vp, _vp, _vp, _vp]),
    "fem_integrate_residual_planned": (_i, [_vp, _i, _i, _i, _i, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp]),
    "fem_integrate_residual_gather_planned": (_i, [_vp, _i, _i, _i, _i, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp]),
    "fem_integrate_residual_backward": (_i, [_i, _i, _i, _i, _i, _i64, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp]),
    "fem_batch_plan_create": (_i, [ctypes.POINTER(fem_mesh_desc), _i, _i, ctypes.POINTER(_vp)]),
    "fem_batch_plan_set_launch": (_i, [_vp, _i, _i]),
    "fem_batch_plan_autotune": (_i, [_vp, _vp, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_int)]),
    "fem_batch_run": (_i, [_vp, _vp]),
    "fem_batch_run_noalloc": (_i, [ctypes.POINTER(fem_mesh_desc), _i, _i, _i, _i, _vp]),
    "fem_batch_capture": (_i, [_vp, _vp]),
    "fem_batch_replay": (_i, [_vp, _vp]),
    "fem_batch_plan_destroy": (None, [_vp]),
    "fem_assembly_plan_create": (_i, [_i, _i64, _i64, _vp, _vp, ctypes.POINTER(_vp)]),
    "fem_assemble": (_i, [_vp, _i, _i, _vp, _vp, _vp]),
    "fem_assembly_plan_info": (_i, [_vp, ctypes.POINTER(_i), ctypes.POINTER(_i64), ctypes.POINTER(_i64)]),
    "fem_assembly_plan_destroy": (None, [_vp]),
    "fem_restrict": (_i, [_i, _i, _i, _i64, _i64, _vp, _vp, _vp, _vp]),
    "fem_get_tuning": (_i, [_i, _i, _i, _i, _i, ctypes.POINTER(fem_tuning)]),
    "fem_set_tuning": (_i, [_i, _i, _i, _i, _i, ctypes.POINTER(fem_tuning)]),
    "fem_autotune": (_i, [_i, _i, _i, _i, _i, _i64, ctypes.c_char_p]),
    "fem_load_tuning": (_i, [ctypes.c_char_p]),
    "fem_stream_copy": (_i, [_vp, _vp, _i64, _vp]),
    "fem_stream_rows": (_i, [_i, _i64, _i, _i, _vp, _vp, _vp]),
    "fem_last_error": (ctypes.c_char_p, []),
}

_LIB = None


def header_functions() -> list[str]:
    """Names of the functions include/fem.h declares."""
    text = HEADER.read_text()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(fem_[a-z_0-9]+)\s*\(", text)))


def lib():
    global _LIB
    if _LIB is None:
        if not LIB_PATH.exists():
            raise RuntimeError(f"{LIB_PATH} is not built: run __graft_entry__.build() "
                               "(there is no fallback compute path)")
        import torch  # noqa: F401  -- bind to torch's HIP runtime
        lib_ = ctypes.CDLL(str(LIB_PATH))
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(lib_, name)
            fn.restype = res
            fn.argtypes = args
        _LIB = lib_
    return _LIB


def last_error() -> str:
    msg = lib().fem_last_error()
    return msg.decode() if msg else ""


def check(status: int, what: str = "") -> int:
    if status != FEM_OK:
        raise FemError(status, f"{what}: {last_error()}" if what else last_error())
    return status
