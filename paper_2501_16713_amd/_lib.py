"""ctypes declarations of the C ABI in include/isg.h (argument marshalling
only; every step of every operator runs in the HIP library)."""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libisg.so")

ISG_OK = 0
STATUS_NAMES = {
    0: "ISG_OK", 1: "ISG_ERR_INVALID_ARG", 2: "ISG_ERR_UNSUPPORTED_SHAPE",
    3: "ISG_ERR_OUT_OF_MEMORY", 4: "ISG_ERR_DEVICE", 5: "ISG_ERR_NOT_FINITE",
    6: "ISG_ERR_CG_BREAKDOWN", 7: "ISG_ERR_STATE",
}
STORAGE = {"fp32": 0, "bf16": 1, "fp16": 2}
OPTIONS = {"spread_chunk": 1, "phase_batch": 2, "graph": 3, "ktile_t1": 4, "kblock": 5, "fft_addr": 6}

# every symbol the header declares, with (restype, argtypes)
_p = C.c_void_p
_i64 = C.c_int64
SIGNATURES = {
    "isg_version": (C.c_char_p, []),
    "isg_last_error": (C.c_char_p, []),
    "isg_device_count": (C.c_int, [C.POINTER(C.c_int)]),
    "isg_plan_create": (C.c_int, [_p, C.POINTER(_p)]),
    "isg_plan_destroy": (C.c_int, [_p]),
    "isg_plan_set_stream": (C.c_int, [_p, _p]),
    "isg_plan_device_bytes": (C.c_int, [_p, C.POINTER(_i64)]),
    "isg_plan_set_timing": (C.c_int, [_p, C.c_int, C.c_char_p]),
    "isg_plan_read_timing": (C.c_int, [_p, C.c_char_p, _i64]),
    "isg_plan_set_option": (C.c_int, [_p, C.c_int, _i64]),
    "isg_plan_get_option": (C.c_int, [_p, C.c_int, C.POINTER(_i64)]),
    "isg_plan_tune": (C.c_int, [_p, C.c_int, _p, _p, _p, _p, C.c_double, C.c_int, C.c_char_p, _i64]),
    "isg_motion_create": (C.c_int, [_p, _p, C.POINTER(_p)]),
    "isg_motion_destroy": (C.c_int, [_p]),
    "isg_traj_create": (C.c_int, [_p, _p, _i64, C.POINTER(_p)]),
    "isg_traj_destroy": (C.c_int, [_p]),
    "isg_traj_count": (C.c_int, [_p, C.POINTER(_i64)]),
    "isg_traj_info": (C.c_int, [_p, C.POINTER(_i64), C.POINTER(_i64), C.POINTER(_i64)]),
    "isg_traj_touched_cells": (C.c_int, [_p, C.POINTER(_i64)]),
    "isg_traj_active_columns": (C.c_int, [_p, C.POINTER(_i64)]),
    "isg_warp": (C.c_int, [_p, _p, _p, _p]),
    "isg_warp_adjoint": (C.c_int, [_p, _p, _p, _p]),
    "isg_warp_adjoint_noalloc": (C.c_int, [_p, _p, _p, _p]),
    "isg_warp_grad_d": (C.c_int, [_p, _p, _p, _p, _p]),
    "isg_sense_forward": (C.c_int, [_p, C.c_int, _p, _p, _p, _p, _p]),
    "isg_sense_adjoint": (C.c_int, [_p, C.c_int, _p, _p, _p, _p, _p]),
    "isg_normal": (C.c_int, [_p, C.c_int, _p, C.c_double, _p, _p, _p, _p]),
    "isg_sense_grad": (C.c_int, [_p, C.c_int, _p, _p, _p, _p, _p, _p, _p]),
    "isg_cg_solve": (C.c_int, [_p, C.c_int, _p, _p, _p, _p, C.c_double, C.c_int, _p,
                               C.POINTER(C.c_double)]),
    "isg_traj_set_shift": (C.c_int, [_p, _p]),
    "isg_traj_dcf": (C.c_int, [_p, _p, C.c_int, _p]),
    "isg_grid_recon": (C.c_int, [_p, _p, _p, _p, _p, _p]),
    "isg_wavelet_forward": (C.c_int, [_p, C.c_int, _p, _p]),
    "isg_wavelet_inverse": (C.c_int, [_p, C.c_int, _p, _p]),
    "isg_power_iteration": (C.c_int, [_p, C.c_int, _p, _p, _p, C.c_int, _p, C.POINTER(C.c_double)]),
    "isg_warp_power_iteration": (C.c_int, [_p, _p, C.c_int, _p, C.POINTER(C.c_double)]),
    "isg_fista_solve": (C.c_int, [_p, C.c_int, _p, _p, _p, _p, C.c_double, C.c_double, C.c_int, C.c_int, _p,
                                  C.POINTER(C.c_double)]),
    "isg_warp_fista_solve": (C.c_int, [_p, _p, _p, C.c_double, C.c_double, C.c_int, C.c_int, _p,
                                       C.POINTER(C.c_double)]),
    "isg_warp_cg_solve": (C.c_int, [_p, _p, _p, C.c_double, C.c_int, _p, C.POINTER(C.c_double)]),
    "isg_register": (C.c_int, [_p, _p, _p, C.c_double, C.c_double, C.c_int, _p, C.POINTER(C.c_double)]),
}


class isg_plan_desc(C.Structure):
    _fields_ = [
        ("ndim", C.c_int),
        ("n", C.c_int64 * 3),
        ("alpha", C.c_int),
        ("width", C.c_int),
        ("beta", C.c_double),
        ("ncoils", C.c_int),
        ("nphases", C.c_int),
        ("storage", C.c_int),
        ("stream", C.c_void_p),
    ]


class IsgError(RuntimeError):
    def __init__(self, status: int, message: str):
        self.status = status
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {message}")


_lib = None


def load(path: str = LIB_PATH):
    """Load libisg.so (once).  Raises if it has not been built: there is no
    fallback path."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise RuntimeError(f"HIP library not built: {path} is missing "
                           "(run __graft_entry__.build() or python -m paper_2501_16713_amd.build)")
    lib = C.CDLL(path)
    for name, (res, args) in SIGNATURES.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def check(status: int) -> None:
    if status != ISG_OK:
        msg = load().isg_last_error().decode(errors="replace")
        raise IsgError(status, msg)
