"""ctypes binding of the C ABI in ``include/dg.h`` (argument marshalling only).

Every compute call goes to ``libdg.so`` (HIP kernels for gfx950).  There is no
fallback: if the library is missing or fails to load, :func:`lib` raises.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libdg.so")

DG_OK, DG_EINVAL, DG_ENOMEM, DG_EHIP, DG_EUNSUPPORTED, DG_ENONPHYSICAL, DG_EMESH = range(7)
DG_EULER, DG_MHD = 0, 1
DG_FP64, DG_FP32 = 0, 1
DG_FLUX_HLL, DG_FLUX_HLLD, DG_FLUX_EXACT = 0, 1, 2
DG_LIMITER_NONE, DG_LIMITER_MINMOD, DG_LIMITER_WENO = 0, 1, 2
DG_RUN_GRAPH = 1
DG_RUN_MUSCL_HANCOCK = 2
DG_RUN_TWO_STAGE = 4

STATUS_NAMES = {0: "DG_OK", 1: "DG_EINVAL", 2: "DG_ENOMEM", 3: "DG_EHIP", 4: "DG_EUNSUPPORTED",
                5: "DG_ENONPHYSICAL", 6: "DG_EMESH"}


class DGError(RuntimeError):
    def __init__(self, status: int, where: str, msg: str):
        super().__init__(f"{where}: {STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


class NonPhysicalState(DGError):
    pass


class dg_config(ctypes.Structure):
    _fields_ = [("physics", ctypes.c_int), ("precision", ctypes.c_int), ("flux", ctypes.c_int),
                ("limiter", ctypes.c_int), ("gamma", ctypes.c_double)]


_dp = ctypes.POINTER(ctypes.c_double)


class dg_mesh_desc(ctypes.Structure):
    _fields_ = [
        ("dim", ctypes.c_int), ("kind", ctypes.c_int),
        ("n", ctypes.c_int64 * 3), ("lo", ctypes.c_double * 3), ("hi", ctypes.c_double * 3),
        ("ncells", ctypes.c_int64), ("nfaces", ctypes.c_int64), ("box", ctypes.c_double * 2),
        ("cell_volume", _dp), ("cell_centroid", _dp), ("cell_moments", _dp),
        ("face_cells", ctypes.POINTER(ctypes.c_int32)), ("face_area", _dp),
        ("face_normal", _dp), ("face_centroid", _dp),
        ("face_shift", ctypes.POINTER(ctypes.c_int8)),
        ("ninst", ctypes.c_int32), ("inst_n", ctypes.POINTER(ctypes.c_int32)),
        ("inst_box", _dp), ("generators", _dp),
    ]


_lib = None

# (name, restype, argtypes) of every exported symbol of include/dg.h
SYMBOLS = [
    ("dg_mesh_create", ctypes.c_int, [ctypes.POINTER(dg_mesh_desc), ctypes.POINTER(dg_config),
                                      ctypes.POINTER(ctypes.c_void_p)]),
    ("dg_mesh_destroy", None, [ctypes.c_void_p]),
    ("dg_state_len", ctypes.c_int64, [ctypes.c_void_p]),
    ("dg_ncoef", ctypes.c_int, [ctypes.c_void_p]),
    ("dg_rhs", ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    ("dg_limit", ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    ("dg_step", ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_double,
                               ctypes.c_void_p]),
    ("dg_stage1", ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                 ctypes.c_double, ctypes.c_void_p, ctypes.c_void_p]),
    ("dg_stage2", ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                 ctypes.c_void_p, ctypes.c_double, ctypes.c_void_p,
                                 ctypes.c_double, ctypes.c_void_p, ctypes.c_void_p]),
    ("dg_step_devdt", ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                     ctypes.c_void_p, ctypes.c_void_p]),
    ("dg_step_cfl", ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                   ctypes.c_void_p, ctypes.c_double, ctypes.c_void_p,
                                   ctypes.c_void_p]),
    ("dg_adjoint_step", ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                       ctypes.c_double, ctypes.c_void_p, ctypes.c_void_p,
                                       ctypes.c_void_p, ctypes.c_void_p]),
    ("dg_step_mh", ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                  ctypes.c_double, ctypes.c_void_p, ctypes.c_double,
                                  ctypes.c_void_p, ctypes.c_void_p]),
    ("dg_run", ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int,
                              ctypes.c_double, ctypes.c_void_p, ctypes.c_int,
                              ctypes.POINTER(ctypes.c_void_p), ctypes.POINTER(ctypes.c_void_p),
                              ctypes.c_int, ctypes.c_void_p]),
    ("dg_ninst", ctypes.c_int, [ctypes.c_void_p]),
    ("dg_instance_offsets", ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_int64)]),
    ("dg_set_launch", ctypes.c_int, [ctypes.c_void_p, ctypes.c_int, ctypes.c_int]),
    ("dg_get_launch", ctypes.c_int, [ctypes.c_void_p, ctypes.POINTER(ctypes.c_int),
                                     ctypes.POINTER(ctypes.c_int)]),
    ("dg_cfl_dt", ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_double,
                                 ctypes.c_void_p, ctypes.c_void_p]),
    ("dg_cfl_dt_static", ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_double,
                                        ctypes.c_void_p, ctypes.c_void_p]),
    ("dg_set_tiling", ctypes.c_int, [ctypes.c_void_p, ctypes.c_int]),
    ("dg_get_tiling", ctypes.c_int, [ctypes.c_void_p]),
    ("dg_check", ctypes.c_int, [ctypes.c_void_p]),
    ("dg_set_mesh_motion", ctypes.c_int, [ctypes.c_void_p, ctypes.c_int]),
    ("dg_set_moving_timing", ctypes.c_int, [ctypes.c_void_p, ctypes.c_int]),
    ("dg_moving_timing", ctypes.c_int, [ctypes.c_void_p, _dp, ctypes.POINTER(ctypes.c_int)]),
    ("dg_mesh_geometry", ctypes.c_int, [ctypes.c_void_p, _dp, _dp, _dp,
                                        ctypes.POINTER(ctypes.c_int32),
                                        ctypes.POINTER(ctypes.c_int32)]),
    ("dg_batch_create", ctypes.c_int, [ctypes.POINTER(ctypes.c_void_p), ctypes.c_int,
                                       ctypes.c_char_p, ctypes.POINTER(ctypes.c_void_p)]),
    ("dg_batch_mesh", ctypes.c_void_p, [ctypes.c_void_p]),
    ("dg_batch_offset", ctypes.c_int64, [ctypes.c_void_p, ctypes.c_int]),
    ("dg_batch_run", ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_double,
                                    ctypes.c_void_p, ctypes.c_int, ctypes.c_void_p]),
    ("dg_batch_adjoint_step", ctypes.c_int, [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                             ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]),
    ("dg_batch_destroy", None, [ctypes.c_void_p]),
    ("dg_last_error", ctypes.c_char_p, []),
]


def lib():
    """Load ``libdg.so`` (raises if it is not built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is not built: run __graft_entry__.build() or "
                               "python paper_1305_5536_amd/build.py")
        L = ctypes.CDLL(LIB_PATH)
        for name, res, args in SYMBOLS:
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def last_error() -> str:
    s = lib().dg_last_error()
    return s.decode() if s else ""


def check(status: int, where: str) -> None:
    if status == DG_OK:
        return
    msg = last_error()
    if status == DG_ENONPHYSICAL:
        raise NonPhysicalState(status, where, msg)
    raise DGError(status, where, msg)
