"""ctypes binding of libcellmech.so: argument marshalling only.

Every computation runs in the HIP library.  If the library is not built the
import of this module fails loudly; there is no fallback.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libcellmech.so")

CM_OK, CM_EINVAL, CM_EDEGENERATE, CM_EHIP, CM_ENOMEM, CM_ESTATE = 0, -1, -2, -3, -4, -5
STATUS = {CM_EINVAL: "CM_EINVAL", CM_EDEGENERATE: "CM_EDEGENERATE",
          CM_EHIP: "CM_EHIP", CM_ENOMEM: "CM_ENOMEM", CM_ESTATE: "CM_ESTATE"}
ORDER_INPUT, ORDER_RCM, ORDER_MORTON = 0, 1, 2


class CellmechError(RuntimeError):
    def __init__(self, status: int, message: str):
        self.status = status
        super().__init__(f"{STATUS.get(status, status)}: {message}")


class Options(ctypes.Structure):
    _fields_ = [("order", ctypes.c_int32), ("tile_tets", ctypes.c_int32),
                ("degenerate_tol", ctypes.c_double)]


class Info(ctypes.Structure):
    _fields_ = [("n_cells", ctypes.c_int64), ("n_nodes", ctypes.c_int64),
                ("n_tets", ctypes.c_int64), ("n_tiles", ctypes.c_int64),
                ("n_shared", ctypes.c_int64), ("n_slots", ctypes.c_int64),
                ("n_chunks", ctypes.c_int64),
                ("tile_tets", ctypes.c_int32),
                ("max_tile_nodes", ctypes.c_int32),
                ("device_bytes", ctypes.c_int64), ("volume", ctypes.c_double),
                ("min_v0", ctypes.c_double), ("max_cond", ctypes.c_double),
                ("n_regions", ctypes.c_int32)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


_vp = ctypes.c_void_p
_i32 = ctypes.c_int32
_i64 = ctypes.c_int64
_int = ctypes.c_int
_p64 = ctypes.POINTER(ctypes.c_int64)

# name -> (restype, argtypes); mirrors include/cellmech.h
SIGNATURES = {
    "cm_last_error": (ctypes.c_char_p, []),
    "cm_version": (_int, []),
    "cm_options_default": (None, [ctypes.POINTER(Options)]),
    "cm_batch_create": (_int, [_i32, _vp, _vp, _vp, _vp,
                               ctypes.POINTER(Options), _vp,
                               ctypes.POINTER(_vp)]),
    "cm_mesh_create": (_int, [_i64, _i64, _vp, _vp, ctypes.POINTER(Options),
                              _vp, ctypes.POINTER(_vp)]),
    "cm_template_create": (_int, [_i32, _i64, _i64, _vp, _vp,
                                  ctypes.POINTER(Options), _vp,
                                  ctypes.POINTER(_vp)]),
    "cm_batch_create_regions": (_int, [_i32, _vp, _vp, _vp, _vp, _vp, _i32,
                                       ctypes.POINTER(Options), _vp,
                                       ctypes.POINTER(_vp)]),
    "cm_template_create_regions": (_int, [_i32, _i64, _i64, _vp, _vp, _vp,
                                          _i32, ctypes.POINTER(Options), _vp,
                                          ctypes.POINTER(_vp)]),
    "cm_destroy": (_int, [_vp]),
    "cm_get_info": (_int, [_vp, ctypes.POINTER(Info)]),
    "cm_permutation": (_int, [_vp, _vp]),
    "cm_set_params": (_int, [_vp, _vp, _vp, _vp, _int, _vp]),
    "cm_forces": (_int, [_vp, _vp, _vp, _vp, _vp, _vp]),
    "cm_forces_noalloc": (_int, [_vp, _vp, _vp, _vp, _vp, _vp]),
    "cm_forces_checked": (_int, [_vp, _vp, _vp, _vp, _vp, _vp, _vp]),
    "cm_forces_backward": (_int, [_vp, _vp, _vp, _vp, _vp, _vp, _vp]),
    "cm_forces_and_backward": (_int, [_vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp,
                                      _vp, _vp]),
    "cm_forces_percell": (_int, [_vp, _vp, _vp, _vp, _vp, _vp]),
    "cm_forces_backward_percell": (_int, [_vp, _vp, _vp, _vp, _vp, _vp, _vp]),
    "cm_batch_create_tuned": (_int, [_i32, _vp, _vp, _vp, _vp,
                                     ctypes.POINTER(Options), _vp, _i32,
                                     ctypes.c_char_p, _vp, _vp,
                                     ctypes.POINTER(_vp)]),
    "cm_set_launch": (_int, [_vp, _i32, _i32]),
    "cm_get_launch": (_int, [_vp, ctypes.POINTER(_i32), ctypes.POINTER(_i32)]),
    "cm_autotune": (_int, [_vp, _vp, ctypes.c_char_p, _vp]),
    "cm_graph_capture": (_int, [_vp, _int, _vp, _vp, _vp, _vp, _vp, _vp, _vp,
                                _vp, _vp]),
    "cm_graph_launch": (_int, [_vp, _vp]),
    "cm_stream_copy": (_int, [_vp, _vp, ctypes.c_int64, _vp]),
    "cm_qs_set_indenter": (_int, [_vp, ctypes.c_double, _vp, _vp]),
    "cm_profile_kernels": (_int, [_vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp,
                                  _i32, _vp, _vp]),
    "cm_plate_step": (_int, [_vp, _vp, _vp, _vp, ctypes.c_double,
                             ctypes.c_double, _vp, _vp, _vp]),
    "cm_plate_step_adjoint": (_int, [_vp, _vp, _vp, _vp, _vp,
                                     ctypes.c_double, ctypes.c_double, _vp,
                                     _vp, ctypes.c_double, _vp, _vp, _vp,
                                     _vp]),
    "cm_plate_forces_step": (_int, [_vp, _vp, _vp, ctypes.c_double,
                                    ctypes.c_double, _vp, _vp, _vp, _vp, _vp]),
    "cm_plate_backward_step": (_int, [_vp, _vp, _vp, _vp, ctypes.c_double,
                                      ctypes.c_double, _vp, _vp,
                                      ctypes.c_double, _vp, _vp, _vp]),
    "cm_layout_create": (_int, [_i32, _vp, _vp, _vp, _vp,
                                ctypes.POINTER(Options), ctypes.POINTER(_vp)]),
    "cm_layout_create_template": (_int, [_i32, _i64, _i64, _vp, _vp,
                                         ctypes.POINTER(Options),
                                         ctypes.POINTER(_vp)]),
    "cm_layout_create_regions": (_int, [_i32, _vp, _vp, _vp, _vp, _vp, _i32,
                                        ctypes.POINTER(Options),
                                        ctypes.POINTER(_vp)]),
    "cm_layout_export_regions": (_int, [_vp, _vp, _vp, _vp]),
    "cm_shape": (_int, [_vp, _vp, _vp, _vp, _vp]),
    "cm_forces_backward_cells": (_int, [_vp, _vp, _vp, _vp, _vp, _i64, _vp,
                                        _vp, _vp]),
    "cm_qs_residual": (_int, [_vp, _vp, _vp, _vp, _vp, ctypes.c_double,
                              ctypes.c_double, ctypes.c_double, ctypes.c_double,
                              ctypes.c_double, ctypes.c_double, _i32, _vp, _vp,
                              _vp, _vp, _vp, _vp, _vp, _vp, _vp]),
    "cm_qs_stiffness": (_int, [_vp, _vp, _vp]),
    "cm_qs_adjoint_rhs": (_int, [_vp, _vp, _vp, ctypes.c_double, _vp, _vp,
                                 _vp, _vp, _vp, _vp, _vp]),
    "cm_qs_ls_start": (_int, [_vp, _vp, _vp, ctypes.c_double, _vp, _vp, _vp,
                              _vp]),
    "cm_qs_ls_accept": (_int, [_vp, _vp, _vp, ctypes.c_double, _vp,
                               ctypes.c_double, ctypes.c_double, _vp, _vp, _vp,
                               _vp, _vp, _vp]),
    "cm_qs_noise": (_int, [_vp, _vp, _vp, _vp]),
    "cm_qs_floor": (_int, [_vp, _vp, _vp, ctypes.c_double, _vp, _vp, _vp,
                           _vp]),
    "cm_qs_cg_step": (_int, [_vp, _vp, _vp, ctypes.c_double, ctypes.c_double,
                             _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp]),
    "cm_qs_update": (_int, [_vp, _vp, ctypes.c_double, _vp, _vp, _vp]),
    "cm_qs_cg_iteration": (_int, [_vp, _vp, _vp, ctypes.c_double,
                                  ctypes.c_double, _vp, _vp, _vp, _vp, _vp,
                                  _vp, _vp, _vp]),
    "cm_qs_predict": (_int, [_vp, _vp, _vp, _vp, _vp]),
    "cm_layout_sizes": (_int, [_vp, _p64]),
    "cm_layout_export": (_int, [_vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp,
                                _vp]),
    "cm_layout_destroy": (_int, [_vp]),
}

_lib = None


def lib():
    """The loaded HIP library (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(
                f"{LIB_PATH} is not built: run `python -m "
                "paper_2003_03130_amd.build` (hipcc, gfx950)")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def check(rc: int):
    if rc != CM_OK:
        raise CellmechError(rc, lib().cm_last_error().decode())
