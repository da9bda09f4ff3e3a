"""ctypes loader of the drt3d HIP library (``libdrt3d.so``, built in-tree).

There is no fallback: if the library is missing or fails to load, every entry
point raises. Argument marshalling only; all compute happens in the library.
"""
from __future__ import annotations

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libdrt3d.so")

DRT3D_I32 = 0
DRT3D_F32 = 1
DRT3D_U8 = 2
DRT3D_ALL = 0xFFF
STATUS = {0: "DRT3D_OK", -1: "DRT3D_EINVAL", -2: "DRT3D_ENOMEM", -3: "DRT3D_EHIP", -4: "DRT3D_EUNSUPPORTED"}

# Every symbol declared in include/drt3d.h, with its ctypes signature.
_vp, _sz, _u32, _int = ctypes.c_void_p, ctypes.c_size_t, ctypes.c_uint32, ctypes.c_int
_ptrs = ctypes.POINTER(ctypes.c_void_p)
_ints = ctypes.POINTER(ctypes.c_int)
SIGNATURES = {
    "drt3d_last_error": (ctypes.c_char_p, []),
    "drt3d_abi_version": (_int, []),
    "drt3d_out_elems": (_sz, [_int, _u32]),
    "djt3d_out_elems": (_sz, [_int, _u32]),
    "drt3d_workspace_bytes": (_sz, [_int, _u32, _int]),
    "djt3d_workspace_bytes": (_sz, [_int, _u32, _int]),
    "drt3d_adjoint_workspace_bytes": (_sz, [_int, _u32, _int]),
    "djt3d_adjoint_workspace_bytes": (_sz, [_int, _u32, _int]),
    "drt3d_forward_batched_workspace_bytes": (_sz, [_int, _ints, _u32, _int]),
    "djt3d_forward_batched_workspace_bytes": (_sz, [_int, _ints, _u32, _int]),
    "drt3d_adjoint_batched_workspace_bytes": (_sz, [_int, _ints, _u32, _int]),
    "djt3d_adjoint_batched_workspace_bytes": (_sz, [_int, _ints, _u32, _int]),
    "drt3d_forward": (_int, [_vp, _vp, _int, _u32, _int, _vp, _sz, _vp]),
    "drt3d_forward_noalloc": (_int, [_vp, _vp, _int, _u32, _int, _vp]),
    "djt3d_forward": (_int, [_vp, _vp, _int, _u32, _int, _vp, _sz, _vp]),
    "drt3d_adjoint": (_int, [_vp, _vp, _int, _u32, _int, _vp, _sz, _vp]),
    "djt3d_adjoint": (_int, [_vp, _vp, _int, _u32, _int, _vp, _sz, _vp]),
    "drt3d_forward_batched": (_int, [_int, _ptrs, _ptrs, _ints, _u32, _int, _vp, _sz, _vp]),
    "djt3d_forward_batched": (_int, [_int, _ptrs, _ptrs, _ints, _u32, _int, _vp, _sz, _vp]),
    "drt3d_adjoint_batched": (_int, [_int, _ptrs, _ptrs, _ints, _u32, _int, _vp, _sz, _vp]),
    "djt3d_adjoint_batched": (_int, [_int, _ptrs, _ptrs, _ints, _u32, _int, _vp, _sz, _vp]),
    "drt3d_net_elems": (_sz, [_int]),
    "drt3d_merge_net": (_int, [_vp, _vp, _int, _int, _vp]),
    "drt3d_detect_planes_workspace_bytes": (_sz, [_int, _u32, _int]),
    "drt3d_detect_planes": (_int, [_vp, _int, _u32, _int, ctypes.c_double, ctypes.c_double, _vp, ctypes.c_longlong,
                                   _vp, _vp, _sz, _vp]),
    "drt3d_backproject_bins_workspace_bytes": (_sz, [_int, _u32, _int]),
    "drt3d_backproject_bins": (_int, [_vp, _vp, ctypes.c_longlong, _vp, _int, _u32, _int, _vp, _sz, _vp]),
    "drt3d_plane_normal": (_int, [_int, _int, _int, _int, _ints]),
    "drt3d_inverse_workspace_bytes": (_sz, [_int]),
    "drt3d_inverse": (_int, [_vp, _vp, _int, _int, ctypes.POINTER(ctypes.c_double), _vp, _sz, _vp]),
    "drt3d_inverse_lambdas": (_int, [_int, ctypes.POINTER(ctypes.c_double), _vp, _sz, _vp]),
    "drt3d_autotune": (_int, [_int, _int, _vp, _vp, _vp, _sz, _vp]),
    "drt3d_tuning_string": (ctypes.c_char_p, [_int, _int]),
    "drt3d_set_tuning": (_int, [_int, _int, ctypes.c_char_p]),
    "drt3d_profile_enable": (_int, [_int]),
    "drt3d_profile_reset": (_int, []),
    "drt3d_pass_times": (_int, [ctypes.c_char_p, ctypes.POINTER(ctypes.c_double),
                                ctypes.POINTER(ctypes.c_longlong), ctypes.POINTER(ctypes.c_double), _int]),
    "drt3d_stream_probe": (_int, [_vp, _sz, _vp, _sz, _vp]),
    "drt3d_frame_map": (_int, [_int, _int, _int, _ints]),
    "drt3d_plan_create": (_int, [_ptrs, _int, _int, _u32, _int]),
    "drt3d_plan_workspace_bytes": (_sz, [_vp]),
    "drt3d_plan_execute": (_int, [_vp, _vp, _vp, _vp, _sz, _vp]),
    "drt3d_plan_destroy": (_int, [_vp]),
    "drt3d_plan_text": (_int, [_int, _int, _u32, _int, ctypes.c_char_p, _sz]),
}

_lib = None


class Drt3dError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__("%s (%d): %s" % (STATUS.get(status, "?"), status, message))
        self.status = status


def lib() -> ctypes.CDLL:
    """The loaded library; raises if it was not built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError("libdrt3d.so is not built (run __graft_entry__.build()); "
                              "there is no fallback implementation")
        handle = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            f = getattr(handle, name)
            f.restype = res
            f.argtypes = args
        _lib = handle
    return _lib


def check(status: int) -> None:
    if status != 0:
        msg = lib().drt3d_last_error()
        raise Drt3dError(status, msg.decode() if msg else "")
