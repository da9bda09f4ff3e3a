"""ctypes wrapper of the C oracle in ``drt3d_oracle.c`` (test infrastructure only).

Every function here returns exact results: int64 for int32 inputs, float64 for
floating inputs (the input is widened to float64 before the transform). The
``def_*`` functions evaluate the paper's definitions (Sec. 3.1 eq. (9), Sec. 4.1
eq. (13), and the transpose of eq. (9) for the adjoint, Sec. 5.1); the ``rec_*``
functions run the paper's recursions naively (Algorithm 1 with eq. (11),
Algorithm 3 with eq. (15), Algorithm 1 reversed with eq. (17)). Index and frame
conventions are stated in the header of the C file.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import threading

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "drt3d_oracle.c")
_LIB = os.path.join(_HERE, "liboracle.so")
_lock = threading.Lock()
_lib = None

__all__ = [
    "build", "line", "line_recursive", "frame_to_orig", "frame_matrix", "in_order_row",
    "drt_point", "djt_point", "adj_point", "djt_adj_point",
    "def_drt", "def_djt", "def_adj", "def_djt_adj",
    "rec_drt", "rec_djt", "rec_adj",
    "wrap_int32", "count_dodecants",
]


def build(force: bool = False) -> str:
    """Compile the oracle with gcc (plain C, -O2). Returns the library path."""
    if force or not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
        tmp = _LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-shared", "-fPIC", "-o", tmp, _SRC])
        os.replace(tmp, _LIB)
    return _LIB


def _load():
    global _lib
    with _lock:
        if _lib is not None:
            return _lib
        lib = ctypes.CDLL(build())
        i32p = np.ctypeslib.ndpointer(np.int32, flags="C_CONTIGUOUS")
        i64p = np.ctypeslib.ndpointer(np.int64, flags="C_CONTIGUOUS")
        f64p = np.ctypeslib.ndpointer(np.float64, flags="C_CONTIGUOUS")
        ip = ctypes.POINTER(ctypes.c_int)
        c_int, c_uint = ctypes.c_int, ctypes.c_uint
        lib.orc_line.argtypes = [c_int, c_int, c_int]
        lib.orc_line.restype = c_int
        lib.orc_line_recursive.argtypes = [c_int, c_int, c_int]
        lib.orc_line_recursive.restype = c_int
        lib.orc_frame_to_orig.argtypes = [c_int, c_int, ip, ip]
        lib.orc_frame_to_orig.restype = None
        lib.orc_in_order_row.argtypes = [c_int, ip]
        lib.orc_in_order_row.restype = None
        lib.orc_frame_matrix.argtypes = [c_int, ip]
        lib.orc_frame_matrix.restype = None
        for suf, inp, acc, accty in (("i", i32p, i64p, ctypes.c_int64), ("f", f64p, f64p, ctypes.c_double)):
            f = getattr(lib, "orc_drt_point_" + suf)
            f.argtypes = [inp, c_int, c_int, c_int, c_int, c_int]
            f.restype = accty
            f = getattr(lib, "orc_djt_point_" + suf)
            f.argtypes = [inp, c_int, c_int, c_int, c_int, c_int, c_int]
            f.restype = accty
            for name in ("adj_point", "djt_adj_point"):
                f = getattr(lib, "orc_%s_%s" % (name, suf))
                f.argtypes = [inp, c_int, c_uint, c_int, c_int, c_int]
                f.restype = accty
            for name in ("drt_def", "djt_def", "adj_def", "djt_adj_def", "drt_rec", "djt_rec", "adj_rec"):
                f = getattr(lib, "orc_%s_%s" % (name, suf))
                f.argtypes = [inp, c_int, c_uint, acc]
                f.restype = c_int
        _lib = lib
        return lib


def count_dodecants(mask: int) -> int:
    return bin(mask & 0xFFF).count("1")


def wrap_int32(a: np.ndarray) -> np.ndarray:
    """Narrow exact int64 results to int32 with two's-complement wrap."""
    return np.asarray(a, dtype=np.int64).astype(np.int32)


def _prep(vol):
    vol = np.asarray(vol)
    if np.issubdtype(vol.dtype, np.integer):
        return np.ascontiguousarray(vol, dtype=np.int32), "i", np.int64
    return np.ascontiguousarray(vol, dtype=np.float64), "f", np.float64


def _N(vol):
    N = vol.shape[0]
    if vol.ndim != 3 or vol.shape != (N, N, N) or N < 2 or N & (N - 1):
        raise ValueError("expected an N x N x N cube with N a power of two >= 2")
    return N


def line(n: int, s: int, x: int) -> int:
    """l^n_s(x), eq. (4) closed form."""
    return _load().orc_line(n, s, x)


def line_recursive(n: int, s: int, x: int) -> int:
    """l^n_s(x), eq. (4) recursive form."""
    return _load().orc_line_recursive(n, s, x)


def frame_to_orig(k: int, N: int, primed) -> tuple:
    p = (ctypes.c_int * 3)(*[int(v) for v in primed])
    o = (ctypes.c_int * 3)()
    _load().orc_frame_to_orig(k, N, p, o)
    return tuple(o)


def in_order_row(k: int) -> tuple:
    """Row k of Algorithm 2's InOrder table as the oracle holds it."""
    r = (ctypes.c_int * 3)()
    _load().orc_in_order_row(k, r)
    return tuple(r)


def frame_matrix(k: int) -> np.ndarray:
    """Signed permutation M with primed = M @ orig + offset."""
    m = (ctypes.c_int * 9)()
    _load().orc_frame_matrix(k, m)
    return np.array(list(m), dtype=np.int64).reshape(3, 3)


def drt_point(vol, k, s1, s2, dd):
    v, suf, _ = _prep(vol)
    return getattr(_load(), "orc_drt_point_" + suf)(v, _N(v), k, s1, s2, dd)


def djt_point(vol, k, s1, s2, e1, e2):
    v, suf, _ = _prep(vol)
    return getattr(_load(), "orc_djt_point_" + suf)(v, _N(v), k, s1, s2, e1, e2)


def adj_point(proj, N, mask, x, y, z):
    p, suf, _ = _prep(proj)
    if p.size != count_dodecants(mask) * N * N * (3 * N - 2):
        raise ValueError("projection size does not match N and mask")
    return getattr(_load(), "orc_adj_point_" + suf)(p.reshape(-1), N, mask, x, y, z)


def djt_adj_point(proj, N, mask, x, y, z):
    """Transpose of eq. (13) at one voxel."""
    p, suf, _ = _prep(proj)
    if p.size != count_dodecants(mask) * N * N * (2 * N - 1) ** 2:
        raise ValueError("projection size does not match N and mask")
    return getattr(_load(), "orc_djt_adj_point_" + suf)(p.reshape(-1), N, mask, x, y, z)


def _run(name, inp, N, mask, out_shape):
    v, suf, accdt = _prep(inp)
    out = np.zeros(out_shape, dtype=accdt)
    rc = getattr(_load(), "orc_%s_%s" % (name, suf))(v.reshape(-1) if v.ndim != 3 else v, N, mask, out)
    if rc != 0:
        raise MemoryError("oracle %s failed with code %d" % (name, rc))
    return out


def _drt_shape(N, mask):
    return (count_dodecants(mask), N, N, 3 * N - 2)


def _djt_shape(N, mask):
    return (count_dodecants(mask), N, N, 2 * N - 1, 2 * N - 1)


def def_drt(vol, mask=0xFFF):
    """eq. (9) by scatter over voxels; [popcount][N][N][3N-2]."""
    N = _N(np.asarray(vol))
    return _run("drt_def", vol, N, mask, _drt_shape(N, mask))


def def_djt(vol, mask=0xFFF):
    """eq. (13) by scatter over voxels; [popcount][N][N][2N-1][2N-1]."""
    N = _N(np.asarray(vol))
    return _run("djt_def", vol, N, mask, _djt_shape(N, mask))


def def_adj(proj, N, mask=0xFFF):
    """Transpose of eq. (9), gathered per voxel; [N][N][N]."""
    proj = np.asarray(proj)
    if proj.shape != _drt_shape(N, mask):
        raise ValueError("projection shape %s != %s" % (proj.shape, _drt_shape(N, mask)))
    return _run("adj_def", proj, N, mask, (N, N, N))


def def_djt_adj(proj, N, mask=0xFFF):
    """Transpose of eq. (13), gathered per voxel; [N][N][N]."""
    proj = np.asarray(proj)
    if proj.shape != _djt_shape(N, mask):
        raise ValueError("projection shape %s != %s" % (proj.shape, _djt_shape(N, mask)))
    return _run("djt_adj_def", proj, N, mask, (N, N, N))


def rec_drt(vol, mask=0xFFF):
    """Algorithm 1 (eq. (11)) per dodecant, naive; [popcount][N][N][3N-2]."""
    N = _N(np.asarray(vol))
    return _run("drt_rec", vol, N, mask, _drt_shape(N, mask))


def rec_djt(vol, mask=0xFFF):
    """Algorithm 3 (eq. (15)) per dodecant, naive; [popcount][N][N][2N-1][2N-1]."""
    N = _N(np.asarray(vol))
    return _run("djt_rec", vol, N, mask, _djt_shape(N, mask))


def rec_adj(proj, N, mask=0xFFF):
    """Algorithm 1 reversed with eq. (17); [N][N][N]."""
    proj = np.asarray(proj)
    if proj.shape != _drt_shape(N, mask):
        raise ValueError("projection shape %s != %s" % (proj.shape, _drt_shape(N, mask)))
    return _run("adj_rec", proj, N, mask, (N, N, N))
