"""Python binding of the drt3d C ABI (include/drt3d.h) over torch tensors.

PyTorch provides device memory and the current stream; every step of every
transform runs in the HIP library. Function names follow the C entry points.
Conventions (frames, output layouts, arithmetic) are those of the header.
"""
from __future__ import annotations

import ctypes
from typing import List, Optional, Sequence

import torch

from ._lib import DRT3D_ALL, DRT3D_F32, DRT3D_I32, DRT3D_U8, check, lib

__all__ = [
    "DRT3D_ALL", "drt3d_forward", "djt3d_forward", "drt3d_adjoint", "djt3d_adjoint",
    "drt3d_forward_batched", "djt3d_forward_batched", "drt3d_adjoint_batched", "djt3d_adjoint_batched",
    "drt3d_inverse", "drt3d_inverse_lambdas", "drt3d_merge_net",
    "drt3d_detect_planes", "drt3d_backproject_bins", "drt3d_plane_normal",
    "drt3d_out_shape", "djt3d_out_shape", "drt3d_autotune", "drt3d_tuning_string",
    "drt3d_set_tuning", "profile", "dodecant_count",
]


def dodecant_count(mask: int) -> int:
    return bin(int(mask) & 0xFFF).count("1")


def drt3d_out_shape(N: int, mask: int = DRT3D_ALL):
    return (dodecant_count(mask), N, N, 3 * N - 2)


def djt3d_out_shape(N: int, mask: int = DRT3D_ALL):
    return (dodecant_count(mask), N, N, 2 * N - 1, 2 * N - 1)


def _dtype_code(t: torch.Tensor) -> int:
    if t.dtype == torch.int32:
        return DRT3D_I32
    if t.dtype == torch.float32:
        return DRT3D_F32
    raise TypeError("drt3d supports int32 and float32 tensors, got %s" % t.dtype)


def _cube(vol: torch.Tensor) -> int:
    if vol.dim() != 3 or not (vol.shape[0] == vol.shape[1] == vol.shape[2]):
        raise ValueError("expected an N x N x N tensor, got %s" % (tuple(vol.shape),))
    if not vol.is_cuda:
        raise ValueError("drt3d runs on the GPU; move the tensor to a HIP device first")
    if not vol.is_contiguous():
        raise ValueError("the volume must be contiguous ([x][y][z], z fastest)")
    return int(vol.shape[0])


def _stream(stream) -> ctypes.c_void_p:
    s = torch.cuda.current_stream() if stream is None else stream
    return ctypes.c_void_p(s.cuda_stream)


def _workspace(nbytes: int, device, workspace: Optional[torch.Tensor]) -> torch.Tensor:
    if workspace is not None:
        if workspace.numel() * workspace.element_size() < nbytes:
            raise ValueError("workspace too small: %d < %d bytes" % (workspace.numel() * workspace.element_size(), nbytes))
        return workspace
    return torch.empty(max(nbytes, 256), dtype=torch.uint8, device=device)


def _ptr(t: torch.Tensor) -> ctypes.c_void_p:
    return ctypes.c_void_p(t.data_ptr())


def drt3d_forward(vol: torch.Tensor, mask: int = DRT3D_ALL, out: Optional[torch.Tensor] = None,
                  workspace: Optional[torch.Tensor] = None, stream=None) -> torch.Tensor:
    """3D DRT of planes over the dodecants of `mask`: [popcount][N][N][3N-2].

    A uint8 volume gives the int32 result of the same values, computed with
    narrow storage in HBM (N >= 32)."""
    N = _cube(vol)
    if vol.dtype == torch.uint8:
        dt, odt = DRT3D_U8, torch.int32
    else:
        dt, odt = _dtype_code(vol), vol.dtype
    shape = drt3d_out_shape(N, mask)
    if out is None:
        out = torch.empty(shape, dtype=odt, device=vol.device)
    elif tuple(out.shape) != shape or out.dtype != odt or not out.is_contiguous():
        raise ValueError("out must be a contiguous %s tensor of shape %s" % (odt, shape))
    need = lib().drt3d_workspace_bytes(N, mask, dt)
    ws = _workspace(need, vol.device, workspace)
    check(lib().drt3d_forward(_ptr(vol), _ptr(out), N, mask, dt, _ptr(ws), ws.numel() * ws.element_size(),
                              _stream(stream)))
    return out


def djt3d_forward(vol: torch.Tensor, mask: int = DRT3D_ALL, out: Optional[torch.Tensor] = None,
                  workspace: Optional[torch.Tensor] = None, stream=None) -> torch.Tensor:
    """3D DJT of lines over the dodecants of `mask`: [popcount][N][N][2N-1][2N-1]."""
    N = _cube(vol)
    dt = _dtype_code(vol)
    shape = djt3d_out_shape(N, mask)
    if out is None:
        out = torch.empty(shape, dtype=vol.dtype, device=vol.device)
    elif tuple(out.shape) != shape or out.dtype != vol.dtype or not out.is_contiguous():
        raise ValueError("out must be a contiguous %s tensor of shape %s" % (vol.dtype, shape))
    need = lib().djt3d_workspace_bytes(N, mask, dt)
    ws = _workspace(need, vol.device, workspace)
    check(lib().djt3d_forward(_ptr(vol), _ptr(out), N, mask, dt, _ptr(ws), ws.numel() * ws.element_size(),
                              _stream(stream)))
    return out


def drt3d_adjoint(proj: torch.Tensor, mask: int = DRT3D_ALL, out: Optional[torch.Tensor] = None,
                  workspace: Optional[torch.Tensor] = None, stream=None) -> torch.Tensor:
    """Backprojection (exact transpose of drt3d_forward): [N][N][N]."""
    if proj.dim() != 4 or proj.shape[0] != dodecant_count(mask):
        raise ValueError("proj must be [popcount(mask)][N][N][3N-2]")
    N = int(proj.shape[1])
    if tuple(proj.shape) != drt3d_out_shape(N, mask) or not proj.is_cuda or not proj.is_contiguous():
        raise ValueError("proj must be a contiguous device tensor of shape %s" % (drt3d_out_shape(N, mask),))
    dt = _dtype_code(proj)
    if out is None:
        out = torch.empty((N, N, N), dtype=proj.dtype, device=proj.device)
    need = lib().drt3d_adjoint_workspace_bytes(N, mask, dt)
    ws = _workspace(need, proj.device, workspace)
    check(lib().drt3d_adjoint(_ptr(proj), _ptr(out), N, mask, dt, _ptr(ws), ws.numel() * ws.element_size(),
                              _stream(stream)))
    return out


def djt3d_adjoint(proj: torch.Tensor, mask: int = DRT3D_ALL, out: Optional[torch.Tensor] = None,
                  workspace: Optional[torch.Tensor] = None, stream=None) -> torch.Tensor:
    """Exact transpose of djt3d_forward: [N][N][N]."""
    if proj.dim() != 5 or proj.shape[0] != dodecant_count(mask):
        raise ValueError("proj must be [popcount(mask)][N][N][2N-1][2N-1]")
    N = int(proj.shape[1])
    if tuple(proj.shape) != djt3d_out_shape(N, mask) or not proj.is_cuda or not proj.is_contiguous():
        raise ValueError("proj must be a contiguous device tensor of shape %s" % (djt3d_out_shape(N, mask),))
    dt = _dtype_code(proj)
    if out is None:
        out = torch.empty((N, N, N), dtype=proj.dtype, device=proj.device)
    elif tuple(out.shape) != (N, N, N) or out.dtype != proj.dtype or not out.is_contiguous():
        raise ValueError("out must be a contiguous %s tensor of shape %s" % (proj.dtype, (N, N, N)))
    need = lib().djt3d_adjoint_workspace_bytes(N, mask, dt)
    ws = _workspace(need, proj.device, workspace)
    check(lib().djt3d_adjoint(_ptr(proj), _ptr(out), N, mask, dt, _ptr(ws), ws.numel() * ws.element_size(),
                              _stream(stream)))
    return out


def _batched(fn_name: str, ws_name: str, ins: Sequence[torch.Tensor], outs: Sequence[torch.Tensor],
             Ns: Sequence[int], mask: int, dt: int, device, workspace, stream):
    count = len(ins)
    a_in = (ctypes.c_void_p * count)(*[t.data_ptr() for t in ins])
    a_out = (ctypes.c_void_p * count)(*[t.data_ptr() for t in outs])
    a_N = (ctypes.c_int * count)(*Ns)
    need = getattr(lib(), ws_name)(count, a_N, mask, dt)
    if need == 0:
        raise ValueError("invalid batched arguments")
    ws = _workspace(need, device, workspace)
    check(getattr(lib(), fn_name)(count, a_in, a_out, a_N, mask, dt, _ptr(ws), ws.numel() * ws.element_size(),
                                  _stream(stream)))


def drt3d_forward_batched(vols: Sequence[torch.Tensor], mask: int = DRT3D_ALL,
                          outs: Optional[Sequence[torch.Tensor]] = None,
                          workspace: Optional[torch.Tensor] = None, stream=None) -> List[torch.Tensor]:
    """DRT of many cubes (mixed N, same dtype) in one set of persistent launches."""
    if not vols:
        return []
    Ns = [_cube(v) for v in vols]
    dt = _dtype_code(vols[0])
    if any(v.dtype != vols[0].dtype for v in vols):
        raise TypeError("all volumes must share one dtype")
    if outs is None:
        outs = [torch.empty(drt3d_out_shape(N, mask), dtype=vols[0].dtype, device=vols[0].device) for N in Ns]
    _batched("drt3d_forward_batched", "drt3d_forward_batched_workspace_bytes", vols, outs, Ns, mask, dt,
             vols[0].device, workspace, stream)
    return list(outs)


def djt3d_forward_batched(vols: Sequence[torch.Tensor], mask: int = DRT3D_ALL,
                          outs: Optional[Sequence[torch.Tensor]] = None,
                          workspace: Optional[torch.Tensor] = None, stream=None) -> List[torch.Tensor]:
    if not vols:
        return []
    Ns = [_cube(v) for v in vols]
    dt = _dtype_code(vols[0])
    if outs is None:
        outs = [torch.empty(djt3d_out_shape(N, mask), dtype=vols[0].dtype, device=vols[0].device) for N in Ns]
    _batched("djt3d_forward_batched", "djt3d_forward_batched_workspace_bytes", vols, outs, Ns, mask, dt,
             vols[0].device, workspace, stream)
    return list(outs)


def drt3d_adjoint_batched(projs: Sequence[torch.Tensor], mask: int = DRT3D_ALL,
                          outs: Optional[Sequence[torch.Tensor]] = None,
                          workspace: Optional[torch.Tensor] = None, stream=None) -> List[torch.Tensor]:
    if not projs:
        return []
    Ns = []
    for p in projs:
        N = int(p.shape[1])
        if tuple(p.shape) != drt3d_out_shape(N, mask) or not p.is_contiguous() or not p.is_cuda:
            raise ValueError("each projection must be a contiguous device tensor [popcount][N][N][3N-2]")
        Ns.append(N)
    dt = _dtype_code(projs[0])
    if outs is None:
        outs = [torch.empty((N, N, N), dtype=projs[0].dtype, device=projs[0].device) for N in Ns]
    _batched("drt3d_adjoint_batched", "drt3d_adjoint_batched_workspace_bytes", projs, outs, Ns, mask, dt,
             projs[0].device, workspace, stream)
    return list(outs)


def djt3d_adjoint_batched(projs: Sequence[torch.Tensor], mask: int = DRT3D_ALL,
                          outs: Optional[Sequence[torch.Tensor]] = None,
                          workspace: Optional[torch.Tensor] = None, stream=None) -> List[torch.Tensor]:
    if not projs:
        return []
    Ns = []
    for p in projs:
        N = int(p.shape[1])
        if tuple(p.shape) != djt3d_out_shape(N, mask) or not p.is_contiguous() or not p.is_cuda:
            raise ValueError("each projection must be a contiguous device tensor [popcount][N][N][2N-1][2N-1]")
        Ns.append(N)
    dt = _dtype_code(projs[0])
    if outs is None:
        outs = [torch.empty((N, N, N), dtype=projs[0].dtype, device=projs[0].device) for N in Ns]
    _batched("djt3d_adjoint_batched", "djt3d_adjoint_batched_workspace_bytes", projs, outs, Ns, mask, dt,
             projs[0].device, workspace, stream)
    return list(outs)


def drt3d_merge_net(proj: torch.Tensor, out: Optional[torch.Tensor] = None, stream=None) -> torch.Tensor:
    """Algorithm 2's merged output: the 12-dodecant DRT rotated and placed in a
    [4N][4N][3N-2] net (the four corner blocks zero)."""
    if proj.dim() != 4:
        raise ValueError("proj must be [12][N][N][3N-2]")
    N = int(proj.shape[1])
    if tuple(proj.shape) != drt3d_out_shape(N) or not proj.is_cuda or not proj.is_contiguous():
        raise ValueError("proj must be a contiguous 12-dodecant device tensor of shape %s" % (drt3d_out_shape(N),))
    dt = _dtype_code(proj)
    shape = (4 * N, 4 * N, 3 * N - 2)
    if out is None:
        out = torch.empty(shape, dtype=proj.dtype, device=proj.device)
    elif tuple(out.shape) != shape or out.dtype != proj.dtype or not out.is_contiguous():
        raise ValueError("out must be a contiguous %s tensor of shape %s" % (proj.dtype, shape))
    check(lib().drt3d_merge_net(_ptr(proj), _ptr(out), N, dt, _stream(stream)))
    return out


def _proj_N(proj: torch.Tensor, mask: int) -> int:
    if proj.dim() != 4:
        raise ValueError("proj must be [count][N][N][3N-2]")
    N = int(proj.shape[1])
    if tuple(proj.shape) != drt3d_out_shape(N, mask) or not proj.is_cuda or not proj.is_contiguous():
        raise ValueError("proj must be a contiguous device tensor of shape %s" % (drt3d_out_shape(N, mask),))
    return N


def drt3d_detect_planes(proj: torch.Tensor, cos_tol: float = 0.05, rel_threshold: float = 0.5,
                        mask: int = DRT3D_ALL, cap: int = 4096, workspace: Optional[torch.Tensor] = None,
                        stream=None):
    """Plane detection in a DRT output (Sec. 6.1): returns (bins, count), bins
    an int64 device tensor of flat output indices (the dominant plane first,
    then the qualifying planes in ascending order, at most cap of them) and
    count the number found (which may exceed cap). Reads count back, so the
    call waits for the stream."""
    N = _proj_N(proj, mask)
    dt = _dtype_code(proj)
    ws = _workspace(lib().drt3d_detect_planes_workspace_bytes(N, mask, dt), proj.device, workspace)
    bins = torch.empty(max(1, int(cap)), dtype=torch.int64, device=proj.device)
    count = torch.empty(1, dtype=torch.int64, device=proj.device)
    check(lib().drt3d_detect_planes(_ptr(proj), N, mask, dt, float(cos_tol), float(rel_threshold), _ptr(bins),
                                    bins.numel(), _ptr(count), _ptr(ws), ws.numel() * ws.element_size(),
                                    _stream(stream)))
    n = int(count.item())
    return bins[:min(n, bins.numel())], n


def drt3d_backproject_bins(bins: torch.Tensor, N: int, mask: int = DRT3D_ALL, dtype=torch.int32,
                           out: Optional[torch.Tensor] = None, workspace: Optional[torch.Tensor] = None,
                           stream=None) -> torch.Tensor:
    """Per voxel, the number of listed planes through it: the adjoint of the
    0/1 projection marking the flat indices in bins (int64 device tensor)."""
    if bins.dtype != torch.int64 or not bins.is_cuda or bins.dim() != 1 or not bins.is_contiguous():
        raise ValueError("bins must be a contiguous 1-D int64 device tensor")
    dt = DRT3D_F32 if dtype == torch.float32 else DRT3D_I32
    if out is None:
        out = torch.empty((N, N, N), dtype=dtype, device=bins.device)
    elif tuple(out.shape) != (N, N, N) or out.dtype != dtype or not out.is_contiguous():
        raise ValueError("out must be a contiguous %s tensor of shape %s" % (dtype, (N, N, N)))
    ws = _workspace(lib().drt3d_backproject_bins_workspace_bytes(N, mask, dt), bins.device, workspace)
    count = torch.full((1,), bins.numel(), dtype=torch.int64, device=bins.device)
    if bins.numel() == 0:  # no planes: a valid pointer, nothing read
        bins = torch.zeros(1, dtype=torch.int64, device=bins.device)
    check(lib().drt3d_backproject_bins(_ptr(bins), _ptr(count), bins.numel(), _ptr(out), N, mask, dt,
                                       _ptr(ws), ws.numel() * ws.element_size(), _stream(stream)))
    return out


def drt3d_plane_normal(k: int, s1: int, s2: int, N: int):
    """Integer normal (x, y, z) of dodecant k's planes at slopes (s1, s2), scaled by N-1."""
    arr = (ctypes.c_int * 3)()
    check(lib().drt3d_plane_normal(k, s1, s2, N, arr))
    return tuple(arr)


def _inverse_workspace(N: int, device, workspace):
    need = lib().drt3d_inverse_workspace_bytes(N)
    if need == 0:
        raise ValueError("the inverse takes N a power of two >= 2, got %d" % N)
    return _workspace(need, device, workspace)


def drt3d_inverse(proj: torch.Tensor, cycles: int = 10, lams: Optional[Sequence[float]] = None,
                  out: Optional[torch.Tensor] = None, workspace: Optional[torch.Tensor] = None,
                  stream=None) -> torch.Tensor:
    """Iterative inverse (Sec. 5.2) of a 12-dodecant float32 DRT: [N][N][N].

    lams: the eigenvalues for sizes 2, 4, ..., N (as drt3d_inverse_lambdas
    returns them), or None to let the library compute and cache them."""
    if proj.dim() != 4 or proj.dtype != torch.float32:
        raise ValueError("proj must be a float32 [12][N][N][3N-2] tensor")
    N = int(proj.shape[1])
    if tuple(proj.shape) != drt3d_out_shape(N) or not proj.is_cuda or not proj.is_contiguous():
        raise ValueError("proj must be a contiguous device tensor of shape %s" % (drt3d_out_shape(N),))
    if out is None:
        out = torch.empty((N, N, N), dtype=torch.float32, device=proj.device)
    elif tuple(out.shape) != (N, N, N) or out.dtype != torch.float32 or not out.is_contiguous():
        raise ValueError("out must be a contiguous float32 tensor of shape %s" % ((N, N, N),))
    ws = _inverse_workspace(N, proj.device, workspace)
    n = N.bit_length() - 1
    arr = None
    if lams is not None:
        if len(lams) != n:
            raise ValueError("lams needs %d values (sizes 2 .. %d)" % (n, N))
        arr = (ctypes.c_double * n)(*[float(v) for v in lams])
    check(lib().drt3d_inverse(_ptr(proj), _ptr(out), N, int(cycles), arr, _ptr(ws), ws.numel() * ws.element_size(),
                              _stream(stream)))
    return out


def drt3d_inverse_lambdas(N: int, device="cuda", workspace: Optional[torch.Tensor] = None, stream=None) -> List[float]:
    """The smoother's eigenvalues for sizes 2, 4, ..., N (computed once per size)."""
    ws = _inverse_workspace(N, device, workspace)
    n = N.bit_length() - 1
    arr = (ctypes.c_double * n)()
    check(lib().drt3d_inverse_lambdas(N, arr, _ptr(ws), ws.numel() * ws.element_size(), _stream(stream)))
    return list(arr)


def drt3d_autotune(N: int, dtype=torch.float32, device="cuda") -> str:
    """Time the tuning candidates of size class N on the GPU; returns the choice."""
    dt = DRT3D_F32 if dtype == torch.float32 else DRT3D_I32
    vol = (torch.randn((N, N, N), device=device) if dt == DRT3D_F32
           else torch.randint(0, 255, (N, N, N), device=device, dtype=torch.int32))
    out = torch.empty(drt3d_out_shape(N, DRT3D_ALL), dtype=vol.dtype, device=device)
    need = lib().drt3d_workspace_bytes(N, DRT3D_ALL, dt)
    ws = torch.empty(need, dtype=torch.uint8, device=device)
    check(lib().drt3d_autotune(N, dt, _ptr(vol), _ptr(out), _ptr(ws), need, _stream(None)))
    torch.cuda.synchronize()
    return drt3d_tuning_string(N, dtype)


def drt3d_tuning_string(N: int, dtype=torch.float32) -> str:
    dt = DRT3D_F32 if dtype == torch.float32 else DRT3D_I32
    return lib().drt3d_tuning_string(N, dt).decode()


def drt3d_set_tuning(N: int, text: str, dtype=torch.float32) -> None:
    dt = DRT3D_F32 if dtype == torch.float32 else DRT3D_I32
    check(lib().drt3d_set_tuning(N, dt, text.encode()))


class profile:
    """Context manager collecting per-kernel HIP-event times of library launches.

    ``with profile() as p: ...`` then ``p.records`` maps kernel name to
    (milliseconds, launches, algorithmic bytes)."""

    def __enter__(self):
        check(lib().drt3d_profile_reset())
        check(lib().drt3d_profile_enable(1))
        self.records = {}
        return self

    def __exit__(self, *exc):
        check(lib().drt3d_profile_enable(0))
        cap = 64
        names = ctypes.create_string_buffer(32 * cap)
        ms = (ctypes.c_double * cap)()
        cnt = (ctypes.c_longlong * cap)()
        by = (ctypes.c_double * cap)()
        n = lib().drt3d_pass_times(names, ms, cnt, by, cap)
        if n < 0:
            check(n)
        for i in range(min(n, cap)):
            name = names.raw[32 * i:32 * i + 32].split(b"\0", 1)[0].decode()
            self.records[name] = (ms[i], int(cnt[i]), by[i])
        return False
