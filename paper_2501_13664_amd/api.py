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
    "drt3d_set_tuning", "profile", "dodecant_count", "drt3d_forward_noalloc", "stream_probe", "Plan",
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


class _on_stream:
    """Makes `stream` (if given) current for the body, so that every tensor the
    wrapper allocates (outputs, workspace) belongs to the stream the library
    runs on and the caching allocator does not hand the workspace out again
    while the library's kernels still use it."""

    def __init__(self, stream):
        self.ctx = torch.cuda.stream(stream) if stream is not None else None

    def __enter__(self):
        if self.ctx is not None:
            self.ctx.__enter__()
        return self

    def __exit__(self, *exc):
        if self.ctx is not None:
            self.ctx.__exit__(*exc)
        return False


def _resolve(device) -> torch.device:
    """`device` with its index filled in ("cuda" means the current device)."""
    d = torch.device(device)
    if d.type == "cuda" and d.index is None:
        d = torch.device("cuda", torch.cuda.current_device())
    return d


def _check_out(out: torch.Tensor, shape, dtype, device, what: str = "out") -> None:
    """A caller-supplied output must match exactly: the C ABI takes no output
    size, so a wrong shape, dtype or layout would be an out-of-bounds write."""
    if (tuple(out.shape) != tuple(shape) or out.dtype != dtype or not out.is_contiguous() or not out.is_cuda
            or out.device != _resolve(device)):
        raise ValueError("%s must be a contiguous %s tensor of shape %s on %s, got %s %s%s on %s"
                         % (what, dtype, tuple(shape), device, out.dtype, tuple(out.shape),
                            "" if out.is_contiguous() else " (non-contiguous)", out.device))


def _workspace(nbytes: int, device, workspace: Optional[torch.Tensor]) -> torch.Tensor:
    if workspace is not None:
        if not workspace.is_cuda or not workspace.is_contiguous() or workspace.device != _resolve(device):
            raise ValueError("workspace must be a contiguous tensor on %s" % (device,))
        if workspace.numel() * workspace.element_size() < nbytes:
            raise ValueError("workspace too small: %d < %d bytes" % (workspace.numel() * workspace.element_size(), nbytes))
        return workspace
    return torch.empty(max(nbytes, 256), dtype=torch.uint8, device=device)


def _ptr(t: torch.Tensor) -> ctypes.c_void_p:
    return ctypes.c_void_p(t.data_ptr())


def _ws_bytes(ws: torch.Tensor) -> int:
    return ws.numel() * ws.element_size()


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
    with _on_stream(stream):
        if out is None:
            out = torch.empty(shape, dtype=odt, device=vol.device)
        else:
            _check_out(out, shape, odt, vol.device)
        ws = _workspace(lib().drt3d_workspace_bytes(N, mask, dt), vol.device, workspace)
        check(lib().drt3d_forward(_ptr(vol), _ptr(out), N, mask, dt, _ptr(ws), _ws_bytes(ws), _stream(stream)))
    return out


def drt3d_forward_noalloc(vol: torch.Tensor, mask: int = DRT3D_ALL, out: Optional[torch.Tensor] = None,
                          stream=None) -> torch.Tensor:
    """drt3d_forward in the library's static scratch: the library call itself
    allocates no device memory (N <= 64 for all 12 dodecants). Calls that
    overlap in time on one GPU race on that scratch; order them on one stream."""
    N = _cube(vol)
    if vol.dtype == torch.uint8:
        dt, odt = DRT3D_U8, torch.int32
    else:
        dt, odt = _dtype_code(vol), vol.dtype
    shape = drt3d_out_shape(N, mask)
    with _on_stream(stream):
        if out is None:
            out = torch.empty(shape, dtype=odt, device=vol.device)
        else:
            _check_out(out, shape, odt, vol.device)
        check(lib().drt3d_forward_noalloc(_ptr(vol), _ptr(out), N, mask, dt, _stream(stream)))
    return out


def djt3d_forward(vol: torch.Tensor, mask: int = DRT3D_ALL, out: Optional[torch.Tensor] = None,
                  workspace: Optional[torch.Tensor] = None, stream=None) -> torch.Tensor:
    """3D DJT of lines over the dodecants of `mask`: [popcount][N][N][2N-1][2N-1]."""
    N = _cube(vol)
    dt = _dtype_code(vol)
    shape = djt3d_out_shape(N, mask)
    with _on_stream(stream):
        if out is None:
            out = torch.empty(shape, dtype=vol.dtype, device=vol.device)
        else:
            _check_out(out, shape, vol.dtype, vol.device)
        ws = _workspace(lib().djt3d_workspace_bytes(N, mask, dt), vol.device, workspace)
        check(lib().djt3d_forward(_ptr(vol), _ptr(out), N, mask, dt, _ptr(ws), _ws_bytes(ws), _stream(stream)))
    return out


def _proj(proj: torch.Tensor, mask: int, kind: str) -> int:
    """N of a DRT ('drt') or DJT ('djt') projection in the forward layout of mask."""
    ndim, shape_of = (4, drt3d_out_shape) if kind == "drt" else (5, djt3d_out_shape)
    if proj.dim() != ndim or proj.shape[0] != dodecant_count(mask):
        raise ValueError("proj must be %s for mask %#x, got %s" % (
            "[popcount][N][N][3N-2]" if kind == "drt" else "[popcount][N][N][2N-1][2N-1]", mask, tuple(proj.shape)))
    N = int(proj.shape[1])
    if tuple(proj.shape) != shape_of(N, mask) or not proj.is_cuda or not proj.is_contiguous():
        raise ValueError("proj must be a contiguous device tensor of shape %s" % (shape_of(N, mask),))
    return N


def drt3d_adjoint(proj: torch.Tensor, mask: int = DRT3D_ALL, out: Optional[torch.Tensor] = None,
                  workspace: Optional[torch.Tensor] = None, stream=None) -> torch.Tensor:
    """Backprojection (exact transpose of drt3d_forward): [N][N][N]."""
    N = _proj(proj, mask, "drt")
    dt = _dtype_code(proj)
    with _on_stream(stream):
        if out is None:
            out = torch.empty((N, N, N), dtype=proj.dtype, device=proj.device)
        else:
            _check_out(out, (N, N, N), proj.dtype, proj.device)
        ws = _workspace(lib().drt3d_adjoint_workspace_bytes(N, mask, dt), proj.device, workspace)
        check(lib().drt3d_adjoint(_ptr(proj), _ptr(out), N, mask, dt, _ptr(ws), _ws_bytes(ws), _stream(stream)))
    return out


def djt3d_adjoint(proj: torch.Tensor, mask: int = DRT3D_ALL, out: Optional[torch.Tensor] = None,
                  workspace: Optional[torch.Tensor] = None, stream=None) -> torch.Tensor:
    """Exact transpose of djt3d_forward: [N][N][N]."""
    N = _proj(proj, mask, "djt")
    dt = _dtype_code(proj)
    with _on_stream(stream):
        if out is None:
            out = torch.empty((N, N, N), dtype=proj.dtype, device=proj.device)
        else:
            _check_out(out, (N, N, N), proj.dtype, proj.device)
        ws = _workspace(lib().djt3d_adjoint_workspace_bytes(N, mask, dt), proj.device, workspace)
        check(lib().djt3d_adjoint(_ptr(proj), _ptr(out), N, mask, dt, _ptr(ws), _ws_bytes(ws), _stream(stream)))
    return out


def _batched(fn_name: str, ws_name: str, ins: Sequence[torch.Tensor], outs: Optional[Sequence[torch.Tensor]],
             out_shape, Ns: Sequence[int], mask: int, dt: int, workspace, stream) -> List[torch.Tensor]:
    """Checks that the inputs share one dtype and device, allocates or checks
    one output per input (out_shape(N)), then makes the batched call."""
    dev, tdt = ins[0].device, ins[0].dtype
    for t in ins:
        if t.dtype != tdt:
            raise TypeError("all inputs of a batched call must share one dtype (%s and %s)" % (tdt, t.dtype))
        if t.device != dev:
            raise ValueError("all inputs of a batched call must be on one device (%s and %s)" % (dev, t.device))
    count = len(ins)
    with _on_stream(stream):
        if outs is None:
            outs = [torch.empty(out_shape(N), dtype=tdt, device=dev) for N in Ns]
        else:
            outs = list(outs)
            if len(outs) != count:
                raise ValueError("outs holds %d tensors for %d inputs" % (len(outs), count))
            for i, (o, N) in enumerate(zip(outs, Ns)):
                _check_out(o, out_shape(N), tdt, dev, "outs[%d]" % i)
        a_in = (ctypes.c_void_p * count)(*[t.data_ptr() for t in ins])
        a_out = (ctypes.c_void_p * count)(*[t.data_ptr() for t in outs])
        a_N = (ctypes.c_int * count)(*Ns)
        need = getattr(lib(), ws_name)(count, a_N, mask, dt)
        if need == 0:
            raise ValueError("invalid batched arguments")
        ws = _workspace(need, dev, workspace)
        check(getattr(lib(), fn_name)(count, a_in, a_out, a_N, mask, dt, _ptr(ws), _ws_bytes(ws), _stream(stream)))
    return outs


def drt3d_forward_batched(vols: Sequence[torch.Tensor], mask: int = DRT3D_ALL,
                          outs: Optional[Sequence[torch.Tensor]] = None,
                          workspace: Optional[torch.Tensor] = None, stream=None) -> List[torch.Tensor]:
    """DRT of many cubes (mixed N, same dtype) in one set of persistent launches."""
    if not vols:
        return []
    Ns = [_cube(v) for v in vols]
    dt = _dtype_code(vols[0])
    return _batched("drt3d_forward_batched", "drt3d_forward_batched_workspace_bytes", vols, outs,
                    lambda N: drt3d_out_shape(N, mask), Ns, mask, dt, workspace, stream)


def djt3d_forward_batched(vols: Sequence[torch.Tensor], mask: int = DRT3D_ALL,
                          outs: Optional[Sequence[torch.Tensor]] = None,
                          workspace: Optional[torch.Tensor] = None, stream=None) -> List[torch.Tensor]:
    """DJT of many cubes (mixed N, same dtype) in one set of persistent launches."""
    if not vols:
        return []
    Ns = [_cube(v) for v in vols]
    dt = _dtype_code(vols[0])
    return _batched("djt3d_forward_batched", "djt3d_forward_batched_workspace_bytes", vols, outs,
                    lambda N: djt3d_out_shape(N, mask), Ns, mask, dt, workspace, stream)


def drt3d_adjoint_batched(projs: Sequence[torch.Tensor], mask: int = DRT3D_ALL,
                          outs: Optional[Sequence[torch.Tensor]] = None,
                          workspace: Optional[torch.Tensor] = None, stream=None) -> List[torch.Tensor]:
    """DRT adjoints of many projections (mixed N, same dtype)."""
    if not projs:
        return []
    Ns = [_proj(p, mask, "drt") for p in projs]
    dt = _dtype_code(projs[0])
    return _batched("drt3d_adjoint_batched", "drt3d_adjoint_batched_workspace_bytes", projs, outs,
                    lambda N: (N, N, N), Ns, mask, dt, workspace, stream)


def djt3d_adjoint_batched(projs: Sequence[torch.Tensor], mask: int = DRT3D_ALL,
                          outs: Optional[Sequence[torch.Tensor]] = None,
                          workspace: Optional[torch.Tensor] = None, stream=None) -> List[torch.Tensor]:
    """DJT adjoints of many projections (mixed N, same dtype)."""
    if not projs:
        return []
    Ns = [_proj(p, mask, "djt") for p in projs]
    dt = _dtype_code(projs[0])
    return _batched("djt3d_adjoint_batched", "djt3d_adjoint_batched_workspace_bytes", projs, outs,
                    lambda N: (N, N, N), Ns, mask, dt, workspace, stream)


def drt3d_merge_net(proj: torch.Tensor, out: Optional[torch.Tensor] = None, stream=None) -> torch.Tensor:
    """Algorithm 2's merged output: the 12-dodecant DRT rotated and placed in a
    [4N][4N][3N-2] net (the four corner blocks zero)."""
    N = _proj(proj, DRT3D_ALL, "drt")
    dt = _dtype_code(proj)
    shape = (4 * N, 4 * N, 3 * N - 2)
    with _on_stream(stream):
        if out is None:
            out = torch.empty(shape, dtype=proj.dtype, device=proj.device)
        else:
            _check_out(out, shape, proj.dtype, proj.device)
        check(lib().drt3d_merge_net(_ptr(proj), _ptr(out), N, dt, _stream(stream)))
    return out


def drt3d_detect_planes(proj: torch.Tensor, cos_tol: float = 0.05, rel_threshold: float = 0.5,
                        mask: int = DRT3D_ALL, cap: int = 4096, workspace: Optional[torch.Tensor] = None,
                        stream=None):
    """Plane detection in a DRT output (Sec. 6.1): returns (bins, count), bins
    an int64 device tensor of flat output indices (the dominant plane first,
    then the qualifying planes in ascending order, at most cap of them) and
    count the number found (which may exceed cap). Reads count back, so the
    call waits for the stream."""
    N = _proj(proj, mask, "drt")
    dt = _dtype_code(proj)
    with _on_stream(stream):
        ws = _workspace(lib().drt3d_detect_planes_workspace_bytes(N, mask, dt), proj.device, workspace)
        bins = torch.empty(max(1, int(cap)), dtype=torch.int64, device=proj.device)
        count = torch.empty(1, dtype=torch.int64, device=proj.device)
        check(lib().drt3d_detect_planes(_ptr(proj), N, mask, dt, float(cos_tol), float(rel_threshold), _ptr(bins),
                                        bins.numel(), _ptr(count), _ptr(ws), _ws_bytes(ws), _stream(stream)))
        n = int(count.item())
    return bins[:min(n, bins.numel())], n


def drt3d_backproject_bins(bins: torch.Tensor, N: int, mask: int = DRT3D_ALL, dtype=torch.int32,
                           out: Optional[torch.Tensor] = None, workspace: Optional[torch.Tensor] = None,
                           stream=None) -> torch.Tensor:
    """Per voxel, the number of listed planes through it: the adjoint of the
    0/1 projection marking the flat indices in bins (int64 device tensor)."""
    if bins.dtype != torch.int64 or not bins.is_cuda or bins.dim() != 1 or not bins.is_contiguous():
        raise ValueError("bins must be a contiguous 1-D int64 device tensor")
    if dtype not in (torch.int32, torch.float32):
        raise TypeError("dtype must be torch.int32 or torch.float32")
    dt = DRT3D_F32 if dtype == torch.float32 else DRT3D_I32
    with _on_stream(stream):
        if out is None:
            out = torch.empty((N, N, N), dtype=dtype, device=bins.device)
        else:
            _check_out(out, (N, N, N), dtype, bins.device)
        ws = _workspace(lib().drt3d_backproject_bins_workspace_bytes(N, mask, dt), bins.device, workspace)
        count = torch.full((1,), bins.numel(), dtype=torch.int64, device=bins.device)
        if bins.numel() == 0:  # no planes: a valid pointer, nothing read
            bins = torch.zeros(1, dtype=torch.int64, device=bins.device)
        check(lib().drt3d_backproject_bins(_ptr(bins), _ptr(count), bins.numel(), _ptr(out), N, mask, dt,
                                           _ptr(ws), _ws_bytes(ws), _stream(stream)))
    return out


def drt3d_plane_normal(k: int, s1: int, s2: int, N: int):
    """Integer normal (x, y, z) of dodecant k's planes at slopes (s1, s2), scaled by N-1."""
    arr = (ctypes.c_int * 3)()
    check(lib().drt3d_plane_normal(k, s1, s2, N, arr))
    return tuple(arr)


def _inverse_workspace(N: int, device, workspace):
    need = lib().drt3d_inverse_workspace_bytes(N)
    if need == 0:
        raise ValueError("the inverse takes N a power of two in [2, 512], got %d" % N)
    return _workspace(need, device, workspace)


def drt3d_inverse(proj: torch.Tensor, cycles: int = 10, lams: Optional[Sequence[float]] = None,
                  out: Optional[torch.Tensor] = None, workspace: Optional[torch.Tensor] = None,
                  stream=None) -> torch.Tensor:
    """Iterative inverse (Sec. 5.2) of a 12-dodecant float32 DRT: [N][N][N].

    lams: the eigenvalues for sizes 2, 4, ..., N (as drt3d_inverse_lambdas
    returns them), or None to let the library compute and cache them."""
    N = _proj(proj, DRT3D_ALL, "drt")
    if proj.dtype != torch.float32:
        raise ValueError("the inverse takes a float32 projection")
    n = N.bit_length() - 1
    arr = None
    if lams is not None:
        if len(lams) != n:
            raise ValueError("lams needs %d values (sizes 2 .. %d)" % (n, N))
        arr = (ctypes.c_double * n)(*[float(v) for v in lams])
    with _on_stream(stream):
        if out is None:
            out = torch.empty((N, N, N), dtype=torch.float32, device=proj.device)
        else:
            _check_out(out, (N, N, N), torch.float32, proj.device)
        ws = _inverse_workspace(N, proj.device, workspace)
        check(lib().drt3d_inverse(_ptr(proj), _ptr(out), N, int(cycles), arr, _ptr(ws), _ws_bytes(ws),
                                  _stream(stream)))
    return out


def drt3d_inverse_lambdas(N: int, device="cuda", workspace: Optional[torch.Tensor] = None, stream=None) -> List[float]:
    """The smoother's eigenvalues for sizes 2, 4, ..., N (computed once per size)."""
    n = N.bit_length() - 1
    arr = (ctypes.c_double * n)()
    with _on_stream(stream):
        ws = _inverse_workspace(N, device, workspace)
        check(lib().drt3d_inverse_lambdas(N, arr, _ptr(ws), _ws_bytes(ws), _stream(stream)))
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


def stream_probe(src: torch.Tensor, read_bytes: int, dst: torch.Tensor, write_bytes: int, stream=None) -> None:
    """The reference stream (drt3d_stream_probe): reads read_bytes of src and
    writes write_bytes of dst, the HBM ceiling for that mix of reads and writes."""
    for t, nb, what in ((src, read_bytes, "src"), (dst, write_bytes, "dst")):
        if not t.is_cuda or not t.is_contiguous() or t.numel() * t.element_size() < nb:
            raise ValueError("%s must be a contiguous device tensor of at least %d bytes" % (what, nb))
    check(lib().drt3d_stream_probe(_ptr(src), int(read_bytes), _ptr(dst), int(write_bytes), _stream(stream)))


class Plan:
    """A fixed transform (drt3d_plan_create): op "drt_forward", "drt_adjoint",
    "djt_forward" or "djt_adjoint" for size N, mask and dtype (torch.int32,
    torch.float32, or torch.uint8 for "drt_forward"), keeping the DRT tuning in
    force when it is made. Calling it runs that transform on `inp` (the op's own
    input layout); results equal the op's own call under that tuning."""

    OPS = {"drt_forward": 0, "drt_adjoint": 1, "djt_forward": 2, "djt_adjoint": 3}
    _CODES = {torch.int32: DRT3D_I32, torch.float32: DRT3D_F32, torch.uint8: DRT3D_U8}

    def __init__(self, op: str, N: int, mask: int = DRT3D_ALL, dtype=torch.int32):
        self._h = None
        if op not in self.OPS:
            raise ValueError("op must be one of %s, got %r" % (sorted(self.OPS), op))
        if dtype not in self._CODES:
            raise TypeError("plans take int32, float32 or uint8, got %s" % (dtype,))
        self.op, self.N, self.mask, self.dtype = op, int(N), int(mask), dtype
        h = ctypes.c_void_p()
        check(lib().drt3d_plan_create(ctypes.byref(h), self.OPS[op], self.N, self.mask, self._CODES[dtype]))
        self._h = h
        self.workspace_bytes = int(lib().drt3d_plan_workspace_bytes(h))

    def shapes(self):
        """(input shape, output shape)."""
        vol = (self.N, self.N, self.N)
        proj = (drt3d_out_shape if self.op.startswith("drt") else djt3d_out_shape)(self.N, self.mask)
        return (vol, proj) if self.op.endswith("forward") else (proj, vol)

    def __call__(self, inp: torch.Tensor, out: Optional[torch.Tensor] = None,
                 workspace: Optional[torch.Tensor] = None, stream=None) -> torch.Tensor:
        if self._h is None:
            raise ValueError("the plan is closed")
        in_shape, out_shape = self.shapes()
        if (tuple(inp.shape) != in_shape or inp.dtype != self.dtype or not inp.is_cuda
                or not inp.is_contiguous()):
            raise ValueError("input must be a contiguous %s device tensor of shape %s, got %s %s"
                             % (self.dtype, in_shape, inp.dtype, tuple(inp.shape)))
        odt = torch.int32 if self.dtype == torch.uint8 else self.dtype
        with _on_stream(stream):
            if out is None:
                out = torch.empty(out_shape, dtype=odt, device=inp.device)
            else:
                _check_out(out, out_shape, odt, inp.device)
            ws = _workspace(self.workspace_bytes, inp.device, workspace)
            check(lib().drt3d_plan_execute(self._h, _ptr(inp), _ptr(out), _ptr(ws), _ws_bytes(ws),
                                           _stream(stream)))
        return out

    def close(self) -> None:
        if self._h is not None:
            lib().drt3d_plan_destroy(self._h)
            self._h = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()
        return False

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


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
