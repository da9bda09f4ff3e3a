"""The Python binding rejects caller buffers that do not match before any
library call (the C ABI takes no output sizes, so a mismatch would be an
out-of-bounds device write), and runs correctly on a caller's own stream."""
import ctypes

import numpy as np
import pytest

import workloads
from tests.gpu_util import announce, to_dev

pytestmark = pytest.mark.gpu


def _api():
    from paper_2501_13664_amd import api
    return api


def test_outputs_that_do_not_match_are_rejected():
    import torch
    api = _api()
    N = 8
    vol = to_dev(workloads.uniform_int_cube(N, 0, 9, seed=1))
    proj = api.drt3d_forward(vol)
    announce("api checks: mismatched outputs")
    bad_outs = [
        torch.empty((N, N, N + 1), dtype=torch.int32, device="cuda"),       # shape
        torch.empty((N, N, N), dtype=torch.float32, device="cuda"),         # dtype
        torch.empty((N, N, 2 * N), dtype=torch.int32, device="cuda")[:, :, ::2],  # layout
        torch.empty((N, N, N), dtype=torch.int32),                          # host memory
    ]
    for o in bad_outs:
        with pytest.raises(ValueError):
            api.drt3d_adjoint(proj, out=o)
    with pytest.raises(ValueError):
        api.drt3d_forward(vol, out=torch.empty((12, N, N, 3 * N - 1), dtype=torch.int32, device="cuda"))
    # batched: every output checked, count too
    vols = [vol, to_dev(workloads.uniform_int_cube(16, 0, 9, seed=2))]
    good = [torch.empty(api.drt3d_out_shape(n), dtype=torch.int32, device="cuda") for n in (8, 16)]
    with pytest.raises(ValueError):
        api.drt3d_forward_batched(vols, outs=[good[0], good[0]])
    with pytest.raises(ValueError):
        api.drt3d_forward_batched(vols, outs=[good[0]])
    with pytest.raises(ValueError):
        api.drt3d_forward_batched(vols, outs=[good[0], good[1].float()])
    with pytest.raises(TypeError):
        api.drt3d_forward_batched([vol, vol.float()])
    projs = api.drt3d_forward_batched(vols, outs=good)
    with pytest.raises(ValueError):
        api.drt3d_adjoint_batched(projs, outs=[torch.empty((8, 8, 8), dtype=torch.int32, device="cuda")] * 2)
    with pytest.raises(TypeError):
        api.drt3d_adjoint_batched([projs[0], projs[1].float()])
    with pytest.raises(ValueError):
        api.drt3d_forward(vol, workspace=torch.empty(1 << 20, dtype=torch.uint8))  # host workspace


def test_a_caller_stream_gives_the_same_results():
    import torch
    api = _api()
    N = 32
    vol = to_dev(workloads.uniform_int_cube(N, 0, 255, seed=3))
    announce("api checks: caller stream")
    ref = api.drt3d_forward(vol)
    back_ref = api.drt3d_adjoint(ref)
    torch.cuda.synchronize()
    s = torch.cuda.Stream()
    out = api.drt3d_forward(vol, stream=s)
    back = api.drt3d_adjoint(out, stream=s)
    outs = api.drt3d_forward_batched([vol, vol], stream=s)
    s.synchronize()
    assert torch.equal(out, ref) and torch.equal(back, back_ref)
    assert all(torch.equal(o, ref) for o in outs)
    assert np.array_equal(back.cpu().numpy(), back_ref.cpu().numpy())


def test_device_given_without_an_index_accepts_buffers_on_the_current_device():
    """'cuda' names the current device: a workspace or output allocated on
    'cuda:0' is accepted when the call names the device as 'cuda'."""
    import torch
    api = _api()
    from paper_2501_13664_amd._lib import lib
    N = 8
    announce("api checks: device named without an index")
    ws = torch.empty(lib().drt3d_inverse_workspace_bytes(N), dtype=torch.uint8, device="cuda:0")
    lams = api.drt3d_inverse_lambdas(N, device="cuda", workspace=ws)
    assert len(lams) > 0 and all(np.isfinite(lams))
    with pytest.raises(ValueError):
        api.drt3d_inverse_lambdas(N, device="cuda", workspace=torch.empty(16, dtype=torch.uint8))


def test_batched_calls_with_many_workspaces_stay_correct():
    """Each fresh workspace address is a new replay graph; past the cache's
    bound the least recently used ones are destroyed and the calls go on
    giving the single-volume results."""
    import torch
    api = _api()
    from paper_2501_13664_amd._lib import lib
    announce("api checks: 40 batched calls on 40 workspaces")
    vols = [to_dev(workloads.uniform_int_cube(n, 0, 99, seed=60 + n)) for n in (8, 16)]
    refs = [api.drt3d_forward(v) for v in vols]
    need = lib().drt3d_forward_batched_workspace_bytes(2, (ctypes.c_int * 2)(8, 16), 0xFFF, 0)
    keep = []
    for i in range(40):
        ws = torch.empty(need + 256 * (i + 1), dtype=torch.uint8, device="cuda")[256 * (i + 1):]
        keep.append(ws)  # distinct addresses
        outs = api.drt3d_forward_batched(vols, workspace=ws)
        if i % 13 == 0 or i == 39:
            torch.cuda.synchronize()
            assert all(torch.equal(o, r) for o, r in zip(outs, refs)), "call %d" % i
    torch.cuda.synchronize()
