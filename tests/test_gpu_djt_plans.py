"""The DJT under every kind of pass plan (stages fused per pass: 1, 2 or 3,
forced through DRT3D_DJT_PASSES): the forward equals the oracle's recursion
and the adjoint equals the one of the built-in plan (itself pinned to the
oracle's definition), bit for bit in int32. The built-in plan uses passes of 1
and 2 stages; this keeps the 3-stage kernels and other orders covered."""
import ctypes

import numpy as np
import pytest

import oracle as O
import workloads
from tests.gpu_util import announce, to_dev

pytestmark = pytest.mark.gpu

PLANS = {16: ["2,2", "1,3", "3,1", "1,1,2", "1,1,1,1"],
         32: ["1,2,2", "3,2", "2,3", "2,1,2", "1,1,3", "3,1,1"]}


@pytest.mark.parametrize("N", [16, 32])
def test_djt_every_plan_is_bit_exact(N, monkeypatch):
    from paper_2501_13664_amd import api
    from paper_2501_13664_amd._lib import lib
    mask = 0xFFF if N == 16 else 0b100100100101
    vol = workloads.noise_with_segments(N, n_segments=4, seed=500 + N)
    ref = O.wrap_int32(O.rec_djt(vol, mask))
    proj = to_dev(np.random.default_rng(510 + N).integers(-500, 500, size=ref.shape).astype(np.int32))
    monkeypatch.delenv("DRT3D_DJT_PASSES", raising=False)
    announce("djt plans N=%d: built-in plan adjoint" % N)
    adj_ref = api.djt3d_adjoint(proj, mask)
    for plan in PLANS[N]:
        monkeypatch.setenv("DRT3D_DJT_PASSES", plan)
        # the override is in force: one launch per pass of the plan
        buf = ctypes.create_string_buffer(4096)
        assert lib().drt3d_plan_text(2, N, mask, 0, buf, 4096) == len(plan.split(",")), plan
        announce("djt plans N=%d plan %s" % (N, plan))
        got = api.djt3d_forward(to_dev(vol), mask).cpu().numpy()
        assert np.array_equal(got, ref), "forward, plan " + plan
        assert np.array_equal(api.djt3d_adjoint(proj, mask).cpu().numpy(), adj_ref.cpu().numpy()), \
            "adjoint, plan " + plan
