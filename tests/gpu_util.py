"""Helpers shared by the GPU tests."""
import sys

import numpy as np
import pytest


def device():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a HIP device")
    return torch.device("cuda:0")


def announce(*parts):
    """Print (and flush) what the next GPU step runs, so a failure names it."""
    print("[gpu-case]", *parts, flush=True)
    sys.stdout.flush()


def to_dev(a):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).to(device())


def float_errors(y32, y64, r_abs):
    """Normwise relative L2 error and max |y32 - y64| / R(|f|) (elementwise bound
    relative to the transform of |f|, computed in float64)."""
    y32 = np.asarray(y32, dtype=np.float64)
    y64 = np.asarray(y64, dtype=np.float64)
    diff = y32 - y64
    normwise = np.linalg.norm(diff) / max(np.linalg.norm(y64), 1e-300)
    denom = np.maximum(np.asarray(r_abs, dtype=np.float64), 1e-300)
    mask = np.asarray(r_abs) > 0
    elem = float(np.max(np.abs(diff[mask]) / denom[mask])) if mask.any() else 0.0
    assert np.all(diff[~mask] == 0) if (~mask).any() else True
    return float(normwise), elem


FLOAT_TOL = 1e-5
