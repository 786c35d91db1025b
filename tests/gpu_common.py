"""Helpers shared by the GPU parity tests (imported only by tests)."""
import numpy as np
import pytest


def gpu_or_skip():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_2112_01508_amd as p3
    p3.load_library()
    return torch, p3


def to_dev(torch, a, dtype=None):
    if a is None:
        return None
    t = torch.from_numpy(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.to("cuda:0")


# Pass/fail bars of the force comparison (relative errors against the FP64
# oracle, see oracle.errors): FP64 path 1e-12, FP32 path 1e-5.
TOL = {"fp64": 1e-12, "fp32": 1e-5}
