"""The allocation-free forward (msim_forward_noalloc, called through the C-ABI)
against the ordinary forward (msim_forward) on the same plans: two calls in a
row, the second on a smaller plan, each bit-equal to msim_forward and within
the parity bar of the FP64 oracle; and the scratch size limit."""
import ctypes as C

import numpy as np
import pytest

from oracle import oracle as O
from paper_2508_03065_amd import scenegen as G

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def noalloc(plan, x, y, torch):
    from paper_2508_03065_amd import _lib
    L = _lib.load()
    return L.msim_forward_noalloc(plan._ptr, C.c_void_p(x.data_ptr()), C.c_void_p(y.data_ptr()),
                                  C.c_void_p(torch.cuda.current_stream().cuda_stream))


def test_noalloc_matches_forward_twice(torch_cuda):
    torch = torch_cuda
    from paper_2508_03065_amd import _lib
    from paper_2508_03065_amd.msim import Plan
    # the second call's plan is smaller (fewer images, shorter signal)
    for seed, order, seconds in ((61, 5, 0.3), (62, 3, 0.1)):
        sc, par = G.small_scene(seed=seed, max_order=order, seconds=seconds, n_mics=2, moving_rcv=True)
        plan = Plan([sc], par)
        assert plan.workspace_bytes(False) <= 64 << 20
        x = plan.pack_x([sc.x])
        y_ref = plan.forward(x)
        y = torch.full_like(y_ref, float("nan"))
        st = noalloc(plan, x, y, torch)
        assert st == 0, _lib.load().msim_last_error().decode()
        torch.cuda.synchronize()
        assert plan.device_status() == 0
        assert torch.equal(y, y_ref)
        got = plan.unpack_y(y)[0].cpu().numpy().astype(np.float64)
        ref = O.forward(sc, par)
        assert np.linalg.norm(got - ref) / np.linalg.norm(ref) <= 1e-5


def test_noalloc_rejects_a_plan_beyond_its_scratch(torch_cuda):
    torch = torch_cuda
    from paper_2508_03065_amd import _lib
    from paper_2508_03065_amd.msim import Plan
    scenes, par = G.config3(n_scenes=8)
    plan = Plan(scenes, par)
    if plan.workspace_bytes(False) <= 64 << 20:
        pytest.skip("this plan fits the fixed scratch")
    x = plan.pack_x([s.x for s in scenes])
    y = torch.zeros(plan.y_total, dtype=torch.float32, device="cuda")
    st = noalloc(plan, x, y, torch)
    assert st == 5          # MSIM_E_WORKSPACE
    assert b"fixed per-GPU scratch" in _lib.load().msim_last_error()
    assert float(y.abs().sum()) == 0.0
