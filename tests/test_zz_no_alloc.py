"""GPU test of gfc_solve_batch_noalloc, the forward solve whose workspace is the library's
fixed device array: called through the C ABI, its output must equal gfc_solve_batch's
(same kernels: bit for bit), on two calls in a row, the second with a smaller input."""
import ctypes
import os
import sys

import numpy as np
import pytest

import gfc_synth as synth

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_1902_00176_amd as gfc  # noqa: E402

GFC_E_WORKSPACE = 4
SCRATCH_BYTES = 64 << 20


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    if not os.path.exists(gfc.lib_path()):
        pytest.fail("libgfc.so is not built: the HIP path must exist where a GPU is present")


def _fields(seed, B, H, W):
    rng = np.random.default_rng(seed)
    gx = np.empty((B, H, W), np.float32)
    gy = np.empty((B, H, W), np.float32)
    for i in range(B):
        a, b = synth.forward_gradient(synth.gaussian_sum_field(rng, H, W))
        gx[i] = a + 0.01 * rng.normal(size=(H, W))
        gy[i] = b
    return torch.from_numpy(gx).cuda(), torch.from_numpy(gy).cuda()


def _noalloc(plan, gx, gy, u, B):
    s = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    return gfc.lib().gfc_solve_batch_noalloc(plan.handle, ctypes.c_void_p(gx.data_ptr()),
                                             ctypes.c_void_p(gy.data_ptr()),
                                             ctypes.c_void_p(u.data_ptr()), B, s)


def test_noalloc_equals_workspace_solve_on_two_calls():
    cases = [(256, 384, 6), (100, 150, 2)]  # the second call is smaller
    outs = []
    for H, W, B in cases:
        _say(f"noalloc: {B} images of {H}x{W}")
        p = gfc.Plan(H, W, tuned=False).build()
        assert p.workspace_size(B) <= SCRATCH_BYTES
        gx, gy = _fields(H * 3 + W, B, H, W)
        u = torch.full_like(gx, float("nan"))
        assert _noalloc(p, gx, gy, u, B) == 0
        outs.append((p, gx, gy, u))
    torch.cuda.synchronize()
    for p, gx, gy, u in outs:
        ref = p.solve(gx, gy)
        torch.cuda.synchronize()
        assert torch.equal(u, ref), (p.H, p.W)


def test_noalloc_same_plan_smaller_batch_after_larger():
    H, W = 801, 1200
    p = gfc.Plan(H, W, tuned=False).build()
    gx, gy = _fields(8011, 7, H, W)
    for B in (7, 3):  # the largest batch the array holds at this size, then a smaller one
        _say(f"noalloc: {B} images of {H}x{W}")
        u = torch.full_like(gx[:B], float("nan"))
        assert _noalloc(p, gx[:B], gy[:B], u, B) == 0
        ref = p.solve(gx[:B], gy[:B])
        torch.cuda.synchronize()
        assert torch.equal(u, ref), B


def test_noalloc_rejects_a_call_larger_than_the_array():
    H, W = 801, 1200
    p = gfc.Plan(H, W, tuned=False).build()
    B = 8
    assert p.workspace_size(B) > SCRATCH_BYTES
    gx = torch.zeros(B, H, W, device="cuda")
    u = torch.full_like(gx, 7.0)
    assert _noalloc(p, gx, gx, u, B) == GFC_E_WORKSPACE
    torch.cuda.synchronize()
    assert bool((u == 7.0).all())  # nothing was launched
