"""GPU parity of every compiled row transform: each row length N the library supports
(gfc_supported_length) runs a forward and a backward solve through the C ABI, compared
with the float64 oracle per image at relative L2 <= 1e-5.

Two shapes per length exercise the two loader variants of the row passes:
  * W = N / 2 on a 20-row image (M = 48): the support fits the first half of each row FFT
    (every default torus), and the plan splits the 4 lowest row bins;
  * W = N - 2 on a 3-row image (M = 8): the widest image a torus of width N accepts, with
    every element column loaded, and a thin torus, whose plan splits up to 32 row bins.
"""
import os
import sys

import numpy as np
import pytest

import gfc_synth as synth
import oracle as O

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_1902_00176_amd as gfc  # noqa: E402

TOL = 1e-5
MAX_N = 8192


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _lengths():
    """Row lengths compiled into the library (empty where it is not built: the GPU fixture
    then fails loudly)."""
    if not os.path.exists(gfc.lib_path()):
        return [0]
    return [n for n in range(2, MAX_N + 1, 2) if gfc.supported_length(n)]


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    if not os.path.exists(gfc.lib_path()):
        pytest.fail("libgfc.so is not built: the HIP path must exist where a GPU is present")


def rel_l2(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def _fields(seed, B, H, W):
    rng = np.random.default_rng(seed)
    gx = np.empty((B, H, W), np.float32)
    gy = np.empty((B, H, W), np.float32)
    for i in range(B):
        a, b = synth.forward_gradient(synth.gaussian_sum_field(rng, H, W))
        gx[i] = a + 0.01 * rng.normal(size=(H, W))  # not conservative: every term matters
        gy[i] = b
    return gx, gy


def _shapes(N):
    return [(20, N // 2, 48, N), (3, N - 2, 8, N)]


@pytest.mark.parametrize("N", _lengths())
def test_every_row_length_forward_and_backward(N):
    for H, W, M, NN in _shapes(N):
        _say(f"length {N}: H={H} W={W} M={M} N={NN}")
        p = gfc.Plan(H, W, M, NN, tuned=False)
        gx, gy = _fields(N * 31 + W, 2, H, W)
        tx = torch.from_numpy(gx).cuda()
        ty = torch.from_numpy(gy).cuda()
        u = p.solve(tx, ty).cpu().numpy()
        ref = O.solve_fft(gx, gy, M, NN)
        errs = [rel_l2(u[i], ref[i]) for i in range(2)]
        assert max(errs) <= TOL, ("forward", N, W, errs)
        du = (np.random.default_rng(N + W).normal(size=(2, H, W)) * 0.1 + 0.01).astype(np.float32)
        dgx, dgy = p.backward(torch.from_numpy(du).cuda())
        dgx, dgy = dgx.cpu().numpy(), dgy.cpu().numpy()
        rx, ry = O.solve_backward(du, M, NN)
        errs = [rel_l2(np.concatenate([dgx[i], dgy[i]]), np.concatenate([rx[i], ry[i]]))
                for i in range(2)]
        assert max(errs) <= TOL, ("backward", N, W, errs)
