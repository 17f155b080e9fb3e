"""GPU parity of the Laplacian-input solve (gfc_solve_laplacian, Algorithm B's literal input)
against the float64 oracle on the same float32 Laplacian.

Bar: 1e-5 relative L2, as for the gradient input. The row bins l <= K, which the Green's
function amplifies most, are float64 direct sums handed over as running sums over the rows
(a float32 FFT of L would leave an error of the size of |L| where their true values nearly
cancel: up to 6e-4 on the thinnest tori in a float32 emulation). The same emulation of the
path as built gives 1.3e-7 at 801x1200 on 1620x2400, 8e-8 at 1024^2 on 2048^2 and 1.3e-6 on
a 2 x 1200 image on 6 x 2400."""
import sys

import numpy as np
import pytest

import gfc_synth as synth
import oracle as O

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_1902_00176_amd as gfc  # noqa: E402

TOL = 1e-5


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _support_div(gx, gy):
    """div E on the (H+1) x (W+1) support (backward differences), float64."""
    B, H, W = gx.shape
    Ex = np.zeros((B, H + 1, W + 1)); Ex[:, :H, :W] = gx
    Ey = np.zeros((B, H + 1, W + 1)); Ey[:, :H, :W] = gy
    L = Ex.copy(); L[:, :, 1:] -= Ex[:, :, :-1]
    L += Ey; L[:, 1:, :] -= Ey[:, :-1, :]
    return L


def _fields(seed, B, H, W):
    gx = np.empty((B, H, W)); gy = np.empty((B, H, W))
    for i, rng in enumerate(synth.image_rngs(seed, B)):
        S = synth.gaussian_sum_field(rng, H, W)
        a, b = synth.forward_gradient(S)
        gx[i] = a + 0.01 * rng.normal(size=(H, W))
        gy[i] = b
    return gx, gy


SHAPES = [(64, 64, 128, 128), (31, 45, 64, 96), (100, 37, 210, 80), (33, 70, 35, 72),
          (801, 1200, 1620, 2400), (1024, 1024, 2048, 2048),
          # thin, wide tori: their plans split 16 and 32 row bins
          (8, 1200, 16, 2400), (2, 1200, 6, 2400), (3, 2046, 6, 2048), (1, 37, 3, 80)]


@pytest.mark.parametrize("shape", SHAPES, ids=lambda s: f"{s[0]}x{s[1]}@{s[2]}x{s[3]}")
def test_laplacian_solve_matches_oracle(shape):
    H, W, M, N = shape
    B = 2 if H * W > 100000 else 3
    _say(f"[laplacian] {H}x{W} on {M}x{N}, B={B}")
    gx, gy = _fields(3401 + H, B, H, W)
    L = _support_div(gx, gy).astype(np.float32)
    u = gfc.solve_laplacian(torch.from_numpy(L).cuda(), M, N).cpu().numpy()
    for i in range(B):
        ref = O.solve_laplacian(L[i], M, N)
        e = float(np.linalg.norm(u[i] - ref) / np.linalg.norm(ref))
        _say(f"  image {i}: rel. L2 {e:.3e}")
        assert e <= TOL


def test_laplacian_of_a_framed_image_reconstructs_it():
    """The 5-point Laplacian (Algorithm A's stencil) of an image with a zero first row and
    column solves back to the image, offset included."""
    H, W, M, N = 96, 128, 192, 256
    rng = np.random.default_rng(3450)
    S = synth.gaussian_sum_field(rng, H, W)
    S[0, :] = 0.0
    S[:, 0] = 0.0
    P = np.zeros((H + 3, W + 3)); P[1:H + 1, 1:W + 1] = S
    L = (P[:-2, 1:-1] + P[2:, 1:-1] + P[1:-1, :-2] + P[1:-1, 2:] - 4 * P[1:-1, 1:-1])
    L = L[:H + 1, :W + 1].astype(np.float32)
    u = gfc.solve_laplacian(torch.from_numpy(L[None]).cuda(), M, N).cpu().numpy()[0]
    ref = O.solve_laplacian(L, M, N)
    assert np.linalg.norm(u - ref) / np.linalg.norm(ref) <= TOL
    assert np.linalg.norm(u - S) / np.linalg.norm(S) <= TOL + 1e-6  # float32 L of S


def test_laplacian_entry_agrees_with_gradient_entry():
    H, W, M, N = 128, 96, 256, 192
    gx, gy = _fields(3460, 2, H, W)
    gx32, gy32 = gx.astype(np.float32), gy.astype(np.float32)
    L = _support_div(gx32.astype(np.float64), gy32.astype(np.float64)).astype(np.float32)
    u_l = gfc.solve_laplacian(torch.from_numpy(L).cuda(), M, N).cpu().numpy()
    u_g = gfc.solve(torch.from_numpy(gx32).cuda(), torch.from_numpy(gy32).cuda(), M, N).cpu().numpy()
    for i in range(2):
        assert np.linalg.norm(u_l[i] - u_g[i]) / np.linalg.norm(u_g[i]) <= TOL


def test_laplacian_solve_with_more_split_bins():
    """A plan that splits more row bins (K = 16): a given divergence has no x/y split, so the
    bins (4, K] keep the FFT values and their side entries must be zero."""
    H, W, M, N = 64, 64, 128, 128
    gx, gy = _fields(3470, 2, H, W)
    L = _support_div(gx, gy).astype(np.float32)
    p = gfc.Plan(H, W, M, N, params={"low_bins": 16}, tuned=False)
    u = p.solve_laplacian(torch.from_numpy(L).cuda()).cpu().numpy()
    for i in range(2):
        ref = O.solve_laplacian(L[i], M, N)
        assert np.linalg.norm(u[i] - ref) / np.linalg.norm(ref) <= TOL
