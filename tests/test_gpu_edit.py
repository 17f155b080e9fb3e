"""GPU parity of the on-device gradient edits (gfc_solve_edit): thresholding (Sec. 3.2.3)
and gradient domain merging (eq. (26)) applied as the row pass loads the field, against
the float64 oracle's edit followed by its solve, on the same float32 inputs."""
import ctypes
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


def rel_l2(a, b):
    return float(np.linalg.norm(np.asarray(a, np.float64) - b) / max(np.linalg.norm(b), 1e-300))


def _fields(seed, B, H, W):
    """Gaussian-sum fields with texture: forward gradient plus N(0, 0.01) on both parts."""
    gx = np.empty((B, H, W), np.float32)
    gy = np.empty((B, H, W), np.float32)
    for i, rng in enumerate(synth.image_rngs(seed, B)):
        S = synth.gaussian_sum_field(rng, H, W)
        a, b = synth.forward_gradient(S)
        gx[i] = a + 0.01 * rng.normal(size=(H, W))
        gy[i] = b + 0.01 * rng.normal(size=(H, W))
    return gx, gy


def _edge_map(seed, B, H, W):
    return np.random.default_rng(seed).uniform(0.0, 1.0, (B, H, W)).astype(np.float32)


SHAPES = [  # H, W, M, N: narrow slots, odd sizes, minimal padding (every column block), 2400
    (64, 64, 128, 128), (31, 45, 64, 96), (100, 37, 210, 80), (33, 70, 35, 72),
    (801, 1200, 1620, 2400), (4, 1200, 10, 2400),  # thin and wide: 16 row bins split
]


def _dev(*arrs):
    return [torch.from_numpy(np.ascontiguousarray(a)).cuda() for a in arrs]


@pytest.mark.parametrize("shape", SHAPES, ids=lambda s: f"{s[0]}x{s[1]}@{s[2]}x{s[3]}")
def test_threshold_edit_matches_oracle(shape):
    H, W, M, N = shape
    B = 2 if H * W > 100000 else 3
    _say(f"[threshold] {H}x{W} on {M}x{N}, B={B}")
    gx, gy = _fields(2801 + H, B, H, W)
    mag = np.hypot(gx.astype(np.float64), gy.astype(np.float64))
    tau = float(np.quantile(mag, 0.6))
    tx, ty = _dev(gx, gy)
    u = gfc.solve_edit(tx, ty, "threshold", tau, M=M, N=N).cpu().numpy()
    for i in range(B):
        ex, ey = O.threshold_edit(gx[i], gy[i], tau)
        ref = O.solve_fft(ex, ey, M, N)
        e = rel_l2(u[i], ref)
        _say(f"  image {i}: rel. L2 {e:.3e}")
        assert e <= TOL


@pytest.mark.parametrize("shape", SHAPES, ids=lambda s: f"{s[0]}x{s[1]}@{s[2]}x{s[3]}")
@pytest.mark.parametrize("alpha", [0.5, 1.0])
def test_gdm_edit_matches_oracle(shape, alpha):
    H, W, M, N = shape
    B = 2 if H * W > 100000 else 3
    _say(f"[gdm] alpha={alpha} {H}x{W} on {M}x{N}, B={B}")
    gx, gy = _fields(2901 + H, B, H, W)
    C = _edge_map(2951 + W, B, H, W)
    tx, ty, tc = _dev(gx, gy, C)
    u = gfc.solve_edit(tx, ty, "gdm", alpha, C=tc, M=M, N=N).cpu().numpy()
    for i in range(B):
        ex, ey = O.gdm_edit(gx[i], gy[i], C[i], alpha)
        ref = O.solve_fft(ex, ey, M, N)
        e = rel_l2(u[i], ref)
        _say(f"  image {i}: rel. L2 {e:.3e}")
        assert e <= TOL


@pytest.mark.parametrize("shape", [(64, 64, 128, 128), (801, 1200, 1620, 2400)],
                         ids=lambda s: f"{s[0]}x{s[1]}")
def test_identity_edits_equal_the_plain_solve(shape):
    """tau = 0 keeps every pixel and alpha = 0 keeps every magnitude: the plain solve."""
    H, W, M, N = shape
    gx, gy = _fields(3001, 2, H, W)
    C = _edge_map(3002, 2, H, W)
    tx, ty, tc = _dev(gx, gy, C)
    plain = gfc.solve(tx, ty, M, N)
    a = gfc.solve_edit(tx, ty, "threshold", 0.0, M=M, N=N)
    b = gfc.solve_edit(tx, ty, "gdm", 0.0, C=tc, M=M, N=N)
    scale = float(plain.abs().max())
    assert float((a - plain).abs().max()) <= 1e-6 * scale
    assert float((b - plain).abs().max()) <= 1e-6 * scale


def test_threshold_with_colour_correction_matches_oracle():
    """The paper's editing pipeline: threshold at a level, solve, correct to the source."""
    H, W, M, N = 128, 160, 256, 320
    B = 2
    gx = np.empty((B, H, W), np.float32)
    gy = np.empty((B, H, W), np.float32)
    means = np.empty(B, np.float32)
    stds = np.empty(B, np.float32)
    for i, rng in enumerate(synth.image_rngs(3101, B)):
        S = synth.gaussian_sum_field(rng, H, W) + 0.02 * rng.normal(size=(H, W))
        gx[i], gy[i] = synth.forward_gradient(S)
        means[i], stds[i] = S.mean(), S.std()
    tau = 0.1 * float(np.hypot(gx, gy).max())  # 10% of the largest gradient present
    tx, ty, tm, ts = _dev(gx, gy, means, stds)
    out = gfc.solve_edit(tx, ty, "threshold", tau, I_mean=tm, I_std=ts, M=M, N=N).cpu().numpy()
    for i in range(B):
        ex, ey = O.threshold_edit(gx[i], gy[i], tau)
        u_ref = O.solve_fft(ex, ey, M, N)
        ref = O.color_correct(u_ref, means[i], stds[i])
        tol = TOL * np.linalg.norm(u_ref) / np.linalg.norm(u_ref - u_ref.mean()) + 1e-6
        e = np.linalg.norm(out[i] - ref) / np.linalg.norm(ref - means[i])
        _say(f"  image {i}: centred rel. L2 {e:.3e} (bar {tol:.3e})")
        assert e <= tol


def test_edit_argument_checks():
    L = gfc.lib()
    p = gfc.Plan(16, 16, 40, 40).build("cuda:0")
    g = torch.zeros((1, 16, 16), device="cuda:0")
    ws = torch.empty(p.workspace_size(1), dtype=torch.uint8, device="cuda:0")
    args = lambda mode, param, C: (p.handle, g.data_ptr(), g.data_ptr(), C, mode,  # noqa: E731
                                   ctypes.c_float(param), None, None, g.data_ptr(), 1,
                                   ws.data_ptr(), ws.numel(), None)
    assert L.gfc_solve_edit(*args(3, 0.5, g.data_ptr())) == 1      # unknown mode
    assert L.gfc_solve_edit(*args(2, 1.5, g.data_ptr())) == 1      # alpha outside [0, 1]
    assert L.gfc_solve_edit(*args(2, 0.5, None)) == 1              # GDM needs C
    assert L.gfc_solve_edit(*args(1, -1.0, None)) == 1             # negative tau
    with pytest.raises(ValueError):
        gfc.solve_edit(g, g, "blur", 1.0)
