"""GPU parity of the colour-preserving correction of eq. (25) (gfc_solve_batch_color):
the HIP path against the float64 oracle's solve followed by its color_correct, on the same
float32 inputs and the same source statistics."""
import sys

import numpy as np
import pytest

import gfc_synth as synth
import oracle as O

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import paper_1902_00176_amd as gfc  # noqa: E402

EPS32 = 2.0 ** -24


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _edited_sources(seed, B, H, W, rect):
    """Gaussian-sum sources S, their gradients with a zeroed rectangle, and S's statistics."""
    gx = np.empty((B, H, W), np.float32)
    gy = np.empty((B, H, W), np.float32)
    means = np.empty(B, np.float32)
    stds = np.empty(B, np.float32)
    for i, rng in enumerate(synth.image_rngs(seed, B)):
        S = synth.gaussian_sum_field(rng, H, W)
        a, b = synth.forward_gradient(S)
        rh, rw = min(rect[0], H), min(rect[1], W)
        y0 = int(rng.integers(0, H - rh + 1))
        x0 = int(rng.integers(0, W - rw + 1))
        a[y0:y0 + rh, x0:x0 + rw] = 0.0
        b[y0:y0 + rh, x0:x0 + rw] = 0.0
        gx[i], gy[i] = a, b
        means[i], stds[i] = S.mean(), S.std()
    return gx, gy, means, stds


def _run(gx, gy, means, stds, M, N):
    dev = torch.device("cuda:0")
    tx, ty = torch.from_numpy(gx).to(dev), torch.from_numpy(gy).to(dev)
    tm, ts = torch.from_numpy(means).to(dev), torch.from_numpy(stds).to(dev)
    out = gfc.solve_color(tx, ty, tm, ts, M, N)
    u = gfc.solve(tx, ty, M, N)
    torch.cuda.synchronize()
    return out.cpu().numpy().astype(np.float64), u.cpu().numpy().astype(np.float64)


CASES = [  # seed, B, H, W, M, N, edit rectangle
    (2601, 1, 64, 64, 128, 128, (16, 16)),
    (2602, 3, 31, 45, 64, 96, (8, 11)),
    (2603, 2, 100, 37, 210, 80, (30, 9)),
    (2604, 2, 801, 1200, 1620, 2400, (200, 300)),
]


@pytest.mark.parametrize("case", CASES, ids=lambda c: f"{c[2]}x{c[3]}_b{c[1]}")
def test_color_corrected_solve_matches_oracle(case):
    seed, B, H, W, M, N, rect = case
    _say(f"[color] {H}x{W} on {M}x{N}, B={B}")
    gx, gy, means, stds = _edited_sources(seed, B, H, W, rect)
    out, u_gpu = _run(gx, gy, means, stds, M, N)
    for i in range(B):
        # 1) the correction arithmetic, on the GPU's own uncorrected solve: float32 rounding only
        ref_own = O.color_correct(u_gpu[i], means[i], stds[i])
        ratio = float(stds[i]) / u_gpu[i].std()
        bound = 8 * EPS32 * (np.max(np.abs(ref_own)) + ratio * abs(u_gpu[i].mean()))
        assert np.max(np.abs(out[i] - ref_own)) <= bound, (i, np.max(np.abs(out[i] - ref_own)), bound)
        # 2) against the oracle end to end: the forward bar (1e-5 relative L2 of u), carried
        # through the affine map, relative to the corrected image's spread about its mean
        u_ref = O.solve_fft(gx[i], gy[i], M, N)
        ref = O.color_correct(u_ref, means[i], stds[i])
        spread = np.linalg.norm(ref - means[i])
        tol = 1e-5 * np.linalg.norm(u_ref) / np.linalg.norm(u_ref - u_ref.mean()) + 1e-6
        err = np.linalg.norm(out[i] - ref) / spread
        _say(f"  image {i}: centred rel. L2 {err:.3e} (bar {tol:.3e})")
        assert err <= tol
        assert abs(out[i].mean() - means[i]) <= 1e-5 * max(1.0, abs(float(means[i])))
        assert abs(out[i].std() - stds[i]) <= 1e-5 * float(stds[i])


def test_color_correction_of_a_zero_gradient_is_the_source_mean():
    """A zero field solves to a constant: no contrast to rescale, the output is mean(I)."""
    H, W = 40, 50
    gx = np.zeros((2, H, W), np.float32)
    out, _ = _run(gx, gx.copy(), np.array([0.3, 0.8], np.float32),
                  np.array([0.1, 0.2], np.float32), 0, 0)
    assert np.all(out[0] == np.float32(0.3)) and np.all(out[1] == np.float32(0.8))


def test_color_entry_rejects_mismatched_statistics():
    dev = torch.device("cuda:0")
    g = torch.zeros((3, 16, 16), device=dev)
    with pytest.raises(ValueError):
        gfc.solve_color(g, g, torch.zeros(2, device=dev), torch.ones(2, device=dev))
