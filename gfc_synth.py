"""Seeded synthetic inputs for the GFC solver: the only code the oracle and the GPU path share.

This module makes inputs and nothing else. It holds none of the solver's arithmetic: no
divergence, no Green's function, no transform. Every workload here stands in for the
natural images the paper edits (Sec. 3.1.3 times an 801x1200 grey image; Sec. 3.1.4 and
Sec. 2.3.2 use the ECSSD images, which are not available here). The fields have the same
sizes, value range ([0, 1] grey levels) and smooth-plus-edges structure, and each edit
reproduces the kind of non-conservative change the paper applies to a gradient (a region
zeroed out, Sec. 3.2.3; a gradient pasted from a second image, Sec. 3.2.1 and 3.2.4).

Gradients follow eq. (1) with forward differences and a zero exterior:
    gx[y, x] = S[y, x+1] - S[y, x],  S[y, W] = 0
    gy[y, x] = S[y+1, x] - S[y, x],  S[H, x] = 0
Everything is cast to float32 exactly once; both the GPU path and the oracle consume those
float32 arrays (the oracle promotes them to float64).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

__all__ = [
    "smooth_number_at_least", "default_grid", "image_rngs", "gaussian_sum_field",
    "forward_gradient", "Workload", "make_workload", "WORKLOADS", "ragged_sizes",
]


def smooth_number_at_least(n: int, even: bool = True) -> int:
    """Smallest 2/3/5-smooth integer >= n (and even if `even`)."""
    m = max(int(n), 1)
    while True:
        if (not even or m % 2 == 0):
            r = m
            for p in (2, 3, 5):
                while r % p == 0:
                    r //= p
            if r == 1:
                return m
        m += 1


def default_grid(H: int, W: int) -> tuple[int, int]:
    """Default torus size: smallest even 2/3/5-smooth M >= max(2H, H + 2) and
    N >= max(2W, W + 2, 16) (16: the shortest row FFT of the library)."""
    return (smooth_number_at_least(max(2 * H, H + 2)),
            smooth_number_at_least(max(2 * W, W + 2, 16)))


def image_rngs(seed: int, count: int) -> list[np.random.Generator]:
    """One independent generator per image: SeedSequence(seed).spawn(count)."""
    return [np.random.default_rng(s) for s in np.random.SeedSequence(seed).spawn(count)]


def gaussian_sum_field(rng: np.random.Generator, H: int, W: int, n: int = 8) -> np.ndarray:
    """Sum of `n` isotropic Gaussians, min-max normalised to [0, 1] (float64).

    Centres ~ U[0,H) x U[0,W), sigma ~ U[0.05, 0.3] * min(H, W), amplitude ~ U[0.2, 1].
    """
    cy = rng.uniform(0.0, H, n)
    cx = rng.uniform(0.0, W, n)
    sig = rng.uniform(0.05, 0.3, n) * min(H, W)
    amp = rng.uniform(0.2, 1.0, n)
    yy = np.arange(H, dtype=np.float64)
    xx = np.arange(W, dtype=np.float64)
    S = np.zeros((H, W), dtype=np.float64)
    for i in range(n):
        gy = np.exp(-0.5 * ((yy - cy[i]) / sig[i]) ** 2)
        gx = np.exp(-0.5 * ((xx - cx[i]) / sig[i]) ** 2)
        S += amp[i] * np.outer(gy, gx)
    lo, hi = S.min(), S.max()
    return (S - lo) / (hi - lo) if hi > lo else np.zeros_like(S)


def forward_gradient(S: np.ndarray) -> tuple[np.ndarray, np.ndarray]:
    """Forward-difference gradient with a zero exterior (eq. (1)); works on [..., H, W]."""
    S = np.asarray(S, dtype=np.float64)
    gx = -S.copy()
    gx[..., :, :-1] += S[..., :, 1:]
    gy = -S.copy()
    gy[..., :-1, :] += S[..., 1:, :]
    return gx, gy


@dataclass
class Workload:
    """A batch of gradient fields (float32, [B, H, W]) plus the torus it is solved on."""
    name: str
    gx: np.ndarray
    gy: np.ndarray
    M: int
    N: int
    extra: dict = field(default_factory=dict)

    @property
    def B(self) -> int:
        return self.gx.shape[0]

    @property
    def H(self) -> int:
        return self.gx.shape[1]

    @property
    def W(self) -> int:
        return self.gx.shape[2]


def _rect_zero(rng, gx, gy, rh, rw):
    H, W = gx.shape
    y0 = int(rng.integers(0, H - rh + 1))
    x0 = int(rng.integers(0, W - rw + 1))
    gx[y0:y0 + rh, x0:x0 + rw] = 0.0
    gy[y0:y0 + rh, x0:x0 + rw] = 0.0


def _small_64(seed: int = 101):
    """64x64 field + U[0,0.05] noise; N(0, 0.01) added to gx only; 128x128 torus."""
    rng = image_rngs(seed, 1)[0]
    S = gaussian_sum_field(rng, 64, 64) + rng.uniform(0.0, 0.05, (64, 64))
    gx, gy = forward_gradient(S)
    gx = gx + rng.normal(0.0, 0.01, gx.shape)
    return Workload("gfc_64x64_on_128x128", gx[None].astype(np.float32),
                    gy[None].astype(np.float32), 128, 128, {"source": S[None]})


def _batch_801x1200(seed: int = 102, B: int = 100):
    """B x 801x1200 fields, a 200x300 gradient rectangle zeroed per image; 1620x2400 torus."""
    H, W = 801, 1200
    gx = np.empty((B, H, W), np.float32)
    gy = np.empty((B, H, W), np.float32)
    for i, rng in enumerate(image_rngs(seed, B)):
        S = gaussian_sum_field(rng, H, W)
        a, b = forward_gradient(S)
        _rect_zero(rng, a, b, 200, 300)
        gx[i] = a
        gy[i] = b
    M, N = default_grid(H, W)
    return Workload("gfc_801x1200_b100", gx, gy, M, N)


def _merge_512(seed: int = 103, pairs: int = 32):
    """Gradient merge: pairs of 3-channel 512x512 fields; inside a random ellipse each pixel
    takes image B's gradient where its magnitude is strictly larger than A's, else A's."""
    H = W = 512
    gx = np.empty((pairs * 3, H, W), np.float32)
    gy = np.empty((pairs * 3, H, W), np.float32)
    yy, xx = np.mgrid[0:H, 0:W].astype(np.float64)
    for p, rng in enumerate(image_rngs(seed, pairs)):
        cy = rng.uniform(H / 4, 3 * H / 4)
        cx = rng.uniform(W / 4, 3 * W / 4)
        a_ax = rng.uniform(64, 192)
        b_ax = rng.uniform(64, 192)
        th = rng.uniform(0.0, math.pi)
        dy, dx = yy - cy, xx - cx
        u = dx * math.cos(th) + dy * math.sin(th)
        v = -dx * math.sin(th) + dy * math.cos(th)
        mask = (u / a_ax) ** 2 + (v / b_ax) ** 2 <= 1.0
        for c in range(3):
            ax_, ay_ = forward_gradient(gaussian_sum_field(rng, H, W))
            bx_, by_ = forward_gradient(gaussian_sum_field(rng, H, W))
            take_b = mask & (bx_ ** 2 + by_ ** 2 > ax_ ** 2 + ay_ ** 2)
            gx[3 * p + c] = np.where(take_b, bx_, ax_)
            gy[3 * p + c] = np.where(take_b, by_, ay_)
    M, N = default_grid(H, W)
    return Workload("gfc_merge_512x512_b96", gx, gy, M, N)


def _layer_256(seed: int = 104, B: int = 16, C: int = 3, H: int = 256, W: int = 256,
               rect: int = 64, target_seed: int = 1104, grid=None):
    """B x C x HxW edited fields (a rect x rect gradient block zeroed), and a U[0,1] target."""
    gx = np.empty((B * C, H, W), np.float32)
    gy = np.empty((B * C, H, W), np.float32)
    for i, rng in enumerate(image_rngs(seed, B * C)):
        a, b = forward_gradient(gaussian_sum_field(rng, H, W))
        _rect_zero(rng, a, b, min(rect, H), min(rect, W))
        gx[i] = a
        gy[i] = b
    t = np.random.default_rng(target_seed).uniform(0.0, 1.0, (B * C, H, W)).astype(np.float32)
    M, N = grid if grid is not None else default_grid(H, W)
    return Workload(f"gfc_layer_{B}x{C}x{H}x{W}", gx, gy, M, N,
                    {"target": t, "shape4d": (B, C, H, W)})


def ragged_sizes(seed: int = 105, B: int = 200, lo: int = 64, hi: int = 1024):
    """Image sizes of the ragged batch: H, W ~ U{lo..hi} (inclusive)."""
    rng = np.random.default_rng(np.random.SeedSequence(seed).spawn(B + 1)[B])
    H = rng.integers(lo, hi + 1, B)
    W = rng.integers(lo, hi + 1, B)
    return [(int(h), int(w)) for h, w in zip(H, W)]


def make_ragged(seed: int = 105, B: int = 200, lo: int = 64, hi: int = 1024, sizes=None):
    """List of (gx, gy) float32 pairs of uneven sizes with a floor(H/4) x floor(W/4) edit."""
    sizes = sizes if sizes is not None else ragged_sizes(seed, B, lo, hi)
    out = []
    for (H, W), rng in zip(sizes, image_rngs(seed, len(sizes))):
        a, b = forward_gradient(gaussian_sum_field(rng, H, W))
        _rect_zero(rng, a, b, max(H // 4, 1), max(W // 4, 1))
        out.append((a.astype(np.float32), b.astype(np.float32)))
    return out


WORKLOADS = {
    "small64": _small_64,
    "batch801x1200": _batch_801x1200,
    "merge512": _merge_512,
    "layer256": _layer_256,
}


def make_workload(name: str, **kw) -> Workload:
    return WORKLOADS[name](**kw)
