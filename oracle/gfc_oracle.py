"""Plain, slow, float64 CPU oracle for the Green Function Convolution (GFC) solve.

TEST INFRASTRUCTURE ONLY. Nothing in the product path may import or call this module;
only tests, the smoke check and the benchmark's CPU-baseline leg use it. It shares no code
with the HIP path and reads nothing the HIP path writes.

What it computes (block-centred convention of Algorithm A/B):

* The torus is Z_M x Z_N. An H x W gradient field (gx, gy) is embedded at offset
  (oy, ox) = (floor((M-H)/2), floor((N-W)/2)) in zeros (the padding of Sec. 2.3.2).
* L = div E with backward differences on the torus (eq. (3)):
      L[y,x] = Ex[y,x] - Ex[y,x-1] + Ey[y,x] - Ey[y-1,x]          (indices mod M, N)
* Green's spectrum (eqs. (19)-(22), Algorithm A): G^ = F(dirac) / F(laplace), the impulse
  at the centre of a 3 x 3 five-point stencil padded to the torus; this equals 1/lambda with
      lambda(k,l) = -4 sin^2(pi k/M) - 4 sin^2(pi l/N).
  Readings taken where the paper is silent or inconsistent:
    - stencil sign: Algorithm A's +Laplacian ([[0,1,0],[1,-4,1],[0,1,0]]), the sign for
      which L = div E reconstructs +I; eq. (15) prints the negated kernel;
    - DC bin: lambda(0,0) = 0 makes Algorithm A divide by zero; G^(0,0) := 0 (the
      pseudo-inverse). The result does not depend on it: sum(L) = 0 exactly on the torus.
* v = R(F^-1(F(L) o G^)) (eq. (23)); u = v[block] - v[0,0] (Algorithm B's constant and
  crop; v[0,0] lies in the zero padding, Sec. 2.3.2's choice of c).
* Backward (adjoint of the linear map (gx, gy) -> u):
      r = embed(du) - sum(du) * delta_(0,0),  w = g (*) r  (g is real and even),
      dgx = -(w[y,x+1] - w[y,x]),  dgy = -(w[y+1,x] - w[y,x])   on the block.

Three independent forward implementations are given so they can check one another:
`solve_fft` (numpy/scipy FFT, the reference for GPU parity), `solve_direct` (explicit DFT
matrices and a literal circular convolution, tiny grids only) and `lstsq_torus` (dense least
squares of the torus gradient system, the optimality statement of Sec. 2.2, tiny grids).
"""
from __future__ import annotations

import os

import numpy as np
import scipy.fft as sfft

__all__ = [
    "block_offset", "laplacian_symbol", "green_spectrum", "green_spectrum_eq22",
    "embed", "divergence", "solve_fft", "solve_direct", "lstsq_torus", "torus_gradient",
    "solve_backward", "green_function", "cpu_workers", "color_correct", "threshold_edit",
    "gdm_edit", "solve_laplacian", "block_offset3", "green_spectrum3", "solve3_fft",
    "lstsq_torus3",
]


def cpu_workers() -> int:
    try:
        return len(os.sched_getaffinity(0))
    except AttributeError:  # pragma: no cover
        return os.cpu_count() or 1


def block_offset(H: int, W: int, M: int, N: int) -> tuple[int, int]:
    """Offset of the image block in the torus: centred, floor((M-H)/2), floor((N-W)/2)."""
    if M < H + 2 or N < W + 2:
        raise ValueError("torus must exceed the image by at least 2 in each direction")
    return (M - H) // 2, (N - W) // 2


def laplacian_symbol(M: int, N: int) -> np.ndarray:
    """lambda(k,l) of the +5-point Laplacian on Z_M x Z_N, shape [M, N], float64."""
    k = np.arange(M, dtype=np.float64)
    l = np.arange(N, dtype=np.float64)
    a = -4.0 * np.sin(np.pi * k / M) ** 2
    b = -4.0 * np.sin(np.pi * l / N) ** 2
    return a[:, None] + b[None, :]


def green_spectrum(M: int, N: int) -> np.ndarray:
    """Numerical Green's spectrum G^ = 1/lambda, G^(0,0) = 0 (eq. (22) in closed form)."""
    lam = laplacian_symbol(M, N)
    G = np.zeros_like(lam)
    nz = lam != 0.0
    G[nz] = 1.0 / lam[nz]
    return G


def green_spectrum_eq22(M: int, N: int, kernel=None, dirac_pos=(1, 1)) -> np.ndarray:
    """Eq. (19) on the M x N torus with the zero-padded kernels of eqs. (20)-(21): the
    discrete Fourier transform of a unit impulse at `dirac_pos` divided by that of a 3 x 3
    stencil whose top-left tap sits at the grid origin.

    Both transforms are written as their finite sums: the impulse contributes the single
    phase e^{-2 pi i (k a / M + l b / N)} of its position (a, b), and the stencil the sum of
    its nine taps times their phases (its symbol). No padded array is transformed. With the
    stencil centred on the impulse the phases cancel and the ratio is real: 1/lambda.
    `kernel` defaults to the +5-point Laplacian (Algorithm A's sign, the stencil-sign
    reading of the module header); the DC bin, where the symbol vanishes, is set to 0. Returns the complex spectrum [M, N]."""
    if kernel is None:
        kernel = np.array([[0.0, 1.0, 0.0], [1.0, -4.0, 1.0], [0.0, 1.0, 0.0]])
    kernel = np.asarray(kernel, dtype=np.float64)
    fk = np.arange(M, dtype=np.float64)[:, None] / M
    fl = np.arange(N, dtype=np.float64)[None, :] / N

    def phase(a, b):
        return np.exp(-2j * np.pi * (fk * a + fl * b))

    symbol = np.zeros((M, N), dtype=np.complex128)
    for a in range(kernel.shape[0]):
        for b in range(kernel.shape[1]):
            if kernel[a, b] != 0.0:
                symbol += kernel[a, b] * phase(a, b)
    num = phase(*dirac_pos)
    out = np.zeros((M, N), dtype=np.complex128)
    nz = np.abs(symbol) > 1e-300
    out[nz] = num[nz] / symbol[nz]
    return out


def green_function(M: int, N: int) -> np.ndarray:
    """Spatial Green's function g = F^-1(G^) (real, even), shape [M, N]."""
    return np.real(np.fft.ifft2(green_spectrum(M, N)))


def embed(a: np.ndarray, M: int, N: int, oy: int, ox: int) -> np.ndarray:
    """Zero-padded copy of a [..., H, W] array at offset (oy, ox) of an [..., M, N] torus."""
    a = np.asarray(a, dtype=np.float64)
    H, W = a.shape[-2:]
    out = np.zeros(a.shape[:-2] + (M, N), dtype=np.float64)
    out[..., oy:oy + H, ox:ox + W] = a
    return out


def divergence(gx, gy, M: int, N: int, oy: int, ox: int) -> np.ndarray:
    """L = div E of the embedded field with backward differences on the torus (eq. (3))."""
    Ex = embed(gx, M, N, oy, ox)
    Ey = embed(gy, M, N, oy, ox)
    return (Ex - np.roll(Ex, 1, axis=-1)) + (Ey - np.roll(Ey, 1, axis=-2))


def _as_batch(a):
    a = np.asarray(a, dtype=np.float64)
    return (a[None], True) if a.ndim == 2 else (a, False)


def solve_fft(gx, gy, M: int, N: int, workers: int | None = None) -> np.ndarray:
    """Forward GFC solve in float64 via library FFTs: eq. (23) and Algorithm B.

    gx, gy: [H, W] or [B, H, W] (float32 inputs are promoted exactly). Returns u like gx.
    """
    gx, single = _as_batch(gx)
    gy, _ = _as_batch(gy)
    B, H, W = gx.shape
    oy, ox = block_offset(H, W, M, N)
    Gh = green_spectrum(M, N)[:, : N // 2 + 1]
    w = workers if workers is not None else cpu_workers()
    out = np.empty((B, H, W), dtype=np.float64)
    for b in range(B):
        L = divergence(gx[b], gy[b], M, N, oy, ox)
        v = sfft.irfft2(sfft.rfft2(L, workers=w) * Gh, s=(M, N), workers=w)
        out[b] = v[oy:oy + H, ox:ox + W] - v[0, 0]
    return out[0] if single else out


def _dft_matrix(n: int, sign: float) -> np.ndarray:
    j = np.arange(n)
    return np.exp(sign * 2j * np.pi * np.outer(j, j) / n)


def solve_direct(gx, gy, M: int, N: int) -> np.ndarray:
    """Forward solve with no FFT: g from explicit inverse-DFT matrices applied to the closed
    form G^, then a literal circular convolution of L over its support (eq. (4)).
    Cost O(M N (H+1) (W+1)); intended for grids of at most ~128 x 128."""
    gx, single = _as_batch(gx)
    gy, _ = _as_batch(gy)
    B, H, W = gx.shape
    oy, ox = block_offset(H, W, M, N)
    Fm = _dft_matrix(M, +1.0)
    Fn = _dft_matrix(N, +1.0)
    g = np.real(Fm @ green_spectrum(M, N) @ Fn.T) / (M * N)
    out = np.empty((B, H, W))
    yy = np.arange(M)[:, None]
    xx = np.arange(N)[None, :]
    for b in range(B):
        L = divergence(gx[b], gy[b], M, N, oy, ox)
        v = np.zeros((M, N))
        for qy, qx in zip(*np.nonzero(L)):
            v += L[qy, qx] * g[(yy - qy) % M, (xx - qx) % N]
        out[b] = v[oy:oy + H, ox:ox + W] - v[0, 0]
    return out[0] if single else out


def torus_gradient(M: int, N: int) -> np.ndarray:
    """Dense forward-difference gradient matrix D (2MN x MN) on Z_M x Z_N; rows [Dx; Dy]."""
    n = M * N
    idx = np.arange(n).reshape(M, N)
    D = np.zeros((2 * n, n))
    r = np.arange(n)
    D[r, idx.ravel()] -= 1.0
    D[r, np.roll(idx, -1, axis=1).ravel()] += 1.0
    D[n + r, idx.ravel()] -= 1.0
    D[n + r, np.roll(idx, -1, axis=0).ravel()] += 1.0
    return D


def lstsq_torus(gx, gy, M: int, N: int) -> np.ndarray:
    """argmin_v ||D v - E||^2 on the torus by dense least squares (the optimality statement
    of Sec. 2.2, eqs. (8)-(14)), then Algorithm B's constant and crop. Tiny grids only."""
    gx = np.asarray(gx, dtype=np.float64)
    gy = np.asarray(gy, dtype=np.float64)
    H, W = gx.shape
    oy, ox = block_offset(H, W, M, N)
    E = np.concatenate([embed(gx, M, N, oy, ox).ravel(), embed(gy, M, N, oy, ox).ravel()])
    v, *_ = np.linalg.lstsq(torus_gradient(M, N), E, rcond=None)
    v = v.reshape(M, N)
    return v[oy:oy + H, ox:ox + W] - v[0, 0]


def solve_backward(du, M: int, N: int, workers: int | None = None):
    """Adjoint of the forward solve: returns (dgx, dgy) with the shape of du."""
    du, single = _as_batch(du)
    B, H, W = du.shape
    oy, ox = block_offset(H, W, M, N)
    Gh = green_spectrum(M, N)[:, : N // 2 + 1]
    wk = workers if workers is not None else cpu_workers()
    dgx = np.empty((B, H, W))
    dgy = np.empty((B, H, W))
    for b in range(B):
        r = embed(du[b], M, N, oy, ox)
        r[0, 0] -= du[b].sum()
        w = sfft.irfft2(sfft.rfft2(r, workers=wk) * Gh, s=(M, N), workers=wk)
        gxf = -(np.roll(w, -1, axis=1) - w)
        gyf = -(np.roll(w, -1, axis=0) - w)
        dgx[b] = gxf[oy:oy + H, ox:ox + W]
        dgy[b] = gyf[oy:oy + H, ox:ox + W]
    if single:
        return dgx[0], dgy[0]
    return dgx, dgy


def color_correct(u, I_mean, I_std) -> np.ndarray:
    """Colour-preserving correction of eq. (25), per image over its H x W crop:
        I_corr = (I_c - mean(I_c)) * sigma(I) / sigma(I_c) + mean(I).
    u: [..., H, W] solved images I_c; I_mean, I_std: mean and standard deviation of each
    source image I (one value per leading index). sigma is the population standard
    deviation. The ratio sigma(I) / sigma(I_c) is the same for any normalisation common to
    both (n or n - 1), so only I_std has to use the same one. Where the paper is silent: a
    constant I_c (sigma(I_c) = 0) has no contrast to rescale, and its output is mean(I)."""
    u = np.asarray(u, dtype=np.float64)
    flat = u.reshape(-1, u.shape[-2] * u.shape[-1])
    means = np.asarray(I_mean, dtype=np.float64).reshape(-1)
    stds = np.asarray(I_std, dtype=np.float64).reshape(-1)
    if means.size != flat.shape[0] or stds.size != flat.shape[0]:
        raise ValueError("one mean and one standard deviation per image")
    out = np.empty_like(flat)
    for i in range(flat.shape[0]):
        mu = flat[i].mean()
        sd = np.sqrt(np.mean((flat[i] - mu) ** 2))
        ratio = stds[i] / sd if sd > 0 else 0.0
        out[i] = (flat[i] - mu) * ratio + means[i]
    return out.reshape(u.shape)


def threshold_edit(gx, gy, tau: float):
    """Gradient thresholding of Sec. 3.2.3: the gradient E = (gx, gy) of a pixel is kept
    where its magnitude reaches tau and set to 0 elsewhere, which removes texture and fine
    elements and keeps strong edges. The paper thresholds at 10% of the highest possible
    gradient; here tau is that absolute level, chosen by the caller.

    The keep/drop decision is an integer outcome of floating-point arithmetic, so it is taken
    in float32, the precision of the inputs and of the GPU path, in this order:
    m = fl(fl(gx*gx) + fl(gy*gy)) compared with t = fl(tau*tau) (tau rounded to float32
    first), keep when m >= t. The kept values are exact."""
    gx = np.asarray(gx, dtype=np.float32)
    gy = np.asarray(gy, dtype=np.float32)
    t = np.float32(np.float32(tau) * np.float32(tau))
    m = (gx * gx) + (gy * gy)  # float32 products and sum, each rounded once
    keep = m >= t
    return (np.where(keep, gx, np.float32(0)).astype(np.float64),
            np.where(keep, gy, np.float32(0)).astype(np.float64))


def gdm_edit(gx, gy, C, alpha: float):
    """Gradient domain merging, eq. (26): the perturbed field keeps the orientation of E and
    takes the weighted geometric mean of the magnitudes, |E_p| = |E|^(1-alpha) * C^alpha, with
    C >= 0 the edge intensity of each pixel and alpha in [0, 1]. Where |E| = 0 the orientation
    is undefined and E_p = 0 (the paper is silent there). float64."""
    gx = np.asarray(gx, dtype=np.float64)
    gy = np.asarray(gy, dtype=np.float64)
    C = np.asarray(C, dtype=np.float64)
    mag = np.hypot(gx, gy)
    nz = mag > 0
    safe = np.where(nz, mag, 1.0)
    scale = np.where(nz, safe ** (-alpha) * C ** alpha, 0.0)
    return gx * scale, gy * scale


def solve_laplacian(L, M: int, N: int, workers: int | None = None) -> np.ndarray:
    """Algorithm B with its literal input: the Laplacian itself rather than a gradient field.

    L: [H+1, W+1] or [B, H+1, W+1], the support of the Laplacian of an H x W image whose
    first row and column are zero (the paper pads before differentiating), i.e. the same
    support as div E for H x W forward-difference fields. It is embedded at the block offset
    (oy, ox) of the H x W image, v = R(F^-1(F(L) o G^)) (eq. (23)), u = v[block] - v[0,0].
    The torus solve only sees L up to its mean (G^(0,0) = 0); L is expected to sum to 0, as
    every divergence and every Laplacian of a zero-padded field does. Returns [.., H, W]."""
    L, single = _as_batch(L)
    B, H1, W1 = L.shape
    H, W = H1 - 1, W1 - 1
    oy, ox = block_offset(H, W, M, N)
    Gh = green_spectrum(M, N)[:, : N // 2 + 1]
    w = workers if workers is not None else cpu_workers()
    out = np.empty((B, H, W), dtype=np.float64)
    for b in range(B):
        Lt = embed(L[b], M, N, oy, ox)
        v = sfft.irfft2(sfft.rfft2(Lt, workers=w) * Gh, s=(M, N), workers=w)
        out[b] = v[oy:oy + H, ox:ox + W] - v[0, 0]
    return out[0] if single else out


# ---------------------------------------------------------------- n-D (three dimensions)
# The method holds in any dimension (eq. (5) and Sec. 2): the Green's function of the
# discrete Laplacian on a P x M x N torus has the spectrum 1 / lambda with
#     lambda(kz, ky, kx) = -4 sin^2(pi kz/P) - 4 sin^2(pi ky/M) - 4 sin^2(pi kx/N),
# the 7-point stencil's symbol, and the same readings apply: G^(0,0,0) = 0, the block is
# centred, the constant is the value at the grid corner (0,0,0). Volumes are [D, H, W]
# (z, y, x); the gradient is (gx, gy, gz) with forward differences and a zero exterior.

def block_offset3(D: int, H: int, W: int, P: int, M: int, N: int):
    if P < D + 2 or M < H + 2 or N < W + 2:
        raise ValueError("torus must exceed the volume by at least 2 in each direction")
    return (P - D) // 2, (M - H) // 2, (N - W) // 2


def green_spectrum3(P: int, M: int, N: int) -> np.ndarray:
    """1 / lambda on the P x M x N torus, 0 at the DC bin."""
    lz = -4.0 * np.sin(np.pi * np.arange(P) / P) ** 2
    ly = -4.0 * np.sin(np.pi * np.arange(M) / M) ** 2
    lx = -4.0 * np.sin(np.pi * np.arange(N) / N) ** 2
    lam = lz[:, None, None] + ly[None, :, None] + lx[None, None, :]
    G = np.zeros_like(lam)
    nz = lam != 0
    G[nz] = 1.0 / lam[nz]
    return G


def _divergence3(gx, gy, gz, P, M, N, o):
    E = []
    for g in (gx, gy, gz):
        t = np.zeros((P, M, N))
        D, H, W = g.shape
        t[o[0]:o[0] + D, o[1]:o[1] + H, o[2]:o[2] + W] = g
        E.append(t)
    return ((E[0] - np.roll(E[0], 1, axis=2)) + (E[1] - np.roll(E[1], 1, axis=1))
            + (E[2] - np.roll(E[2], 1, axis=0)))


def solve3_fft(gx, gy, gz, P: int, M: int, N: int, workers: int | None = None) -> np.ndarray:
    """Three-dimensional GFC of one volume: L = div E (7-point, backward differences on the
    torus), v = R(F^-1(F(L) o G^)), u = v[block] - v[0,0,0]. float64, library FFTs."""
    gx = np.asarray(gx, dtype=np.float64)
    gy = np.asarray(gy, dtype=np.float64)
    gz = np.asarray(gz, dtype=np.float64)
    D, H, W = gx.shape
    o = block_offset3(D, H, W, P, M, N)
    L = _divergence3(gx, gy, gz, P, M, N, o)
    w = workers if workers is not None else cpu_workers()
    G = green_spectrum3(P, M, N)[:, :, : N // 2 + 1]
    v = sfft.irfftn(sfft.rfftn(L, workers=w) * G, s=(P, M, N), workers=w)
    return v[o[0]:o[0] + D, o[1]:o[1] + H, o[2]:o[2] + W] - v[0, 0, 0]


def lstsq_torus3(gx, gy, gz, P: int, M: int, N: int) -> np.ndarray:
    """Dense least squares of the 3-D torus gradient system (Sec. 2.2 in three dimensions),
    minimum-norm solution aligned to the same corner constant. Tiny tori only."""
    gx = np.asarray(gx, dtype=np.float64)
    D, H, W = gx.shape
    o = block_offset3(D, H, W, P, M, N)
    n = P * M * N
    idx = np.arange(n).reshape(P, M, N)
    rows = []
    for ax in (2, 1, 0):  # x, y, z forward differences
        Dm = np.zeros((n, n))
        nb = np.roll(idx, -1, axis=ax)
        Dm[idx.ravel(), nb.ravel()] += 1.0
        Dm[idx.ravel(), idx.ravel()] -= 1.0
        rows.append(Dm)
    A = np.vstack(rows)
    E = []
    for g in (gx, gy, gz):
        t = np.zeros((P, M, N))
        t[o[0]:o[0] + D, o[1]:o[1] + H, o[2]:o[2] + W] = g
        E.append(t.ravel())
    v = np.linalg.lstsq(A, np.concatenate(E), rcond=None)[0].reshape(P, M, N)
    return v[o[0]:o[0] + D, o[1]:o[1] + H, o[2]:o[2] + W] - v[0, 0, 0]
