"""Pins for the float64 oracle: each test ties it to something other than itself.

The paper prints no worked numeric example, so the pins are the paper's printed kernels
(tests/golden/paper_kernels.json), a hand-derived 4x4 spectrum (tests/golden/green_4x4_hand.json),
identities the paper states (eqs. (4), (8)-(14), (16), (22), (23)), brute force on tiny grids
and closed-form asymptotics (eq. (5)). Three forward implementations of different construction
(library FFT, explicit DFT matrices plus literal convolution, dense least squares) must agree.
"""
import json
import math
import os

import numpy as np
import pytest

import gfc_synth as synth
import oracle as O

pytestmark = pytest.mark.filterwarnings("ignore::RuntimeWarning")


def _load(golden_dir, name):
    with open(os.path.join(golden_dir, name)) as f:
        return json.load(f)


def _rand_field(rng, H, W):
    return rng.normal(size=(H, W)), rng.normal(size=(H, W))


def _framed_conservative(rng, H, W):
    """Image with zero first row and first column (padding taken before the gradient,
    Sec. 2.3.2) and its forward-difference gradient with zero exterior."""
    S = synth.gaussian_sum_field(rng, H, W) + 0.1 * rng.normal(size=(H, W))
    S[0, :] = 0.0
    S[:, 0] = 0.0
    gx, gy = synth.forward_gradient(S)
    return S, gx, gy


# ---------------------------------------------------------------- Green's spectrum (A0)

@pytest.mark.parametrize("M,N", [(12, 10), (16, 16), (9, 14), (30, 24)])
def test_closed_form_equals_eq22_with_printed_kernels(golden_dir, M, N):
    k = _load(golden_dir, "paper_kernels.json")
    lap = np.array(k["algorithm_a_laplace"]["value"], dtype=float)
    pos = tuple(k["algorithm_a_dirac_position"]["value"])
    Ga = O.green_spectrum_eq22(M, N, kernel=lap, dirac_pos=pos)
    Gc = O.green_spectrum(M, N)
    mask = np.ones((M, N), bool)
    mask[0, 0] = False
    assert np.max(np.abs(Ga.imag[mask])) < 1e-12
    rel = np.abs(Ga.real[mask] - Gc[mask]) / np.abs(Gc[mask])
    assert rel.max() < 1e-12
    # Algorithm A's literal division is 1/0 at DC: the oracle's DC reading is 0.
    assert Gc[0, 0] == 0.0


def _algorithm_b_literal(gx, gy, pad, lap, pos):
    """Algorithms A and B step by step: the field padded by `pad` on each side at explicit
    indices, its divergence pixel by pixel (backward differences on the torus, eq. (3)), the
    eq. (22) spectrum of the given kernels, a complex 2-D FFT solve, the corner subtracted,
    [pad:-pad, pad:-pad] kept."""
    H, W = gx.shape
    M, N = H + 2 * pad, W + 2 * pad
    Ex = np.zeros((M, N))
    Ey = np.zeros((M, N))
    Ex[pad:pad + H, pad:pad + W] = gx
    Ey[pad:pad + H, pad:pad + W] = gy
    padded_L = np.zeros((M, N))
    for y in range(M):
        for x in range(N):
            padded_L[y, x] = (Ex[y, x] - Ex[y, x - 1]) + (Ey[y, x] - Ey[y - 1, x])
    green_F = O.green_spectrum_eq22(M, N, kernel=lap, dirac_pos=pos)
    I = np.fft.ifft2(np.fft.fft2(padded_L) * green_F)
    assert np.max(np.abs(I.imag)) < 1e-12 * np.max(np.abs(I.real))
    I = I.real - I.real[0, 0]
    return I[pad:-pad, pad:-pad], padded_L, green_F


@pytest.mark.parametrize("H,W,pad", [(56, 72, 4), (7, 10, 4), (20, 31, 3)])
def test_block_offset_is_algorithm_b_pad(golden_dir, H, W, pad):
    """Algorithm A pads the image by `pad` on every side and Algorithm B crops
    [pad:-pad, pad:-pad]: on a torus of H + 2 pad by W + 2 pad the block sits at (pad, pad)."""
    assert O.block_offset(H, W, H + 2 * pad, W + 2 * pad) == (pad, pad)
    k = _load(golden_dir, "paper_kernels.json")
    if pad == k["algorithm_a_pad"]["value"]:
        assert (H + 8, W + 8) == (H + 2 * pad, W + 2 * pad)


def test_block_offset_floor_on_odd_margins():
    """Reading of the crop for an odd margin M - H (the 801 x 1200 workload on 1620 x 2400):
    the block starts at floor((M - H) / 2), so the larger half of the padding is below it."""
    assert O.block_offset(801, 1200, 1620, 2400) == (409, 600)
    assert O.block_offset(5, 6, 8, 9) == (1, 1)


@pytest.mark.parametrize("H,W", [(56, 72), (12, 22)])
def test_algorithm_a_and_b_run_literally_with_pad_4(golden_dir, H, W):
    """Algorithms A and B taken step by step with their pad of 4 on a non-conservative field:
    the spectrum of eq. (22) from the printed kernels, the divergence of the field padded by
    4 pixels on each side (explicit indices, not block_offset), a full complex 2-D FFT solve,
    the corner value subtracted and [4:-4, 4:-4] kept. The oracle's solve on the
    (H + 8) x (W + 8) torus must agree, which fixes its block placement and its constant."""
    k = _load(golden_dir, "paper_kernels.json")
    pad = k["algorithm_a_pad"]["value"]
    lap = np.array(k["algorithm_a_laplace"]["value"], dtype=float)
    pos = tuple(k["algorithm_a_dirac_position"]["value"])
    M, N = H + 2 * pad, W + 2 * pad
    rng = np.random.default_rng(4004 + H)
    gx, gy = _rand_field(rng, H, W)
    I, padded_L, green_F = _algorithm_b_literal(gx, gy, pad, lap, pos)
    ref = O.solve_fft(gx, gy, M, N)
    assert np.max(np.abs(I - ref)) < 1e-11 * max(1.0, np.abs(ref).max())
    # the corner matters for a non-conservative field: a block one row lower changes u
    shifted = np.fft.ifft2(np.fft.fft2(np.roll(padded_L, 1, axis=0)) * green_F).real
    shifted = (shifted - shifted[0, 0])[pad + 1:M - pad + 1, pad:-pad]
    assert np.max(np.abs(shifted - ref)) > 1e-6  # far above the 1e-11 agreement


def test_green_4x4_hand_derived(golden_dir):
    g = _load(golden_dir, "green_4x4_hand.json")
    expect = np.array([[n / d for n, d in row] for row in g["G_hat_numerator_over_denominator"]])
    assert np.allclose(O.green_spectrum(4, 4), expect, rtol=0, atol=1e-15)
    n, d = g["g00_num_den"]
    assert abs(O.green_function(4, 4)[0, 0] - n / d) < 1e-15


@pytest.mark.parametrize("M,N", [(6, 8), (7, 5)])
def test_green_function_is_pseudo_inverse_of_dense_laplacian(M, N):
    """Brute force: g = pinv(Laplacian matrix) applied to a Dirac (no FFT involved)."""
    D = O.torus_gradient(M, N)
    lap = -(D.T @ D)  # +5-point Laplacian as a dense MN x MN matrix
    e0 = np.zeros(M * N)
    e0[0] = 1.0
    g_brute = (np.linalg.pinv(lap) @ e0).reshape(M, N)
    assert np.max(np.abs(O.green_function(M, N) - g_brute)) < 1e-12


def test_discrete_green_identity_eq16():
    """K (*) g = delta - 1/(MN): eq. (16) on the torus with the DC projection."""
    M, N = 64, 48
    g = O.green_function(M, N)
    lap_g = (np.roll(g, 1, 0) + np.roll(g, -1, 0) + np.roll(g, 1, 1) + np.roll(g, -1, 1) - 4 * g)
    target = -np.full((M, N), 1.0 / (M * N))
    target[0, 0] += 1.0
    assert np.max(np.abs(lap_g - target)) < 1e-12
    assert np.max(np.abs(g - g[(-np.arange(M)) % M][:, (-np.arange(N)) % N])) < 1e-14  # even


def test_far_field_matches_eq5_logarithm(golden_dir):
    """Away from the source, g behaves like ln(r)/S_1 (eq. (5)-(6), n = 2), with the sign that
    goes with Algorithm A's +Laplacian (reading of the stencil sign)."""
    s2 = _load(golden_dir, "paper_kernels.json")["eq6_surface_2d"]["value"]
    assert abs(s2 - 2 * math.pi) < 1e-15
    g = O.green_function(512, 512)
    for r1, r2 in [(10, 20), (16, 64), (8, 40)]:
        d_num = g[r1, 0] - g[r2, 0]
        d_cont = math.log(r1 / r2) / s2
        assert abs(d_num - d_cont) < 5e-3


# ---------------------------------------------------------------- forward solve (A1-A7)

def test_three_independent_forward_solvers_agree():
    rng = np.random.default_rng(7)
    H, W, M, N = 5, 6, 12, 14
    gx, gy = _rand_field(rng, H, W)
    u_fft = O.solve_fft(gx, gy, M, N)
    u_dir = O.solve_direct(gx, gy, M, N)
    u_ls = O.lstsq_torus(gx, gy, M, N)
    assert np.max(np.abs(u_fft - u_dir)) < 1e-12
    assert np.max(np.abs(u_fft - u_ls)) < 1e-11


def test_direct_equals_fft_on_the_small_workload():
    w = synth.make_workload("small64")
    u_fft = O.solve_fft(w.gx, w.gy, w.M, w.N)
    u_dir = O.solve_direct(w.gx[0], w.gy[0], w.M, w.N)
    assert np.max(np.abs(u_fft[0] - u_dir)) < 1e-10 * np.max(np.abs(u_fft))


@pytest.mark.parametrize("H,W,M,N", [(6, 7, 14, 16), (20, 31, 40, 64), (64, 64, 128, 128)])
def test_framed_conservative_field_reconstructs_exactly(H, W, M, N):
    """A conservative field taken after zero padding reconstructs its image exactly, offset
    included because the reference pixel lies in the padding (Sec. 2.3.2, eq. (23))."""
    rng = np.random.default_rng(H * 1000 + W)
    S, gx, gy = _framed_conservative(rng, H, W)
    u = O.solve_fft(gx, gy, M, N)
    assert np.max(np.abs(u - S)) < 1e-12
    if M * N <= 14 * 16:
        assert np.max(np.abs(O.solve_direct(gx, gy, M, N) - S)) < 1e-12


def test_unframed_field_misses_boundary_flux():
    """Negative control: without the zero frame the left/top boundary fluxes are absent from
    H x W difference arrays and the reconstruction is off by O(1)."""
    rng = np.random.default_rng(3)
    S = synth.gaussian_sum_field(rng, 6, 7) + 0.5
    gx, gy = synth.forward_gradient(S)
    u = O.solve_fft(gx, gy, 14, 16)
    assert np.max(np.abs(u - S)) > 0.1


def test_eq15_sign_reconstructs_the_negative_image(golden_dir):
    """Reading of the stencil sign: with eq. (15)'s kernel the solve returns -I."""
    k = _load(golden_dir, "paper_kernels.json")
    lap15 = np.array(k["eq15_laplace"]["value"], dtype=float)
    H, W, M, N = 6, 7, 14, 16
    rng = np.random.default_rng(11)
    S, gx, gy = _framed_conservative(rng, H, W)
    G15 = O.green_spectrum_eq22(M, N, kernel=lap15)
    oy, ox = O.block_offset(H, W, M, N)
    L = O.divergence(gx, gy, M, N, oy, ox)
    v = np.real(np.fft.ifft2(np.fft.fft2(L) * G15))
    u15 = v[oy:oy + H, ox:ox + W] - v[0, 0]
    assert np.max(np.abs(u15 + S)) < 1e-12


def test_gfc_equals_dense_torus_least_squares():
    """Sec. 2.2: the GFC output is the least-squares potential of the padded torus field."""
    rng = np.random.default_rng(5)
    for H, W, M, N in [(4, 5, 8, 10), (6, 6, 12, 12)]:
        gx, gy = _rand_field(rng, H, W)
        assert np.max(np.abs(O.solve_fft(gx, gy, M, N) - O.lstsq_torus(gx, gy, M, N))) < 1e-11


def test_least_error_against_other_reconstructions():
    """Hilbert projection (eqs. (8)-(14)): no other potential has a smaller torus gradient
    error than GFC's. Checked against random perturbations and a Neumann least-squares solve
    restricted to the image (a Perez-style solution) embedded in the torus."""
    rng = np.random.default_rng(9)
    H, W, M, N = 6, 7, 14, 16
    gx, gy = _rand_field(rng, H, W)
    oy, ox = O.block_offset(H, W, M, N)
    D = O.torus_gradient(M, N)
    E = np.concatenate([O.embed(gx, M, N, oy, ox).ravel(), O.embed(gy, M, N, oy, ox).ravel()])
    u = O.solve_fft(gx, gy, M, N)
    # rebuild the full-torus GFC potential from the definition (eq. (23))
    v = np.real(np.fft.ifft2(np.fft.fft2(O.divergence(gx, gy, M, N, oy, ox)) * O.green_spectrum(M, N)))
    err = np.linalg.norm(D @ v.ravel() - E)
    for _ in range(20):
        d = rng.normal(size=(M, N))
        assert np.linalg.norm(D @ (v + 1e-3 * d).ravel() - E) > err
    # Neumann LS on the image only (interior edges), embedded with zero outside, best constant
    nx = np.zeros((H * (W - 1), H * W))
    ny = np.zeros(((H - 1) * W, H * W))
    idx = np.arange(H * W).reshape(H, W)
    r = 0
    for y in range(H):
        for x in range(W - 1):
            nx[r, idx[y, x]] = -1
            nx[r, idx[y, x + 1]] = 1
            r += 1
    r = 0
    for y in range(H - 1):
        for x in range(W):
            ny[r, idx[y, x]] = -1
            ny[r, idx[y + 1, x]] = 1
            r += 1
    A = np.vstack([nx, ny])
    rhs = np.concatenate([gx[:, :-1].ravel(), gy[:-1, :].ravel()])
    p, *_ = np.linalg.lstsq(A, rhs, rcond=None)
    best = np.inf
    for c in np.linspace(-5, 5, 201):
        vv = O.embed(p.reshape(H, W) + c, M, N, oy, ox)
        best = min(best, np.linalg.norm(D @ vv.ravel() - E))
    assert err < best
    # and GFC's own crop is the image part of that optimum up to the constant
    assert np.max(np.abs(u - (v[oy:oy + H, ox:ox + W] - v[0, 0]))) < 1e-13


def test_interior_laplacian_of_output_equals_input_laplacian():
    rng = np.random.default_rng(13)
    H, W, M, N = 40, 50, 96, 100
    gx, gy = _rand_field(rng, H, W)
    u = O.solve_fft(gx, gy, M, N)
    oy, ox = O.block_offset(H, W, M, N)
    L = O.divergence(gx, gy, M, N, oy, ox)[oy:oy + H, ox:ox + W]
    lap = u[2:, 1:-1] + u[:-2, 1:-1] + u[1:-1, 2:] + u[1:-1, :-2] - 4 * u[1:-1, 1:-1]
    assert np.max(np.abs(lap - L[1:-1, 1:-1])) < 1e-12


def test_linearity_and_translation_equivariance():
    rng = np.random.default_rng(17)
    H, W, M, N = 10, 12, 24, 30
    a = _rand_field(rng, H, W)
    b = _rand_field(rng, H, W)
    ua = O.solve_fft(*a, M, N)
    ub = O.solve_fft(*b, M, N)
    uab = O.solve_fft(2.0 * a[0] - 0.5 * b[0], 2.0 * a[1] - 0.5 * b[1], M, N)
    assert np.max(np.abs(uab - (2.0 * ua - 0.5 * ub))) < 1e-12
    # another block position changes u only by a constant (torus translation equivariance)
    oy, ox = O.block_offset(H, W, M, N)
    G = O.green_spectrum(M, N)
    for (py, px) in [(0, 0), (3, 17), (M - H, N - W)]:
        L = O.divergence(*a, M, N, py, px)
        v = np.real(np.fft.ifft2(np.fft.fft2(L) * G))
        d = v[py:py + H, px:px + W] - ua
        assert np.ptp(d) < 1e-12
        # with the reference pixel moved along with the block, u is identical
        ref = v[(py - oy) % M, (px - ox) % N]
        assert np.max(np.abs(v[py:py + H, px:px + W] - ref - ua)) < 1e-12


def test_dc_bin_value_is_irrelevant():
    rng = np.random.default_rng(19)
    H, W, M, N = 8, 9, 20, 22
    gx, gy = _rand_field(rng, H, W)
    oy, ox = O.block_offset(H, W, M, N)
    L = O.divergence(gx, gy, M, N, oy, ox)
    assert abs(L.sum()) < 1e-12
    G = O.green_spectrum(M, N)
    G2 = G.copy()
    G2[0, 0] = 123.0
    v1 = np.fft.ifft2(np.fft.fft2(L) * G)
    v2 = np.fft.ifft2(np.fft.fft2(L) * G2)
    u1 = np.real(v1)[oy:oy + H, ox:ox + W] - np.real(v1)[0, 0]
    u2 = np.real(v2)[oy:oy + H, ox:ox + W] - np.real(v2)[0, 0]
    assert np.max(np.abs(u1 - u2)) < 1e-12
    # eq. (23)'s real part: the imaginary residue is rounding only
    assert np.max(np.abs(v1.imag)) < 1e-13 * np.max(np.abs(v1.real))


# ---------------------------------------------------------------- backward (A8)

def test_adjoint_dot_product():
    rng = np.random.default_rng(23)
    for H, W, M, N in [(7, 9, 16, 20), (32, 32, 64, 64), (31, 17, 64, 36)]:
        gx, gy = _rand_field(rng, H, W)
        du = rng.normal(size=(H, W))
        u = O.solve_fft(gx, gy, M, N)
        dgx, dgy = O.solve_backward(du, M, N)
        lhs = np.sum(u * du)
        rhs = np.sum(gx * dgx) + np.sum(gy * dgy)
        assert abs(lhs - rhs) < 1e-12 * max(abs(lhs), 1.0)


def test_backward_matches_central_finite_differences():
    """Differentiable layer on the 2x1x32x32 / 64x64 instance: loss = mean((u - t)^2),
    gradient from the adjoint vs float64 central differences with h = 1e-6."""
    w = synth.make_workload("layer256", B=2, C=1, H=32, W=32, rect=8, grid=(64, 64))
    gx = w.gx.astype(np.float64)
    gy = w.gy.astype(np.float64)
    t = w.extra["target"].astype(np.float64)
    M, N = w.M, w.N
    n = gx.size

    def loss(ax, ay):
        return np.sum((O.solve_fft(ax, ay, M, N) - t) ** 2) / n

    u = O.solve_fft(gx, gy, M, N)
    dgx, dgy = O.solve_backward(2.0 * (u - t) / n, M, N)
    rng = np.random.default_rng(29)
    h = 1e-6
    for _ in range(40):
        b, y, x = rng.integers(0, 2), rng.integers(0, 32), rng.integers(0, 32)
        for arr, grad in ((gx, dgx), (gy, dgy)):
            p = arr.copy()
            m = arr.copy()
            p[b, y, x] += h
            m[b, y, x] -= h
            fd = (loss(p, gy) - loss(m, gy)) / (2 * h) if arr is gx else (loss(gx, p) - loss(gx, m)) / (2 * h)
            assert abs(fd - grad[b, y, x]) < 1e-8 + 1e-5 * abs(grad[b, y, x])


def test_backward_reference_term_is_required():
    """Dropping the -sum(du) delta term of the adjoint breaks the dot-product identity."""
    rng = np.random.default_rng(31)
    H, W, M, N = 7, 9, 16, 20
    gx, gy = _rand_field(rng, H, W)
    du = rng.normal(size=(H, W)) + 1.0
    u = O.solve_fft(gx, gy, M, N)
    oy, ox = O.block_offset(H, W, M, N)
    r = O.embed(du, M, N, oy, ox)  # no delta term
    w = np.real(np.fft.ifft2(np.fft.fft2(r) * O.green_spectrum(M, N)))
    bx = -(np.roll(w, -1, 1) - w)[oy:oy + H, ox:ox + W]
    by = -(np.roll(w, -1, 0) - w)[oy:oy + H, ox:ox + W]
    assert abs(np.sum(u * du) - (np.sum(gx * bx) + np.sum(gy * by))) > 1e-6


# ---------------------------------------------------------------- pin sensitivity

@pytest.mark.parametrize("mutation", ["forward_difference_div", "drop_y_term", "transpose_grid",
                                      "reference_pixel", "stencil_sign", "block_offset"])
def test_planted_oracle_mistakes_are_caught(monkeypatch, mutation):
    """Plant a plausible mistake in the oracle (on the CPU) and check a pin fails."""
    import oracle.gfc_oracle as G
    real_div = G.divergence
    real_green = G.green_spectrum

    if mutation == "forward_difference_div":
        def bad(gx, gy, M, N, oy, ox):
            Ex, Ey = G.embed(gx, M, N, oy, ox), G.embed(gy, M, N, oy, ox)
            return (np.roll(Ex, -1, -1) - Ex) + (np.roll(Ey, -1, -2) - Ey)
        monkeypatch.setattr(G, "divergence", bad)
    elif mutation == "drop_y_term":
        def bad(gx, gy, M, N, oy, ox):
            Ex = G.embed(gx, M, N, oy, ox)
            return Ex - np.roll(Ex, 1, -1)
        monkeypatch.setattr(G, "divergence", bad)
    elif mutation == "transpose_grid":
        def bad(M, N):  # the two axis lengths swapped inside the symbol
            k = np.arange(M)[:, None]
            l = np.arange(N)[None, :]
            lam = -4 * np.sin(np.pi * k / N) ** 2 - 4 * np.sin(np.pi * l / M) ** 2
            out = np.zeros((M, N))
            out[lam != 0] = 1.0 / lam[lam != 0]
            return out
        monkeypatch.setattr(G, "green_spectrum", bad)
    elif mutation == "stencil_sign":
        monkeypatch.setattr(G, "green_spectrum", lambda M, N: -real_green(M, N))
    elif mutation == "reference_pixel":
        def bad(gx, gy, M, N, oy, ox):
            return np.roll(real_div(gx, gy, M, N, oy, ox), 1, axis=-1)
        monkeypatch.setattr(G, "divergence", bad)
    elif mutation == "block_offset":
        real_off = G.block_offset
        monkeypatch.setattr(G, "block_offset",
                            lambda H, W, M, N: (real_off(H, W, M, N)[0] + 1, real_off(H, W, M, N)[1]))

    rng = np.random.default_rng(37)
    H, W, M, N = 6, 7, 14, 16
    S, gx, gy = _framed_conservative(rng, H, W)
    framed_ok = np.max(np.abs(G.solve_fft(gx, gy, M, N) - S)) < 1e-12
    a = _rand_field(rng, H, W)
    ls_ok = np.max(np.abs(G.solve_fft(*a, M, N) - G.lstsq_torus(*a, M, N))) < 1e-11
    lap = np.array([[0.0, 1.0, 0.0], [1.0, -4.0, 1.0], [0.0, 1.0, 0.0]])
    lit = _algorithm_b_literal(*a, 4, lap, (1, 1))[0]
    lit_ok = np.max(np.abs(G.solve_fft(*a, H + 8, W + 8) - lit)) < 1e-11
    assert not (framed_ok and ls_ok and lit_ok), f"mutation {mutation} went unnoticed"


# ---------------------------------------------------------------- colour correction (eq. (25))

def test_color_correction_restores_source_statistics():
    """Eq. (25) maps each solved image onto the mean and standard deviation of its source."""
    rng = np.random.default_rng(2501)
    u = rng.normal(size=(3, 17, 23)) * np.array([0.5, 2.0, 7.0])[:, None, None] + 3.0
    m = np.array([0.2, 0.5, -1.0])
    s = np.array([0.1, 0.3, 2.5])
    out = O.color_correct(u, m, s)
    for i in range(3):
        assert abs(out[i].mean() - m[i]) < 1e-13
        assert abs(out[i].std() - s[i]) < 1e-13 * max(1.0, s[i])


@pytest.mark.parametrize("k", [1.0, 0.25, 3.0])
def test_color_correction_undoes_a_uniform_gradient_scale(k):
    """Sec. 3.2.2: the sigma ratio only changes the norm of the gradient by a constant factor.
    A framed image S whose gradient is scaled by k > 0 solves to k S (eq. (23)); the
    correction with S's own statistics returns S exactly (k = 1 is the paper's unperturbed
    case, I_corr = I_c)."""
    rng = np.random.default_rng(int(k * 100))
    H, W, M, N = 20, 31, 40, 64
    S, gx, gy = _framed_conservative(rng, H, W)
    u = O.solve_fft(k * gx, k * gy, M, N)
    out = O.color_correct(u + 5.0, S.mean(), S.std())
    assert np.max(np.abs(out - S)) < 1e-12


def test_color_correction_is_invariant_to_positive_affine_maps():
    rng = np.random.default_rng(2503)
    u = rng.normal(size=(2, 9, 11))
    m, s = np.array([0.4, 0.6]), np.array([0.2, 0.05])
    ref = O.color_correct(u, m, s)
    assert np.max(np.abs(O.color_correct(4.0 * u - 7.0, m, s) - ref)) < 1e-13
    # a negative scale flips the image: the correction keeps the sign of the contrast
    flipped = O.color_correct(-u, m, s)
    assert np.max(np.abs((flipped - m[:, None, None]) + (ref - m[:, None, None]))) < 1e-13


def test_color_correction_of_a_constant_image_is_the_source_mean():
    out = O.color_correct(np.full((1, 4, 5), 3.0), [0.7], [0.2])
    assert np.all(out == 0.7)


# ---------------------------------------------------------------- gradient edits (Sec. 3.2.3, eq. (26))

def test_threshold_edit_keeps_strong_and_drops_weak_gradients():
    rng = np.random.default_rng(2701)
    gx = rng.normal(size=(40, 50)).astype(np.float32)
    gy = rng.normal(size=(40, 50)).astype(np.float32)
    mag = np.hypot(gx.astype(np.float64), gy.astype(np.float64))
    ex, ey = O.threshold_edit(gx, gy, 0.0)  # tau = 0 keeps every pixel
    assert np.array_equal(ex, gx) and np.array_equal(ey, gy)
    ex, ey = O.threshold_edit(gx, gy, 2 * mag.max())  # above every magnitude: all removed
    assert not ex.any() and not ey.any()
    tau = float(np.median(mag))
    ex, ey = O.threshold_edit(gx, gy, tau)
    kept = (ex != 0) | (ey != 0)
    assert 0.3 < kept.mean() < 0.7
    assert np.all(mag[kept] >= tau * (1 - 1e-6)) and np.all(mag[~kept] < tau * (1 + 1e-6))
    assert np.array_equal(ex[kept], gx[kept]) and np.array_equal(ey[kept], gy[kept])
    # a magnitude exactly at the level is kept: 3-4-5 with tau = 5
    ex, ey = O.threshold_edit(np.float32([[3.0]]), np.float32([[4.0]]), 5.0)
    assert ex[0, 0] == 3.0 and ey[0, 0] == 4.0


def test_gdm_edit_special_cases_and_geometric_mean():
    """Eq. (26): orientation of E, magnitude |E|^(1-alpha) C^alpha."""
    rng = np.random.default_rng(2702)
    gx = rng.normal(size=(30, 20))
    gy = rng.normal(size=(30, 20))
    C = rng.uniform(0.0, 2.0, size=(30, 20))
    mag = np.hypot(gx, gy)
    ex, ey = O.gdm_edit(gx, gy, C, 0.0)  # alpha = 0: the gradient alone
    assert np.allclose(ex, gx, rtol=1e-14, atol=0) and np.allclose(ey, gy, rtol=1e-14, atol=0)
    ex, ey = O.gdm_edit(gx, gy, C, 1.0)  # alpha = 1: the edge map's magnitude, E's direction
    assert np.allclose(np.hypot(ex, ey), C, rtol=1e-13, atol=1e-15)
    assert np.allclose(ex * gy - ey * gx, 0.0, atol=1e-13) and np.all(ex * gx + ey * gy >= 0)
    ex, ey = O.gdm_edit(gx, gy, mag, 0.37)  # C = |E|: unchanged for any alpha
    assert np.allclose(ex, gx, rtol=1e-13) and np.allclose(ey, gy, rtol=1e-13)
    # log |E_p| is affine in alpha (a weighted geometric mean)
    logs = [np.log(np.hypot(*O.gdm_edit(gx, gy, C + 0.1, a))) for a in (0.2, 0.5, 0.8)]
    assert np.allclose(logs[1] - logs[0], logs[2] - logs[1], atol=1e-12)
    # zero gradient: no orientation, E_p = 0
    ex, ey = O.gdm_edit(np.zeros((2, 2)), np.zeros((2, 2)), np.ones((2, 2)), 0.5)
    assert not ex.any() and not ey.any()


# ---------------------------------------------------------------- Laplacian input (Algorithm B)

def _support_divergence(gx, gy):
    """div E on the (H+1) x (W+1) support, from the definition (backward differences)."""
    H, W = gx.shape
    Ex = np.zeros((H + 1, W + 1)); Ex[:H, :W] = gx
    Ey = np.zeros((H + 1, W + 1)); Ey[:H, :W] = gy
    Exl = np.zeros_like(Ex); Exl[:, 1:] = Ex[:, :-1]
    Eyu = np.zeros_like(Ey); Eyu[1:, :] = Ey[:-1, :]
    return (Ex - Exl) + (Ey - Eyu)


def test_laplacian_input_equals_gradient_input():
    """Solving div E directly is the gradient solve (eq. (3) then eq. (23))."""
    rng = np.random.default_rng(3301)
    for H, W, M, N in ((6, 7, 14, 16), (20, 31, 40, 64)):
        gx, gy = _rand_field(rng, H, W)
        L = _support_divergence(gx, gy)
        assert abs(L.sum()) < 1e-12
        ref = O.solve_fft(gx, gy, M, N)
        assert np.max(np.abs(O.solve_laplacian(L, M, N) - ref)) < 1e-12 * max(1, np.abs(ref).max())


def test_laplacian_of_a_framed_image_reconstructs_it():
    """Algorithm B on the 5-point Laplacian (Algorithm A's stencil) of a zero-framed image
    returns the image, offset included (the corner lies in the padding)."""
    rng = np.random.default_rng(3302)
    H, W, M, N = 20, 31, 40, 64
    S, _, _ = _framed_conservative(rng, H, W)
    P = np.zeros((H + 3, W + 3)); P[1:H + 1, 1:W + 1] = S  # S with a zero ring
    Lfull = P[:-2, 1:-1] + P[2:, 1:-1] + P[1:-1, :-2] + P[1:-1, 2:] - 4 * P[1:-1, 1:-1]
    L = Lfull[:H + 1, :W + 1]  # row -1 and column -1 are zero for a framed image
    assert np.allclose(Lfull[H + 1:, :], 0) or Lfull.shape[0] == H + 1
    u = O.solve_laplacian(L, M, N)
    assert np.max(np.abs(u - S)) < 1e-12
    # and Algorithm A's spectrum built from the printed kernels gives the same solve
    Gh = O.green_spectrum_eq22(M, N)
    oy, ox = O.block_offset(H, W, M, N)
    v = np.real(np.fft.ifft2(np.fft.fft2(O.embed(L, M, N, oy, ox)) * Gh))
    assert np.max(np.abs((v[oy:oy + H, ox:ox + W] - v[0, 0]) - S)) < 1e-11


# ---------------------------------------------------------------- three dimensions

def _framed_volume(rng, D, H, W):
    """A volume with zero first plane, row and column (padding before the gradient) and its
    forward-difference gradient (gx, gy, gz) with a zero exterior."""
    S = rng.normal(size=(D, H, W))
    S[0, :, :] = 0.0
    S[:, 0, :] = 0.0
    S[:, :, 0] = 0.0
    g = []
    for ax in (2, 1, 0):
        Sp = np.concatenate([S, np.zeros_like(np.take(S, [0], axis=ax))], axis=ax)
        g.append(np.diff(Sp, axis=ax))
    return S, g[0], g[1], g[2]


def test_3d_framed_conservative_volume_reconstructs_exactly():
    rng = np.random.default_rng(3501)
    for D, H, W, P, M, N in ((5, 6, 7, 12, 14, 16), (9, 12, 10, 20, 24, 20)):
        S, gx, gy, gz = _framed_volume(rng, D, H, W)
        assert np.max(np.abs(O.solve3_fft(gx, gy, gz, P, M, N) - S)) < 1e-12


def test_3d_gfc_equals_dense_torus_least_squares():
    """Sec. 2.2 in three dimensions: the Fourier solve is the least-squares potential."""
    rng = np.random.default_rng(3502)
    D, H, W, P, M, N = 3, 4, 3, 6, 6, 6
    gx, gy, gz = (rng.normal(size=(D, H, W)) for _ in range(3))
    a = O.solve3_fft(gx, gy, gz, P, M, N)
    b = O.lstsq_torus3(gx, gy, gz, P, M, N)
    assert np.max(np.abs(a - b)) < 1e-10


def test_3d_green_spectrum_inverts_the_7_point_stencil():
    """1 / lambda is the spectrum of the pseudo-inverse of the 7-point Laplacian: K * g =
    delta - 1 / (P M N) (eq. (16) in three dimensions, DC projected out)."""
    P, M, N = 6, 8, 10
    g = np.real(np.fft.ifftn(O.green_spectrum3(P, M, N)))
    Kg = -6 * g
    for ax in range(3):
        Kg += np.roll(g, 1, axis=ax) + np.roll(g, -1, axis=ax)
    d = -np.full((P, M, N), 1.0 / (P * M * N))
    d[0, 0, 0] += 1.0
    assert np.max(np.abs(Kg - d)) < 1e-13


def test_3d_interior_laplacian_equals_divergence():
    rng = np.random.default_rng(3503)
    D, H, W, P, M, N = 8, 9, 10, 18, 18, 20
    gx, gy, gz = (rng.normal(size=(D, H, W)) for _ in range(3))
    u = O.solve3_fft(gx, gy, gz, P, M, N)
    lap = -6 * u[1:-1, 1:-1, 1:-1]
    for ax in range(3):
        lap += np.roll(u, 1, axis=ax)[1:-1, 1:-1, 1:-1] + np.roll(u, -1, axis=ax)[1:-1, 1:-1, 1:-1]
    L = (gx[1:-1, 1:-1, 1:-1] - gx[1:-1, 1:-1, :-2] + gy[1:-1, 1:-1, 1:-1] - gy[1:-1, :-2, 1:-1]
         + gz[1:-1, 1:-1, 1:-1] - gz[:-2, 1:-1, 1:-1])
    assert np.max(np.abs(lap - L)) < 1e-11
