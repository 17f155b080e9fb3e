"""Pass-level GPU checks: the forward row pass, the column pass and the inverse row pass, and
the first and last backward passes, each alone, through gfc_solve_batch_stage and
gfc_solve_backward_stage, against float64 numpy transforms of the same inputs. The intermediate
layout is the library's workspace (spectra T, B images of (H+1) x NHP complex64 from offset 0,
each stored tile-major: bin l of row y at ((l // 16) * (H+1) + y) * 16 + l % 16, so that a
column tile's 16 bins run contiguously down the rows; the split side array SB [B][H][KP]
row-major at the next 256-byte boundary; column partials after it), so these tests know that
layout on purpose."""
import ctypes
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


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module", autouse=True)
def _need_gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    if not os.path.exists(gfc.lib_path()):
        pytest.fail("libgfc.so is not built: the HIP path must exist where a GPU is present")


def _align256(n):
    return (n + 255) // 256 * 256


def _fields(seed, B, H, W):
    rng = np.random.default_rng(seed)
    gx = np.empty((B, H, W), np.float32)
    gy = np.empty((B, H, W), np.float32)
    for i in range(B):
        a, b = synth.forward_gradient(synth.gaussian_sum_field(rng, H, W))
        gx[i] = a + 0.01 * rng.normal(size=(H, W))
        gy[i] = b
    return gx, gy


def _stage(plan, k, gx, gy, u, B, ws):
    st = torch.cuda.current_stream()
    r = gfc.lib().gfc_solve_batch_stage(plan.handle, k, gx.data_ptr(), gy.data_ptr(),
                                        u.data_ptr(), B, ws.data_ptr(), ws.numel(),
                                        ctypes.c_void_p(st.cuda_stream))
    assert r == 0, gfc.lib().gfc_status_str(r)


def _from_tiles(flat, B, R, NHP):
    """Spectra in the workspace's tile-major order -> [B][R][NHP]."""
    return flat.reshape(B, NHP // 16, R, 16).transpose(0, 2, 1, 3).reshape(B, R, NHP)


def _to_tiles(a):
    """[B][R][NHP] -> the workspace's tile-major order, flat."""
    B, R, NHP = a.shape
    return np.ascontiguousarray(a.reshape(B, R, NHP // 16, 16).transpose(0, 2, 1, 3)).reshape(-1)


def _rel(a, b):
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


@pytest.mark.parametrize("H,W,M,N,K", [(33, 70, 35, 72, 4), (129, 200, 260, 400, 4),
                                       (801, 1200, 1620, 2400, 4), (40, 300, 84, 640, 16),
                                       (3, 1250, 8, 2400, 32)])
def test_forward_row_pass_alone(H, W, M, N, K):
    """Row pass (divergence fused into the row R2C, eq. (3) and the row half of F(L) in
    eq. (23)): T1[y, l] = L^[y, l] for l > K, and the split form (1 - w^l) Ex^[y, l] with
    SB[y, l] = Ey^[y, l] for l <= K (T1[y, 0] = 0), the block at the torus origin."""
    B = 2
    _say(f"row pass alone H={H} W={W} M={M} N={N} K={K}")
    plan = gfc.Plan(H, W, M, N, params={"low_bins": K}, tuned=False).build()
    NH = N // 2 + 1
    NHP = (NH + 31) // 32 * 32
    KP = (K + 1 + 7) // 8 * 8
    gx, gy = _fields(H + W, B, H, W)
    tx, ty = torch.from_numpy(gx).cuda(), torch.from_numpy(gy).cuda()
    u = torch.empty_like(tx)
    ws = torch.zeros(plan.workspace_size(B), dtype=torch.uint8, device="cuda")
    _stage(plan, 1, tx, ty, u, B, ws)
    torch.cuda.synchronize()
    raw = ws.cpu().numpy()
    t_bytes = B * (H + 1) * NHP * 8
    T = _from_tiles(raw[:t_bytes].view(np.complex64), B, H + 1, NHP)[:, :, :NH].astype(np.complex128)
    s0 = _align256(t_bytes)
    SB = raw[s0:s0 + B * H * KP * 8].view(np.complex64).reshape(B, H, KP)[:, :, :K + 1]
    l = np.arange(NH)
    one_minus_w = 1.0 - np.exp(-2j * np.pi * l / N)
    for b in range(B):
        L = O.divergence(gx[b], gy[b], M, N, 0, 0)[:H + 1]
        Lh = np.fft.fft(L, axis=1)[:, :NH]
        Ex = np.zeros((H + 1, N))
        Ex[:H, :W] = gx[b]
        Ey = np.zeros((H, N))
        Ey[:, :W] = gy[b]
        want = Lh.copy()
        want[:, :K + 1] = (np.fft.fft(Ex, axis=1)[:, :NH] * one_minus_w)[:, :K + 1]
        e1 = _rel(T[b], want)
        e2 = _rel(SB[b].astype(np.complex128), np.fft.fft(Ey, axis=1)[:, :K + 1])
        _say(f"  image {b}: T1 rel {e1:.2e}, SB rel {e2:.2e}")
        assert e1 <= TOL and e2 <= TOL, (b, e1, e2)


@pytest.mark.parametrize("H,W,M,N", [(33, 70, 35, 72), (129, 200, 260, 400),
                                     (801, 1200, 1620, 2400)])
def test_inverse_row_pass_alone(H, W, M, N):
    """Inverse row pass (row C2R of eq. (23), real part, crop, Algorithm B's constant) on a
    given spectrum: u[y, x] = sum_l T2[y, l] w^(-l x) over the Hermitian extension (no
    1/N: the column pass folds it in), x < W, minus the sum of the column partials."""
    B = 2
    _say(f"inverse row pass alone H={H} W={W} M={M} N={N}")
    plan = gfc.Plan(H, W, M, N, tuned=False).build()
    NH = N // 2 + 1
    NHP = (NH + 31) // 32 * 32
    K = plan.get_param("low_bins")
    KP = (K + 1 + 7) // 8 * 8
    Kb = plan.get_param("low_bins_b")
    KbP = (Kb + 1 + 31) // 32 * 32
    C = plan.get_param("col_c")
    ntiles = (NH + C - 1) // C
    rng = np.random.default_rng(H * W)
    T2 = (rng.normal(size=(B, H + 1, NHP)) + 1j * rng.normal(size=(B, H + 1, NHP))) / N
    T2[:, :, 0] = T2[:, :, 0].real  # a real row has real DC and Nyquist bins
    if N % 2 == 0:
        T2[:, :, N // 2] = T2[:, :, N // 2].real
    T2 = T2.astype(np.complex64)
    part = rng.normal(size=(B, ntiles))
    ws = torch.zeros(plan.workspace_size(B), dtype=torch.uint8, device="cuda")
    raw = np.zeros(ws.numel(), np.uint8)
    t_bytes = B * (H + 1) * NHP * 8
    raw[:t_bytes] = _to_tiles(T2).view(np.uint8)
    side = _align256(t_bytes)
    red = side + _align256(max(B * H * KP * 8, B * H * KbP * 8))
    raw[red:red + part.nbytes] = part.reshape(-1).view(np.uint8)
    ws.copy_(torch.from_numpy(raw))
    u = torch.empty((B, H, W), dtype=torch.float32, device="cuda")
    dummy = torch.empty(1, device="cuda")
    _stage(plan, 3, dummy, dummy, u, B, ws)
    torch.cuda.synchronize()
    got = u.cpu().numpy()
    for b in range(B):
        v = np.fft.irfft(T2[b, :H, :NH].astype(np.complex128), n=N, axis=1) * N
        want = v[:, :W] - part[b].sum()
        e = _rel(got[b], want)
        _say(f"  image {b}: rel {e:.2e}")
        assert e <= TOL, (b, e)


@pytest.mark.parametrize("H,W,M,N", [(33, 70, 35, 72), (129, 200, 260, 400),
                                     (100, 37, 210, 80), (801, 1200, 1620, 2400)])
def test_column_pass_alone(H, W, M, N):
    """Column pass (the column slices of G^ of eq. (22) applied per row frequency l, the
    reference term of Algorithm B) on given row spectra T1 [H+1] and side array SB [H]:
    for every l the column input is T1[., l] plus the y-difference of SB[., l] (l <= K),
    zero-extended to M rows; T2[y, l] = IDFT_M(G^(., l) DFT_M(column))[y] / N for y < H
    (column 0 up to a constant that cancels), and the column partials sum to v at the grid
    corner (r0, c0) of the block at the origin."""
    B = 2
    _say(f"column pass alone H={H} W={W} M={M} N={N}")
    plan = gfc.Plan(H, W, M, N, tuned=False).build()
    NH = N // 2 + 1
    NHP = (NH + 31) // 32 * 32
    K = plan.get_param("low_bins")
    KP = (K + 1 + 7) // 8 * 8
    Kb = plan.get_param("low_bins_b")
    KbP = (Kb + 1 + 31) // 32 * 32
    C = plan.get_param("col_c")
    ntiles = (NH + C - 1) // C
    oy, ox = O.block_offset(H, W, M, N)
    r0, c0 = M - oy, N - ox
    rng = np.random.default_rng(7 * H + W)
    T1 = rng.normal(size=(B, H + 1, NHP)) + 1j * rng.normal(size=(B, H + 1, NHP))
    T1[:, :, 0] = 0.0  # the row pass's split form leaves (1 - w^0) Ex^ = 0
    T1[:, :, N // 2] = T1[:, :, N // 2].real  # real rows: real Nyquist bin
    SB = rng.normal(size=(B, H, KP)) + 1j * rng.normal(size=(B, H, KP))
    SB[:, :, 0] = SB[:, :, 0].real
    T1 = T1.astype(np.complex64)
    SB = SB.astype(np.complex64)
    raw = np.zeros(plan.workspace_size(B), np.uint8)
    t_bytes = B * (H + 1) * NHP * 8
    raw[:t_bytes] = _to_tiles(T1).view(np.uint8)
    side = _align256(t_bytes)
    raw[side:side + SB.nbytes] = SB.reshape(-1).view(np.uint8)
    red = side + _align256(max(B * H * KP * 8, B * H * KbP * 8))
    ws = torch.from_numpy(raw).cuda()
    dummy = torch.empty(1, device="cuda")
    _stage(plan, 2, dummy, dummy, dummy, B, ws)
    torch.cuda.synchronize()
    out = ws.cpu().numpy()
    T2 = _from_tiles(out[:t_bytes].view(np.complex64), B, H + 1, NHP)
    part = out[red:red + B * ntiles * 8].view(np.float64).reshape(B, ntiles)
    G = O.green_spectrum(M, N)[:, :NH]
    for b in range(B):
        col = np.zeros((M, NH), np.complex128)
        col[:H + 1] = T1[b, :, :NH]
        d = np.zeros((M, K + 1), np.complex128)
        d[:H] += SB[b, :, :K + 1]
        d[1:H + 1] -= SB[b, :, :K + 1]
        col[:, :K + 1] += d
        v = np.fft.ifft(G * np.fft.fft(col, axis=0), axis=0) / N
        got = T2[b, :H, :NH].astype(np.complex128)
        # column 0 (the pseudo-inverse, G^(0, 0) = 0) is fixed only up to a constant c: it
        # adds c to every pixel and to the corner alike, and the corner subtraction of
        # Algorithm B removes it; the pass may pick any c, the same in both places
        c = np.mean(got[:, 0] - v[:H, 0])
        v[:, 0] += c
        e = _rel(got, v[:H])
        row = np.fft.irfft(v[r0 % M], n=N) * N  # v on the corner's row, with c
        corner = row[c0 % N]
        ec = abs(part[b].sum() - corner) / np.abs(row).max()
        _say(f"  image {b}: T2 rel {e:.2e}, corner {part[b].sum():.6e} vs {corner:.6e} "
             f"(column-0 constant {c.real:.3e})")
        assert e <= TOL, (b, e)
        assert ec <= TOL, (b, ec)


def _bstage(plan, k, du, dgx, dgy, B, ws):
    st = torch.cuda.current_stream()
    r = gfc.lib().gfc_solve_backward_stage(plan.handle, k, du.data_ptr(), dgx.data_ptr(),
                                           dgy.data_ptr(), B, ws.data_ptr(), ws.numel(),
                                           ctypes.c_void_p(st.cuda_stream))
    assert r == 0, gfc.lib().gfc_status_str(r)


@pytest.mark.parametrize("H,W,M,N", [(33, 70, 35, 72), (129, 200, 260, 400),
                                     (801, 1200, 1620, 2400)])
def test_backward_row_pass_alone(H, W, M, N):
    """First backward pass (the adjoint of the inverse row pass): U[y, l] = the row DFT of
    du (forward sign) for y < H, and partial sums whose total is sum(du), the weight of the
    adjoint of Algorithm B's corner subtraction."""
    B = 2
    _say(f"backward row pass alone H={H} W={W} M={M} N={N}")
    plan = gfc.Plan(H, W, M, N, tuned=False).build()
    NH = N // 2 + 1
    NHP = (NH + 31) // 32 * 32
    K = plan.get_param("low_bins")
    KP = (K + 1 + 7) // 8 * 8
    Kb = plan.get_param("low_bins_b")
    KbP = (Kb + 1 + 31) // 32 * 32
    du = np.random.default_rng(H + W).normal(size=(B, H, W)).astype(np.float32)
    tdu = torch.from_numpy(du).cuda()
    ws = torch.zeros(plan.workspace_size(B), dtype=torch.uint8, device="cuda")
    dummy = torch.empty(1, device="cuda")
    _bstage(plan, 1, tdu, dummy, dummy, B, ws)
    torch.cuda.synchronize()
    raw = ws.cpu().numpy()
    t_bytes = B * (H + 1) * NHP * 8
    U = _from_tiles(raw[:t_bytes].view(np.complex64), B, H + 1, NHP)
    red = _align256(t_bytes) + _align256(max(B * H * KP * 8, B * H * KbP * 8))
    sums = raw[red:red + (len(raw) - red) // 8 * 8].view(np.float64)
    for b in range(B):
        want = np.fft.fft(np.pad(du[b].astype(np.float64), ((0, 0), (0, N - W))), axis=1)[:, :NH]
        e = _rel(U[b, :H, :NH].astype(np.complex128), want)
        _say(f"  image {b}: U rel {e:.2e}")
        assert e <= TOL, (b, e)
    # the reduction region starts with the partial sums, [B][nsums]; nsums (row blocks per
    # image) depends on the FFT slot width, so it is found as the split that gives every
    # image its own total (the rest of the zero-filled region adds nothing)
    tot = du.astype(np.float64).sum(axis=(1, 2))
    assert np.isclose(sums.sum(), tot.sum(), rtol=1e-6, atol=1e-6 * np.abs(du).sum())
    found = False
    for nsums in range(1, len(sums) // B + 1):
        s = sums[:B * nsums].reshape(B, nsums).sum(axis=1)
        if np.allclose(s, tot, rtol=1e-6, atol=1e-6 * np.abs(du).sum()):
            found = True
            break
    assert found, "no prefix of the reduction region sums to sum(du) per image"


@pytest.mark.parametrize("H,W,M,N", [(33, 70, 35, 72), (129, 200, 260, 400),
                                     (801, 1200, 1620, 2400)])
def test_backward_inverse_row_pass_alone(H, W, M, N):
    """Last backward pass on given W [H+1] and SD [H] (l <= Kb): dgx[y] = C2R of
    (1 - w^(-l)) W[y, l] (-D_x as its symbol, forward differences), dgy[y] = C2R of SD[y, l]
    for l <= Kb and of W[y, l] - W[y+1, l] above (-D_y), both unnormalised, x < W."""
    B = 2
    _say(f"backward inverse row pass alone H={H} W={W} M={M} N={N}")
    plan = gfc.Plan(H, W, M, N, tuned=False).build()
    NH = N // 2 + 1
    NHP = (NH + 31) // 32 * 32
    K = plan.get_param("low_bins")
    KP = (K + 1 + 7) // 8 * 8
    Kb = plan.get_param("low_bins_b")
    KbP = (Kb + 1 + 31) // 32 * 32
    rng = np.random.default_rng(3 * H + W)
    Wv = (rng.normal(size=(B, H + 1, NHP)) + 1j * rng.normal(size=(B, H + 1, NHP))) / N
    Wv[:, :, 0] = Wv[:, :, 0].real
    Wv[:, :, N // 2] = Wv[:, :, N // 2].real
    SD = (rng.normal(size=(B, H, KbP)) + 1j * rng.normal(size=(B, H, KbP))) / N
    SD[:, :, 0] = SD[:, :, 0].real
    if Kb == N // 2:
        SD[:, :, Kb] = SD[:, :, Kb].real
    Wv = Wv.astype(np.complex64)
    SD = SD.astype(np.complex64)
    raw = np.zeros(plan.workspace_size(B), np.uint8)
    t_bytes = B * (H + 1) * NHP * 8
    raw[:t_bytes] = _to_tiles(Wv).view(np.uint8)
    side = _align256(t_bytes)
    raw[side:side + SD.nbytes] = SD.reshape(-1).view(np.uint8)
    ws = torch.from_numpy(raw).cuda()
    dgx = torch.empty((B, H, W), dtype=torch.float32, device="cuda")
    dgy = torch.empty_like(dgx)
    dummy = torch.empty(1, device="cuda")
    _bstage(plan, 3, dummy, dgx, dgy, B, ws)
    torch.cuda.synchronize()
    l = np.arange(NH)
    sym = 1.0 - np.exp(2j * np.pi * l / N)
    for b in range(B):
        Wb = Wv[b, :, :NH].astype(np.complex128)
        X1 = sym * Wb[:H]
        X2 = Wb[:H] - Wb[1:H + 1]
        X2[:, :Kb + 1] = SD[b, :, :Kb + 1]
        wx = np.fft.irfft(X1, n=N, axis=1)[:, :W] * N
        wy = np.fft.irfft(X2, n=N, axis=1)[:, :W] * N
        ex = _rel(dgx[b].cpu().numpy(), wx)
        ey = _rel(dgy[b].cpu().numpy(), wy)
        _say(f"  image {b}: dgx rel {ex:.2e}, dgy rel {ey:.2e}")
        assert ex <= TOL and ey <= TOL, (b, ex, ey)
