"""GPU parity: the HIP path (through the C ABI) against the float64 oracle, element by
element on the same float32 inputs. Bar: per-image relative L2 <= 1e-5 (max over the
batch), forward and backward."""
import math
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


def rel_l2(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-300))


def per_image_rel(a, b):
    return [rel_l2(x, y) for x, y in zip(a, b)]


def _gpu_solve(gx, gy, M, N):
    tx = torch.from_numpy(np.ascontiguousarray(gx)).cuda()
    ty = torch.from_numpy(np.ascontiguousarray(gy)).cuda()
    u = gfc.solve(tx, ty, M, N)
    torch.cuda.synchronize()
    return u.cpu().numpy()


def _gpu_backward(du, M, N):
    td = torch.from_numpy(np.ascontiguousarray(du)).cuda()
    dgx, dgy = gfc.solve_backward(td, M, N)
    torch.cuda.synchronize()
    return dgx.cpu().numpy(), dgy.cpu().numpy()


def _rand_fields(seed, B, H, W):
    rng = np.random.default_rng(seed)
    gx = np.empty((B, H, W), np.float32)
    gy = np.empty((B, H, W), np.float32)
    for i in range(B):
        S = synth.gaussian_sum_field(rng, H, W)
        a, b = synth.forward_gradient(S)
        gx[i] = a + 0.01 * rng.normal(size=(H, W))
        gy[i] = b
    return gx, gy


# small and odd shapes: several row strips, column tiles and segments, ragged tails
SHAPES = [
    (64, 64, 128, 128),    # the 64x64 workload's torus
    (1, 1, 16, 16),        # one pixel
    (1, 37, 3, 80),        # one row, minimal vertical padding
    (37, 1, 80, 16),       # one column
    (31, 45, 64, 96),
    (100, 37, 210, 80),    # odd M, R = H + 1 not a multiple of anything
    (33, 70, 35, 72),      # minimal padding in both directions (M = H + 2, N = W + 2)
    (129, 200, 260, 400),
    (255, 300, 513, 640),
    (3, 1250, 8, 2400),    # 2W > N on the longest rows: every element column is loaded
    (2, 2398, 6, 2400),    # the widest image a plan accepts (W = N - 2) on the longest rows
    (3, 2046, 6, 2048),    # the same on the longest power-of-two row
    (2, 1200, 6, 2400),    # the widest default row (one FFT slot per wavefront), K = 32
    (8, 1200, 16, 2400),   # thin and wide: 16 row bins split
    (16, 1200, 32, 2400),  # 8 row bins split
    (5000, 6, 10000, 16),  # a tall column: over 300 row segments in one workgroup
]


@pytest.mark.parametrize("H,W,M,N", SHAPES)
def test_forward_parity_small_shapes(H, W, M, N):
    _say(f"forward parity H={H} W={W} M={M} N={N}")
    gx, gy = _rand_fields(H * 7 + W, 3, H, W)
    u = _gpu_solve(gx, gy, M, N)
    ref = O.solve_fft(gx, gy, M, N)
    errs = per_image_rel(u, ref)
    assert max(errs) <= TOL, errs


@pytest.mark.parametrize("K", [5, 16, 32])
def test_forward_more_split_bins(K):
    """Raising K moves the row bins (4, K] from the FFT to the split form of the extension
    pass: the exact result is the same, so the oracle bar holds for every K."""
    H, W, M, N = 40, 300, 84, 640
    _say(f"forward parity with low_bins={K} H={H} W={W} M={M} N={N}")
    gx, gy = _rand_fields(777 + K, 3, H, W)
    p = gfc.Plan(H, W, M, N, params={"low_bins": K}, tuned=False)
    assert p.get_param("low_bins") == K
    tx = torch.from_numpy(gx).cuda()
    ty = torch.from_numpy(gy).cuda()
    u = p.solve(tx, ty).cpu().numpy()
    errs = per_image_rel(u, O.solve_fft(gx, gy, M, N))
    assert max(errs) <= TOL, errs
    # and agrees with the default split to float32 rounding
    u4 = gfc.Plan(H, W, M, N, params={"low_bins": 4}, tuned=False).solve(tx, ty).cpu().numpy()
    assert max(per_image_rel(u, u4)) <= TOL


@pytest.mark.parametrize("H,W", [(1, 1), (4, 4), (32767, 4)])
def test_default_tori_at_the_size_limits(H, W):
    """Default tori of the smallest images and of the tallest one a plan accepts (1024
    column segments of 32 rows in one workgroup), forward and backward."""
    p = gfc.Plan(H, W, tuned=False)
    M, N = p.M, p.N
    _say(f"default torus H={H} W={W} -> M={M} N={N}")
    gx, gy = _rand_fields(H + 5 * W, 2, H, W)
    u = _gpu_solve(gx, gy, M, N)
    errs = per_image_rel(u, O.solve_fft(gx, gy, M, N))
    assert max(errs) <= TOL, errs
    du = (0.1 * np.random.default_rng(H).normal(size=(2, H, W)) + 0.02).astype(np.float32)
    dgx, dgy = _gpu_backward(du, M, N)
    rx, ry = O.solve_backward(du, M, N)
    for i in range(2):
        e = rel_l2(np.concatenate([dgx[i], dgy[i]]), np.concatenate([rx[i], ry[i]]))
        assert e <= TOL, (i, e)


def test_forward_small64_workload():
    w = synth.make_workload("small64")
    _say("forward parity small64")
    u = _gpu_solve(w.gx, w.gy, w.M, w.N)
    ref = O.solve_direct(w.gx[0], w.gy[0], w.M, w.N)
    assert rel_l2(u[0], ref) <= TOL


def test_forward_framed_conservative_reconstructs_image():
    rng = np.random.default_rng(4)
    H, W = 200, 300
    S = synth.gaussian_sum_field(rng, H, W)
    S[0, :] = 0
    S[:, 0] = 0
    gx, gy = synth.forward_gradient(S)
    u = _gpu_solve(gx[None].astype(np.float32), gy[None].astype(np.float32), 400, 600)[0]
    assert rel_l2(u, S) <= TOL


def test_forward_batch801x1200_sampled():
    """The 801x1200 x 100 workload on its 1620x2400 torus, in the launch configuration the
    benchmark times (all 100 images in one call); the oracle checks sampled images."""
    _say("forward parity 801x1200 B=100 (sampled)")
    w = synth.make_workload("batch801x1200")
    u = _gpu_solve(w.gx, w.gy, w.M, w.N)
    assert np.all(np.isfinite(u))
    for i in (0, 41, 99):
        ref = O.solve_fft(w.gx[i], w.gy[i], w.M, w.N)
        e = rel_l2(u[i], ref)
        _say(f"  image {i}: rel L2 {e:.3e}")
        assert e <= TOL


def test_backward_batch801x1200_sampled():
    """The backward solve of 100 images of 801x1200 in one call, as the benchmark's fwd+bwd
    step launches it (the column pass then runs its low tiles on the side stream); the
    oracle checks sampled images."""
    _say("backward parity 801x1200 B=100 (sampled)")
    H, W, M, N, B = 801, 1200, 1620, 2400, 100
    du = (np.random.default_rng(8011200).normal(size=(B, H, W)) * 0.1 + 0.01).astype(np.float32)
    dgx, dgy = _gpu_backward(du, M, N)
    assert np.all(np.isfinite(dgx)) and np.all(np.isfinite(dgy))
    for i in (0, 57, 99):
        rx, ry = O.solve_backward(du[i:i + 1], M, N)
        e = rel_l2(np.concatenate([dgx[i], dgy[i]]), np.concatenate([rx[0], ry[0]]))
        _say(f"  image {i}: rel L2 {e:.3e}")
        assert e <= TOL


def test_forward_merge512_sampled():
    _say("forward parity merge512 (sampled)")
    w = synth.make_workload("merge512")
    u = _gpu_solve(w.gx, w.gy, w.M, w.N)
    for i in (0, 50, 95):
        e = rel_l2(u[i], O.solve_fft(w.gx[i], w.gy[i], w.M, w.N))
        assert e <= TOL, (i, e)


def test_interior_laplacian_property_full_size():
    """At full size, a property that holds at any size: the output's 5-point Laplacian equals
    the input divergence in the interior (to float32 rounding)."""
    w = synth.make_workload("batch801x1200", B=4)
    u = _gpu_solve(w.gx, w.gy, w.M, w.N).astype(np.float64)
    for i in range(4):
        gx = w.gx[i].astype(np.float64)
        gy = w.gy[i].astype(np.float64)
        L = np.zeros_like(gx)
        L[:, 1:] += gx[:, 1:] - gx[:, :-1]
        L[1:, :] += gy[1:, :] - gy[:-1, :]
        ui = u[i]
        lap = ui[2:, 1:-1] + ui[:-2, 1:-1] + ui[1:-1, 2:] + ui[1:-1, :-2] - 4 * ui[1:-1, 1:-1]
        assert np.max(np.abs(lap - L[1:-1, 1:-1])) <= 2e-4 * np.max(np.abs(L))


def test_forward_is_deterministic():
    gx, gy = _rand_fields(5, 4, 129, 200)
    a = _gpu_solve(gx, gy, 260, 400)
    b = _gpu_solve(gx, gy, 260, 400)
    assert np.array_equal(a, b)


def test_forward_batch_independence():
    """Each image's result does not depend on the other images of the batch."""
    gx, gy = _rand_fields(6, 5, 64, 80)
    full = _gpu_solve(gx, gy, 130, 160)
    one = _gpu_solve(gx[2:3], gy[2:3], 130, 160)
    assert np.array_equal(full[2], one[0])


def test_zero_batch_is_noop():
    t = torch.zeros((0, 16, 16), device="cuda")
    u = gfc.solve(t, t, 40, 40)
    assert u.shape == (0, 16, 16)


def test_nonfinite_input_propagates():
    gx, gy = _rand_fields(7, 1, 32, 32)
    gx[0, 5, 5] = np.nan
    u = _gpu_solve(gx, gy, 64, 64)
    assert np.isnan(u).any()


# ---------------------------------------------------------------- backward

@pytest.mark.parametrize("H,W,M,N", [(64, 64, 128, 128), (31, 45, 64, 96), (100, 37, 210, 80),
                                     (1, 37, 3, 80), (33, 70, 35, 72), (129, 200, 260, 400),
                                     (2, 1200, 6, 2400), (2, 2398, 6, 2400),
                                     (5000, 6, 10000, 16)])
def test_backward_parity(H, W, M, N):
    _say(f"backward parity H={H} W={W} M={M} N={N}")
    rng = np.random.default_rng(H + 3 * W)
    du = (0.1 * rng.normal(size=(3, H, W)) + 0.02).astype(np.float32)
    dgx, dgy = _gpu_backward(du, M, N)
    rx, ry = O.solve_backward(du, M, N)
    for i in range(3):
        e = rel_l2(np.concatenate([dgx[i], dgy[i]]), np.concatenate([rx[i], ry[i]]))
        assert e <= TOL, (i, e)


def test_backward_layer256_workload():
    _say("backward parity layer256")
    w = synth.make_workload("layer256")
    t = torch.from_numpy(w.extra["target"]).cuda()
    gx = torch.from_numpy(w.gx).cuda().requires_grad_(True)
    gy = torch.from_numpy(w.gy).cuda().requires_grad_(True)
    u = gfc.GFCFunction.apply(gx, gy, w.M, w.N)
    loss = ((u - t) ** 2).mean()
    loss.backward()
    torch.cuda.synchronize()
    u64 = O.solve_fft(w.gx, w.gy, w.M, w.N)
    n = u64.size
    du = 2.0 * (u64 - w.extra["target"].astype(np.float64)) / n
    rx, ry = O.solve_backward(du, w.M, w.N)
    gxn, gyn = gx.grad.cpu().numpy(), gy.grad.cpu().numpy()
    errs = [rel_l2(np.concatenate([gxn[i], gyn[i]]), np.concatenate([rx[i], ry[i]]))
            for i in range(0, w.B, 7)]
    assert max(errs) <= TOL, errs


def test_backward_matches_finite_differences_on_gpu_layer():
    """GPU backward vs float64 central differences (h = 1e-6) of the float64 oracle's loss on
    the 2x1x32x32 instance (64x64 torus)."""
    w = synth.make_workload("layer256", B=2, C=1, H=32, W=32, rect=8, grid=(64, 64))
    t = w.extra["target"].astype(np.float64)
    gx = torch.from_numpy(w.gx).cuda().requires_grad_(True)
    gy = torch.from_numpy(w.gy).cuda().requires_grad_(True)
    u = gfc.GFCFunction.apply(gx, gy, 64, 64)
    loss = ((u - torch.from_numpy(w.extra["target"]).cuda()) ** 2).mean()
    loss.backward()
    gpu = np.concatenate([gx.grad.cpu().numpy().ravel(), gy.grad.cpu().numpy().ravel()])
    a = w.gx.astype(np.float64)
    b = w.gy.astype(np.float64)
    n = a.size

    def f(ax, ay):
        return np.sum((O.solve_fft(ax, ay, 64, 64) - t) ** 2) / n

    h = 1e-6
    fd = np.empty_like(gpu)
    flat = [a, b]
    k = 0
    for arr in flat:
        it = np.nditer(arr, flags=["multi_index"])
        for _ in it:
            idx = it.multi_index
            p = arr.copy()
            m = arr.copy()
            p[idx] += h
            m[idx] -= h
            if arr is a:
                fd[k] = (f(p, b) - f(m, b)) / (2 * h)
            else:
                fd[k] = (f(a, p) - f(a, m)) / (2 * h)
            k += 1
    assert rel_l2(gpu, fd) <= TOL


def test_adjoint_identity_on_gpu():
    H, W, M, N = 129, 200, 260, 400
    gx, gy = _rand_fields(8, 2, H, W)
    rng = np.random.default_rng(9)
    du = rng.normal(size=(2, H, W)).astype(np.float32)
    u = _gpu_solve(gx, gy, M, N).astype(np.float64)
    dgx, dgy = _gpu_backward(du, M, N)
    lhs = np.sum(u * du)
    rhs = np.sum(gx.astype(np.float64) * dgx) + np.sum(gy.astype(np.float64) * dgy)
    assert abs(lhs - rhs) <= 1e-5 * (abs(lhs) + abs(rhs))


def test_solves_capture_into_a_graph_and_replay():
    """Forward and backward solves enqueue kernels and events only, so they can be captured
    into a HIP graph (the forward column pass forks its low tiles to the plan's side stream
    and joins back). Each replay, with eager work and new inputs between replays, equals the
    eager solve of the same inputs bit for bit."""
    H, W, M, N, B = 129, 200, 260, 400, 3
    _say("graph capture of forward and backward solves")
    plan = gfc.Plan(H, W, M, N, tuned=False).build()
    gx, gy = _rand_fields(91, B, H, W)
    tx = torch.from_numpy(gx).cuda()
    ty = torch.from_numpy(gy).cuda()
    u = torch.empty_like(tx)
    ws = torch.empty(plan.workspace_size(B), dtype=torch.uint8, device="cuda")
    ws_e = torch.empty_like(ws)
    cap = torch.cuda.Stream()
    cap.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(cap):
        plan.solve(tx, ty, out=u, workspace=ws)  # warm-up outside the capture
    torch.cuda.current_stream().wait_stream(cap)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        plan.solve(tx, ty, out=u, workspace=ws)
        dgx, dgy = plan.backward(u, workspace=ws)
    torch.cuda.synchronize()
    rng = np.random.default_rng(5)
    for rep in range(3):
        scale = float(rng.uniform(0.5, 2.0))
        tx.copy_(torch.from_numpy(gx * scale))
        ty.copy_(torch.from_numpy(gy[::-1].copy()))
        g.replay()
        torch.cuda.synchronize()
        ue = plan.solve(tx, ty, workspace=ws_e)
        ex, ey = plan.backward(ue, workspace=ws_e)
        torch.cuda.synchronize()
        assert torch.equal(u, ue), rep
        assert torch.equal(dgx, ex) and torch.equal(dgy, ey), rep


def test_one_plan_from_several_host_threads():
    """Two host threads solve with one plan on their own streams and workspaces, many calls
    each; every result equals the single-threaded solve of the same input bit for bit."""
    import threading
    H, W, M, N, B = 129, 200, 260, 400, 2
    _say("one plan, two host threads")
    plan = gfc.Plan(H, W, M, N, tuned=False).build()
    gx, gy = _rand_fields(97, 2 * B, H, W)
    tx = torch.from_numpy(gx).cuda()
    ty = torch.from_numpy(gy).cuda()
    ref = plan.solve(tx, ty)
    torch.cuda.synchronize()
    errors = []

    def worker(k):
        try:
            st = torch.cuda.Stream()
            ws = torch.empty(plan.workspace_size(B), dtype=torch.uint8, device="cuda")
            out = torch.empty((B, H, W), dtype=torch.float32, device="cuda")
            sl = slice(k * B, (k + 1) * B)
            with torch.cuda.stream(st):
                for _ in range(50):
                    plan.solve(tx[sl], ty[sl], out=out, workspace=ws)
            st.synchronize()
            if not torch.equal(out, ref[sl]):
                errors.append(k)
        except Exception as e:  # noqa: BLE001
            errors.append(repr(e))

    ts = [threading.Thread(target=worker, args=(k,)) for k in range(2)]
    for t in ts:
        t.start()
    for t in ts:
        t.join()
    assert not errors, errors


def test_bad_outputs_and_workspaces_raise_before_any_launch():
    """A caller's `out` or workspace on the wrong device, too small, of the wrong shape or
    aliasing an input is refused by the binding (no pointer reaches a kernel)."""
    p = gfc.Plan(20, 30, tuned=False)
    gx = torch.zeros(2, 20, 30, device="cuda")
    gy = torch.zeros(2, 20, 30, device="cuda")
    need = p.workspace_size(2)
    with pytest.raises(ValueError):
        p.solve(gx, gy, out=torch.empty(2, 20, 30))  # host memory
    with pytest.raises(ValueError):
        p.solve(gx, gy, out=torch.empty(1, 20, 30, device="cuda"))
    with pytest.raises(ValueError):
        p.solve(gx, gy, out=gx)
    with pytest.raises(ValueError):
        p.solve(gx, gy, workspace=torch.empty(need - 1, dtype=torch.uint8, device="cuda"))
    with pytest.raises(ValueError):
        p.solve(gx, gy, workspace=torch.empty(need, dtype=torch.uint8))
    # a float32 workspace of enough bytes is accepted (bytes, not elements, are counted)
    ws = torch.empty((need + 3) // 4, dtype=torch.float32, device="cuda")
    u = p.solve(gx + 1e-3, gy, workspace=ws)
    torch.cuda.synchronize()
    assert bool(torch.isfinite(u).all())
