"""GPU parity of ragged batches (gfc_ragged_*): images of different sizes solved in one
graph replay. The result must equal, bit for bit, solving each image alone with its plan
(the only correct result, since each image's solve is unique), and match the float64
oracle per image at relative L2 <= 1e-5."""
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


def _fields(sizes, seed):
    out = []
    for (H, W), rng in zip(sizes, synth.image_rngs(seed, len(sizes))):
        a, b = synth.forward_gradient(synth.gaussian_sum_field(rng, H, W))
        a += rng.normal(0.0, 0.01, a.shape)  # not conservative: every term matters
        out.append((a.astype(np.float32), b.astype(np.float32)))
    return out


# mixed sizes: tiny, odd, one image taller than its torus allows for widened segments (tail),
# repeated sizes (shared plan), low and high row lengths
# and thin, wide images whose plans split more row bins (K = 32 and 16)
MIXED = [(64, 64, 0, 0), (37, 45, 0, 0), (1, 37, 3, 80), (33, 70, 35, 72), (64, 64, 0, 0),
         (129, 200, 260, 400), (5, 3, 16, 16), (255, 300, 513, 640), (100, 37, 210, 80),
         (3, 1250, 8, 2400), (2, 300, 0, 0)]


def _run_mixed(flags=0):
    r = gfc.Ragged(MIXED, flags=flags)
    pairs = _fields([(s[0], s[1]) for s in MIXED], seed=404)
    dev = torch.device("cuda:0")
    gx = r.pack([p[0] for p in pairs], dev)
    gy = r.pack([p[1] for p in pairs], dev)
    return r, pairs, gx, gy


def test_ragged_mixed_equals_sequential_and_oracle():
    _say("ragged mixed sizes: graph vs sequential vs oracle")
    r, pairs, gx, gy = _run_mixed()
    u = r.solve(gx, gy)
    us = r.solve_sequential(gx, gy)
    torch.cuda.synchronize()
    assert torch.equal(u, us), "ragged solve differs from the per-image plain solves"
    for k, ((a, b), ui) in enumerate(zip(pairs, r.unpack(u))):
        H, W, M, N = r.sizes[k]
        ref = O.solve_fft(a, b, M, N)
        e = rel_l2(ui.cpu().numpy(), ref)
        _say(f"  image {k} {H}x{W} on {M}x{N}: rel L2 {e:.2e}")
        assert e <= TOL, (k, e)


def test_ragged_no_graph_flag_matches_graph():
    _say("ragged: direct launches vs graph replay")
    r, _, gx, gy = _run_mixed()
    rn, _, _, _ = _run_mixed(flags=gfc.RAGGED_NO_GRAPH)
    u = r.solve(gx, gy)
    un = rn.solve(gx, gy)
    torch.cuda.synchronize()
    assert torch.equal(u, un)


def test_ragged_graph_replays_and_recaptures():
    _say("ragged: graph replays with eager work between, then new buffers")
    r, _, gx, gy = _run_mixed()
    out = torch.empty_like(gx)
    ref = r.solve_sequential(gx, gy)
    torch.cuda.synchronize()
    for rep in range(3):
        out.fill_(float("nan"))
        junk = torch.randn(1 << 20, device=gx.device).sum()  # unrelated eager work
        r.solve(gx, gy, out=out)
        torch.cuda.synchronize()
        assert torch.isfinite(junk)
        assert torch.equal(out, ref), f"replay {rep}"
    out2 = torch.empty_like(gx)  # new address: the graph is captured again
    r.solve(gx, gy, out=out2)
    torch.cuda.synchronize()
    assert torch.equal(out2, ref)


def test_ragged_alternating_outputs_replay_cached_graphs():
    """Outputs at alternating addresses (a caller that keeps the previous result): each call
    replays or captures a graph without waiting on the GPU, and every result is exact."""
    _say("ragged: alternating output buffers")
    r, _, gx, gy = _run_mixed()
    ref = r.solve_sequential(gx, gy)
    torch.cuda.synchronize()
    outs = [torch.empty_like(gx) for _ in range(6)]
    for rep in range(3):
        for o in outs:  # six address sets: more than the graphs kept, so some are evicted
            o.fill_(float("nan"))
            r.solve(gx, gy, out=o)
    torch.cuda.synchronize()
    for k, o in enumerate(outs):
        assert torch.equal(o, ref), k


def test_ragged_empty_batch():
    r = gfc.Ragged([])
    dev = torch.device("cuda:0")
    e = torch.empty(0, device=dev)
    u = r.solve(e, e)
    torch.cuda.synchronize()
    assert u.numel() == 0


def test_ragged_uneven_batch_full_size():
    """The uneven-size workload: 200 images, H, W ~ U{64..1024}, default tori (128..2048),
    in the launch configuration the benchmark times (one graph replay). Every image is
    compared with the float64 oracle, and the whole batch with the per-image plain solves."""
    _say("ragged 200 images (64..1024): graph vs sequential and every image vs the oracle")
    sizes = synth.ragged_sizes()
    pairs = synth.make_ragged(sizes=sizes)
    r = gfc.Ragged(sizes)
    dev = torch.device("cuda:0")
    gx = r.pack([p[0] for p in pairs], dev)
    gy = r.pack([p[1] for p in pairs], dev)
    u = r.solve(gx, gy)
    us = r.solve_sequential(gx, gy)
    torch.cuda.synchronize()
    assert torch.equal(u, us)
    assert bool(torch.isfinite(u).all())
    ul = [t.cpu().numpy() for t in r.unpack(u)]
    worst = (0.0, -1)
    for k in range(len(sizes)):
        H, W, M, N = r.sizes[k]
        ref = O.solve_fft(pairs[k][0], pairs[k][1], M, N)
        e = rel_l2(ul[k], ref)
        worst = max(worst, (e, k))
        assert e <= TOL, (k, (H, W, M, N), e)
    _say(f"  worst image {worst[1]} {r.sizes[worst[1]]}: rel L2 {worst[0]:.2e}")


def test_ragged_solve_helper():
    pairs = _fields([(40, 50), (64, 31)], seed=405)
    tp = [(torch.from_numpy(a).cuda(), torch.from_numpy(b).cuda()) for a, b in pairs]
    us = gfc.ragged_solve(tp)
    torch.cuda.synchronize()
    for (a, b), u in zip(pairs, us):
        ref = O.solve_fft(a, b, *synth.default_grid(*a.shape))
        assert rel_l2(u.cpu().numpy(), ref) <= TOL
